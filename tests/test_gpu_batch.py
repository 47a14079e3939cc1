"""Batched reconstruction (several segments x references with uneven neighbour
sets, one persistent launch in a captured graph) against per-call results
and the FP64 oracle."""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mf as omf
from oracle import peaks as opk
from oracle import ratio as orat
from paper_2511_12894_amd import synth

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_12894_amd import rf as rfmod
    rfmod.load()
    return rfmod


@pytest.fixture(scope="module")
def work():
    """Two 64 s segments at 1024 Hz, three references with 16, 5 and 45 neighbours."""
    g = synth.make_grid(1024.0, 65536, 30.0)
    psd = synth.make_psd(g)
    refs = [(1.4, 1.4), (1.6, 1.2), (2.0, 1.5)]
    groups = [synth.neighbour_lattice(*r, g.f_low, c) for r, c in zip(refs, (16, 5, 45))]
    segs = []
    for s in range(2):
        xf = synth.noise(g, psd, seed=3000 + s)
        m1, m2 = groups[2 * s][3]
        xf = synth.inject(g, psd, xf, m1, m2, 11.0 + s, 20.0 + 15.0 * s, 0.3)
        segs.append(xf)
    return dict(grid=g, psd=psd, refs=refs, groups=groups, segs=np.stack(segs))


@pytest.fixture(scope="module")
def setup(rf, work):
    stream = torch.cuda.Stream()
    ctx = rf.Context(0, stream)
    g = work["grid"]
    psd = torch.from_numpy(work["psd"]).cuda()
    xf = torch.from_numpy(work["segs"]).cuda()
    _say("batch: building kernel sets")
    with torch.cuda.stream(stream):
        ksets = [rf.ratio_kernel_build(ctx, g, psd, r, grp) for r, grp in zip(work["refs"], work["groups"])]
        batch = rf.Batch(ctx, g, psd, work["refs"], ksets, nseg=2)
    yield dict(ctx=ctx, psd=psd, xf=xf, ksets=ksets, batch=batch, stream=stream)
    torch.cuda.synchronize()
    batch.free()
    for k in ksets:
        k.free()
    ctx.close()


def _per_call(rf, work, st, thr):
    """Per-(segment, reference) reference MF + fused split-FP16 reconstruction."""
    ctx, g = st["ctx"], work["grid"]
    kbase = st["batch"].info()["kbase"]
    peaks = np.zeros((2, st["batch"].ktotal, 2), dtype=np.float64)
    trig = set()
    with torch.cuda.stream(st["stream"]):
        for s in range(2):
            for r, K in enumerate(st["ksets"]):
                z, _ = rf.mf_ref_snr(ctx, g, st["xf"][s].contiguous(), st["psd"], [work["refs"][r]])
                out = rf.snr_reconstruct(ctx, K, z[0].contiguous(), prec="split16", store=False, fused_thr=thr)
                v, i = rf.decode_peaks(out["peaks"])
                peaks[s, kbase[r]:kbase[r] + K.nk, 0] = v
                peaks[s, kbase[r]:kbase[r] + K.nk, 1] = i
                for t in rf.decode_triggers(out["trig"], out["ntrig"]):
                    trig.add((s, kbase[r] + t[0], t[2], t[3]))
    torch.cuda.synchronize()
    return peaks, trig


def _decode(rf, out, nseg, ktot):
    p = out["peaks"].cpu().contiguous().view(nseg * ktot, 2)
    v, i = rf.decode_peaks(p)
    trig = set((t[1], t[0], t[2], t[3]) for t in rf.decode_triggers(out["trig"], out["ntrig"]))
    return np.stack([v.reshape(nseg, ktot), i.reshape(nseg, ktot)], axis=-1).astype(np.float64), trig


@pytest.mark.parametrize("chunk", [256, 512, 1024])
def test_batch_matches_per_call_exactly(rf, work, setup, chunk):
    """Any window chunk size gives the per-call path's sums (the same folds and
    the same steps with correction products): bit-identical peaks and triggers."""
    b = setup["batch"]
    b.set_chunks([chunk, chunk, chunk])
    _say(f"batch info {b.info()}")
    out = b.run(setup["xf"], 6.0)
    got_p, got_t = _decode(rf, out, 2, b.ktotal)
    ref_p, ref_t = _per_call(rf, work, setup, 6.0)
    np.testing.assert_array_equal(got_p, ref_p)
    assert got_t == ref_t and len(got_t) > 0


@pytest.mark.parametrize("blocks,xcd,bounds", [((2, 4, 1), 0, None), ((1, 1, 1), 1, None),
                                               ((4, 2, 2), 1, [0, 10 ** 9])])
def test_batch_launch_settings_keep_results(rf, work, setup, blocks, xcd, bounds):
    """Time blocks per work item, one queue or one per XCD, and the bucket
    bounds only move work between workgroups: peaks and triggers stay
    bit-identical to the per-call path's."""
    b = setup["batch"]
    b.set_tuning(chunk=[512, 512, 512], blocks=list(blocks), xcd_queues=xcd, bucket_hi=bounds)
    t = b.tuning()
    _say(f"batch tuning {t}, {b.info()['nitems']} work items")
    assert t["blocks"] == list(blocks) and t["xcd_queues"] == xcd
    out = b.run(setup["xf"], 6.0)
    got_p, got_t = _decode(rf, out, 2, b.ktotal)
    ref_p, ref_t = _per_call(rf, work, setup, 6.0)
    np.testing.assert_array_equal(got_p, ref_p)
    assert got_t == ref_t and len(got_t) > 0
    b.set_tuning(blocks=[1, 1, 1], xcd_queues=0)


def test_batch_tuning_rejects_bad_settings(rf, work, setup):
    b = setup["batch"]
    t0 = b.tuning()
    assert 0 <= t0["bucket_hi"][0] <= t0["bucket_hi"][1]
    for kw in (dict(chunk=[512, 300, 512]), dict(blocks=[1, 3, 1]), dict(xcd_queues=2),
               dict(bucket_hi=[5, 4]), dict(bucket_hi=[-1, 4])):
        with pytest.raises(rf.RfError):
            b.set_tuning(**kw)
    assert b.tuning() == t0


def test_batch_graph_replay_and_recapture(rf, work, setup):
    """New output and input buffers replay the captured graph (it holds only
    the batch's own buffers); a new threshold re-captures it."""
    b = setup["batch"]
    a = _decode(rf, b.run(setup["xf"], 6.0), 2, b.ktotal)
    cap0, rep0 = b.graph_stats()
    xf2 = setup["xf"].clone()                                      # another input pointer
    outs = [b.run(xf2 if i % 2 else setup["xf"], 6.0) for i in range(3)]   # fresh outputs each time
    cap1, rep1 = b.graph_stats()
    assert cap1 == cap0 and rep1 == rep0 + 3
    for o in outs:
        c = _decode(rf, o, 2, b.ktotal)
        np.testing.assert_array_equal(a[0], c[0])
        assert a[1] == c[1]
    d = _decode(rf, b.run(setup["xf"], 7.5), 2, b.ktotal)       # new threshold: re-capture
    assert b.graph_stats()[0] == cap1 + 1
    np.testing.assert_array_equal(a[0], d[0])
    assert d[1] == set(t for t in a[1] if t[3] > 7.5)


def test_batch_overflow_reports_true_count(rf, work, setup):
    b = setup["batch"]
    full = b.run(setup["xf"], 6.0)
    small = b.run(setup["xf"], 6.0, trig_cap=3)
    assert small["overflow"] and small["ntrig"] == full["ntrig"] > 3


def test_batch_autotune_and_cache(rf, work, setup, tmp_path):
    b = setup["batch"]
    path = str(tmp_path / "tune.txt")
    chunks = b.autotune(setup["xf"], path)
    tuned = b.tuning()
    _say(f"autotuned {tuned}")
    assert all(c in (256, 512, 1024) for c in chunks) and tuned["chunk"] == chunks
    assert all(x in (1, 2, 4) for x in tuned["blocks"]) and tuned["xcd_queues"] in (0, 1)
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and len(lines[0].split()) == 10
    b.set_tuning(chunk=[256, 256, 256], blocks=[1, 1, 1], xcd_queues=1 - tuned["xcd_queues"])
    assert b.autotune(setup["xf"], path) == chunks          # from the cache
    assert b.tuning() == tuned
    assert open(path).read().count("\n") == 1
    out = b.run(setup["xf"], 6.0)
    got_p, _ = _decode(rf, out, 2, b.ktotal)
    ref_p, _ = _per_call(rf, work, setup, 6.0)
    # another chunk size only reorders roundings
    np.testing.assert_allclose(got_p[..., 0], ref_p[..., 0], rtol=1e-6)


def test_batch_peaks_match_oracle(rf, work, setup):
    b = setup["batch"]
    b.set_chunks([512, 512, 512])
    got_p, _ = _decode(rf, b.run(setup["xf"], 6.0), 2, b.ktotal)
    g = work["grid"]
    kbase = b.info()["kbase"]
    for s in range(2):
        xf = work["segs"][s]
        for r, ref in enumerate(work["refs"]):
            zr, nr = omf.grid_snr_series(g, xf, work["psd"], *ref)
            for k in (0, len(work["groups"][r]) - 1):
                nb = work["groups"][r][k]
                kb = orat.build_kernel(g, ref, nb)
                nk = omf.norm(g.fs, g.n, g.f_low, g.f_high, work["psd"], omf.template_spectrum(g.fs, g.n, *nb))
                zo = orat.reconstruct(zr, kb["m_lo"], kb["taps"], nr / nk)
                pv, pi = opk.peak(zo)
                assert abs(got_p[s, kbase[r] + k, 0] - pv) <= 1e-5
