"""Parity at the full sizes of the two large workloads, in the launch
configurations the library runs them in:

* batched uneven: 8 segments of 256 s at 4096 Hz, 64 references with 32-512
  lattice neighbours each, one persistent split-FP16 launch with the fused
  read-out; sampled peaks against the FP64 oracle and every injection found;
* next-generation-detector shape: 4 references x 1024 neighbours on 2^23
  samples at f_low = 10 Hz, split-FP16 reconstruction with the fused read-out;
  the peak of every one of the 4096 series against direct matched filtering
  of the same template, and sampled peaks against the oracle.
"""
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


def _oracle_peak(g, xf, psd, ref, nb):
    zr, nr = omf.grid_snr_series(g, xf, psd, *ref)
    kb = orat.build_kernel(g, ref, nb)
    nk = omf.norm(g.fs, g.n, g.f_low, g.f_high, psd, omf.template_spectrum(g.fs, g.n, *nb))
    return opk.peak(orat.reconstruct(zr, kb["m_lo"], kb["taps"], nr / nk))


def test_batched_full_shape(rf):
    w = synth.workload_batched()
    g = w["grid"]
    nseg = len(w["segments"])
    stream = torch.cuda.Stream()
    ctx = rf.Context(0, stream)
    psd = torch.from_numpy(w["psd"]).cuda()
    xf = torch.from_numpy(np.stack(w["segments"])).cuda()
    _say(f"batched full: {nseg} segments, {len(w['refs'])} references, "
         f"{sum(len(x) for x in w['groups'])} kernels; building")
    with torch.cuda.stream(stream):
        ksets = [rf.ratio_kernel_build(ctx, g, psd, r, grp) for r, grp in zip(w["refs"], w["groups"])]
        lens = np.concatenate([k.info()["len"] for k in ksets])
        batch = rf.Batch(ctx, g, psd, w["refs"], ksets, nseg=nseg)
        _say(f"batched full: kernel taps {lens.min()}..{lens.max()}, running")
        out = batch.run(xf, 6.0, trig_cap=1 << 20)
    torch.cuda.synchronize()
    assert not out["overflow"]
    ktot = batch.ktotal
    kbase = batch.info()["kbase"]
    v, i = rf.decode_peaks(out["peaks"].cpu().contiguous().view(nseg * ktot, 2))
    v, i = v.reshape(nseg, ktot), i.reshape(nseg, ktot)
    # sampled (segment, reference, neighbour) against the oracle
    rng = np.random.default_rng(11)
    for _ in range(4):
        s = int(rng.integers(nseg))
        r = int(rng.integers(len(w["refs"])))
        k = int(rng.integers(len(w["groups"][r])))
        pv, pi = _oracle_peak(g, w["segments"][s], w["psd"], w["refs"][r], w["groups"][r][k])
        _say(f"seg {s} ref {r} nbr {k}: GPU {v[s, kbase[r] + k]:.6f} @ {i[s, kbase[r] + k]}, oracle {pv:.6f} @ {pi}")
        assert abs(v[s, kbase[r] + k] - pv) <= 1e-5
    # every injection: its template's peak at the injection time
    for s, m1, m2, snr, t0, _phi in w["injections"]:
        hits = [(r, k) for r, grp in enumerate(w["groups"]) for k, nb in enumerate(grp) if nb == (m1, m2)]
        r, k = hits[0]
        _say(f"injection seg {s}: SNR {snr} at {t0:.1f} s -> peak {v[s, kbase[r] + k]:.3f} "
             f"at {i[s, kbase[r] + k] / g.fs:.3f} s")
        assert v[s, kbase[r] + k] > 0.7 * snr
        assert abs(i[s, kbase[r] + k] / g.fs - t0) < 0.05
    batch.free()
    for K in ksets:
        K.free()
    torch.cuda.synchronize()
    ctx.close()


def test_stress_full_shape(rf):
    w = synth.workload_stress()
    g = w["grid"]
    ctx = rf.Context(0)
    psd = torch.from_numpy(w["psd"]).cuda()
    xf = torch.from_numpy(w["xf"]).cuda()
    worst = 0.0
    rng = np.random.default_rng(12)
    for r, (ref, nbrs) in enumerate(zip(w["refs"], w["groups"])):
        _say(f"stress full: reference {r} ({ref}), {len(nbrs)} neighbours")
        K = rf.ratio_kernel_build(ctx, g, psd, ref, nbrs)
        z, _ = rf.mf_ref_snr(ctx, g, xf, psd, [ref], want_sigma=False)
        out = rf.snr_reconstruct(ctx, K, z[0].contiguous(), prec="split16", store=False, fused_thr=6.0,
                                 trig_cap=1 << 18)
        vr, ir = rf.decode_peaks(out["peaks"])
        del z
        # direct matched filtering of every neighbour, 128 at a time
        vd = np.zeros(len(nbrs))
        for a in range(0, len(nbrs), 128):
            zd, _ = rf.mf_ref_snr(ctx, g, xf, psd, nbrs[a:a + 128], want_sigma=False)
            pk = rf.snr_peaks(ctx, zd, 1e9)
            vd[a:a + 128] = rf.decode_peaks(pk["peaks"])[0]
            del zd, pk
        err = np.abs(vr - vd).max()
        worst = max(worst, err)
        _say(f"  {len(nbrs)} peaks vs direct MF: max |dpeak| = {err:.3e}; taps "
             f"{min(K.info()['len'])}..{max(K.info()['len'])}")
        assert err <= 2e-4
        k = int(rng.integers(len(nbrs)))
        pv, pi = _oracle_peak(g, w["xf"], w["psd"], ref, nbrs[k])
        _say(f"  neighbour {k}: GPU {vr[k]:.6f}, oracle {pv:.6f}")
        assert abs(vr[k] - pv) <= 1e-5
        K.free()
        torch.cuda.synchronize()
    _say(f"stress full: worst peak difference against direct MF over 4096 templates {worst:.3e}")
    ctx.close()
