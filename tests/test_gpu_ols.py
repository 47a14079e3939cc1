"""Blocked frequency-domain (overlap-save) reconstruction against the FP64 oracle
with the same truncated kernels, against direct matched filtering, and its
fused read-out against the stored series."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mf as omf
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
def ctx(rf):
    c = rf.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _setup(rf, ctx, w, nbrs):
    g = w["grid"]
    zr, nr = omf.grid_snr_series(g, w["xf"], w["psd"], *w["ref"])
    ks = [orat.build_kernel(g, w["ref"], nb) for nb in nbrs]
    norms = [omf.norm(g.fs, g.n, g.f_low, g.f_high, w["psd"], omf.template_spectrum(g.fs, g.n, *nb)) for nb in nbrs]
    xf = torch.from_numpy(w["xf"]).cuda()
    psd = torch.from_numpy(w["psd"]).cuda()
    K = rf.ratio_kernel_build(ctx, g, psd, w["ref"], nbrs)
    z, _ = rf.mf_ref_snr(ctx, g, xf, psd, [w["ref"]])
    return dict(w=w, zr=zr, nr=nr, ks=ks, norms=norms, xf=xf, psd=psd, K=K, z=z[0].contiguous())


@pytest.fixture(scope="module")
def small(rf, ctx):
    w = synth.workload_small()
    _say("ols small: oracle")
    d = _setup(rf, ctx, w, w["nbrs"])
    yield d
    d["K"].free()


def test_small_every_sample_against_the_oracle(rf, ctx, small):
    """64 s at 1024 Hz (16 blocks of 4096 outputs), 16 kernels: every sample of
    every series against the oracle's circular correlation with the same taps."""
    g = small["w"]["grid"]
    O = rf.Ols(ctx, small["K"], g.n)
    info = O.info()
    assert info["block"] == 8192 and info["hop"] == 4096
    assert all(p >= 1 for p in info["parts"])
    z = O.reconstruct(small["z"])["z"].cpu().numpy()
    err = 0.0
    for k, kb in enumerate(small["ks"]):
        zo = orat.reconstruct(small["zr"], kb["m_lo"], kb["taps"], small["nr"] / small["norms"][k])
        err = max(err, np.abs(z[k] - zo).max())
    _say(f"ols small vs oracle (every sample): max|dz| = {err:.3e}, partitions {info['parts']}")
    assert err <= 1e-5
    # and the dense reconstruction of the same kernels
    zd = rf.snr_reconstruct(ctx, small["K"], small["z"], prec="fp32")["z"].cpu().numpy()
    assert np.abs(z - zd).max() <= 1e-5
    O.free()


def test_partition_counts(rf, ctx, small):
    """P_k = ceil((d_k - o_k + L_k) / 4096) with o_k the 2048-grid point at or
    below the kernel's offset d_k from the set's first tap."""
    info = small["K"].info()
    O = rf.Ols(ctx, small["K"], small["w"]["grid"].n)
    m0 = min(info["m_lo"])
    exp = []
    for lo, ln in zip(info["m_lo"], info["len"]):
        d = lo - m0
        o = (d // 2048) * 2048
        exp.append(-(-(d - o + ln) // 4096))
    oi = O.info()
    assert oi["parts"] == exp and oi["pmax"] == max(exp)
    assert oi["spectra_bytes"] == sum(exp) * 8192 * 8
    O.free()


@pytest.fixture(scope="module")
def real64(rf, ctx):
    """Realistic structure at 64 s: 4096 Hz, f_low 20 Hz, ref 1.6+1.2, 64 lattice
    neighbours (kernels of ~12k taps: four partitions, spectra in registers),
    four injections."""
    w = synth.workload_realistic(n_nbr=64, duration=64.0)
    _say("ols realistic-64s: oracle kernels")
    d = _setup(rf, ctx, w, w["nbrs"])
    yield d
    d["K"].free()


def test_realistic_against_oracle_and_direct_mf(rf, ctx, real64):
    w = real64["w"]
    g = w["grid"]
    O = rf.Ols(ctx, real64["K"], g.n)
    info = O.info()
    assert info["pmax"] <= 4
    out = O.reconstruct(real64["z"], fused_thr=6.0, trig_cap=1 << 14)
    z = out["z"]
    zh = z.cpu().numpy()
    err = 0.0
    for k, kb in enumerate(real64["ks"]):
        zo = orat.reconstruct(real64["zr"], kb["m_lo"], kb["taps"], real64["nr"] / real64["norms"][k])
        err = max(err, np.abs(zh[k] - zo).max())
    _say(f"ols realistic-64s vs oracle (every sample of every series): {err:.3e}")
    assert err <= 1e-5
    zd, _ = rf.mf_ref_snr(ctx, g, real64["xf"], real64["psd"], w["nbrs"])
    ed = (z - zd).abs().max().item()
    _say(f"ols realistic-64s vs direct MF: {ed:.3e}")
    assert ed <= 2e-4
    ref = rf.snr_peaks(ctx, z, 6.0, trig_cap=1 << 14)
    torch.cuda.synchronize()
    assert torch.equal(out["peaks"], ref["peaks"])
    got = set(rf.decode_triggers(out["trig"], out["ntrig"]))
    exp = set(rf.decode_triggers(ref["trig"], ref["ntrig"]))
    assert got == exp and out["ntrig"] > 0
    # fused read-out alone
    fo = O.reconstruct(real64["z"], store=False, fused_thr=6.0, trig_cap=1 << 14)
    assert torch.equal(fo["peaks"], ref["peaks"])
    assert set(rf.decode_triggers(fo["trig"], fo["ntrig"])) == exp
    O.free()


def test_trigger_overflow_keeps_the_count(rf, ctx, real64):
    g = real64["w"]["grid"]
    O = rf.Ols(ctx, real64["K"], g.n)
    full = O.reconstruct(real64["z"], store=False, fused_thr=4.0, trig_cap=1 << 16)
    assert full["ntrig"] > 8 and not full["overflow"]
    cut = O.reconstruct(real64["z"], store=False, fused_thr=4.0, trig_cap=8)
    assert cut["overflow"] and cut["ntrig"] == full["ntrig"]
    assert torch.equal(cut["peaks"], full["peaks"])
    O.free()


def test_empty_and_delta_kernels(rf, ctx, small):
    """A threshold no kernel reaches leaves them all empty (zero series, peak 0
    at sample 0); at 500 / s the reference itself keeps the central taps of
    its band-limited delta while farther neighbours may keep none: every
    series against the oracle with the same truncation."""
    w = small["w"]
    g = w["grid"]
    psd = small["psd"]
    K0 = rf.ratio_kernel_build(ctx, g, psd, w["ref"], w["nbrs"][:3], thr=1e9)
    assert K0.info()["len"] == [0, 0, 0]
    O = rf.Ols(ctx, K0, g.n)
    out = O.reconstruct(small["z"], fused_thr=1.0)
    assert torch.count_nonzero(out["z"]).item() == 0
    v, i = rf.decode_peaks(out["peaks"])
    assert list(v) == [0.0, 0.0, 0.0] and list(i) == [0, 0, 0] and out["ntrig"] == 0
    O.free()
    K0.free()
    nbrs = [w["nbrs"][0], w["ref"], w["nbrs"][5]]
    K = rf.ratio_kernel_build(ctx, g, psd, w["ref"], nbrs, thr=500.0)
    lens = K.info()["len"]
    assert lens[1] >= 1
    O = rf.Ols(ctx, K, g.n)
    z = O.reconstruct(small["z"])["z"].cpu().numpy()
    for k, nb in enumerate(nbrs):
        kb = orat.build_kernel(g, w["ref"], nb, threshold=500.0)
        nk = omf.norm(g.fs, g.n, g.f_low, g.f_high, w["psd"], omf.template_spectrum(g.fs, g.n, *nb))
        zo = orat.reconstruct(small["zr"], kb["m_lo"], kb["taps"], small["nr"] / nk)
        assert np.abs(z[k] - zo).max() <= 1e-5, (k, lens)
    O.free()
    K.free()


def test_kernels_built_on_a_shorter_period(rf, ctx, small):
    """Kernels built with n_build = n / 4 applied to the full segment: the same
    series as the dense reconstruction of that kernel set."""
    w = small["w"]
    g = w["grid"]
    K = rf.ratio_kernel_build(ctx, g, small["psd"], w["ref"], w["nbrs"][:6], n_build=g.n // 4)
    O = rf.Ols(ctx, K, g.n)
    z = O.reconstruct(small["z"])["z"]
    zd = rf.snr_reconstruct(ctx, K, small["z"], prec="fp32")["z"]
    assert (z - zd).abs().max().item() <= 1e-5
    O.free()
    K.free()


def test_argument_errors(rf, ctx, small):
    g = small["w"]["grid"]
    h = __import__("ctypes").c_void_p()
    for bad in (g.n + 1, 2048, 1 << 25, g.n // 2):        # the last: shorter than the kernels' build
        st = ctx.lib.rf_ols_build(ctx.h, small["K"].h, bad, __import__("ctypes").byref(h))
        assert st == rf.RF_E_INVAL, bad
    O = rf.Ols(ctx, small["K"], g.n)
    short = torch.zeros(g.n // 2, dtype=torch.complex64, device="cuda")
    with pytest.raises(rf.RfError) as e:
        O.reconstruct(short)
    assert e.value.code == rf.RF_E_INVAL
    st = ctx.lib.snr_reconstruct_ols(ctx.h, O.h, small["z"].data_ptr(), g.n, None, None)
    assert st == rf.RF_E_INVAL
    O.free()
