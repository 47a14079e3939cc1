"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (max |dz| in SNR units, sigma = 1 per quadrature):
  * 1e-5 against the oracle with the same truncated kernels, for both the
    FP32 and the split-FP16 reconstruction, and for the FP32 FFT matched filter;
  * 2e-4 against direct matched filtering of every neighbour (the truncation
    error of the paper's threshold, plus arithmetic).
Integer results (supports, argmax, trigger sets) are compared exactly, with
decisions re-taken in FP32 on the oracle side where FP32 decides them.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mf as omf
from oracle import peaks as opk
from oracle import ratio as orat
from paper_2511_12894_amd import synth

pytestmark = pytest.mark.gpu

TOL_SAME_KERNELS = 1e-5
TOL_DIRECT = 2e-4


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


def _dev(x, dtype):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dtype).cuda()


@pytest.fixture(scope="module")
def small():
    w = synth.workload_small()
    g = w["grid"]
    zr, nr = omf.grid_snr_series(g, w["xf"], w["psd"], *w["ref"])
    kern = [orat.build_kernel(g, w["ref"], nb) for nb in w["nbrs"]]
    direct = [omf.grid_snr_series(g, w["xf"], w["psd"], *nb) for nb in w["nbrs"]]
    return dict(w=w, zr=zr, nr=nr, kern=kern, direct=direct)


@pytest.fixture(scope="module")
def small_gpu(rf, ctx, small):
    w = small["w"]
    xf = _dev(w["xf"], torch.complex128)
    psd = _dev(w["psd"], torch.float64)
    _say("small: mf_ref_snr")
    z, sig = rf.mf_ref_snr(ctx, w["grid"], xf, psd, [w["ref"]])
    _say("small: ratio_kernel_build")
    K = rf.ratio_kernel_build(ctx, w["grid"], psd, w["ref"], w["nbrs"])
    torch.cuda.synchronize()
    return dict(xf=xf, psd=psd, zref=z[0].contiguous(), sig=sig, K=K)


# ------------------------------------------------------------ matched filter

def test_mf_ref_snr_matches_oracle(rf, ctx, small, small_gpu):
    w = small["w"]
    z = small_gpu["zref"].cpu().numpy().astype(np.complex128)
    err = np.abs(z - small["zr"]).max()
    _say(f"mf_ref_snr small: max|dz| = {err:.3e}")
    assert err <= TOL_SAME_KERNELS
    assert small_gpu["sig"][0] == pytest.approx(small["nr"], rel=1e-12)


def test_mf_ref_snr_many_templates_and_tiny_grid(rf, ctx):
    """nt = 3 templates on the smallest grid (n = 2^8 ... 2^11) vs the brute-force DFT, and
    the transform's own read-out against the read-out of the stored series."""
    for n, fs in ((256, 256.0), (2048, 256.0)):
        g = synth.make_grid(fs, n, 20.0)
        psd = synth.make_psd(g)
        xf = synth.noise(g, psd, seed=17 + n)
        tm = [(3.0, 2.5), (2.0, 1.5), (1.2, 1.1)]
        _say(f"tiny mf n={n}")
        xf_d, psd_d = _dev(xf, torch.complex128), _dev(psd, torch.float64)
        z, sig = rf.mf_ref_snr(ctx, g, xf_d, psd_d, tm)
        # the read-out in the last transform pass (two 16-point passes at n = 256,
        # a 16- and a 128-point pass at n = 2048)
        # equals the read-out of the stored series, with a threshold some samples cross
        thr = float(0.5 * z.abs().max().item())
        a = rf.mf_snr_peaks(ctx, g, xf_d, psd_d, tm, thr)
        b = rf.snr_peaks(ctx, z, thr)
        v1, i1 = rf.decode_peaks(a["peaks"])
        v2, i2 = rf.decode_peaks(b["peaks"])
        np.testing.assert_array_equal(i1, i2)
        np.testing.assert_array_equal(v1, v2)
        assert a["ntrig"] == b["ntrig"] > 0
        assert sorted(rf.decode_triggers(a["trig"], a["ntrig"])) == sorted(rf.decode_triggers(b["trig"], b["ntrig"]))
        z = z.cpu().numpy()
        for i, t in enumerate(tm):
            zo, no = omf.snr_series_bruteforce(g.fs, g.n, g.f_low, g.f_high, xf, psd, *t)
            assert np.abs(z[i] - zo).max() <= TOL_SAME_KERNELS
            assert sig[i] == pytest.approx(no, rel=1e-12)


def test_two_pass_matched_filter_sizes(rf, ctx):
    """The two-pass form (n = 2^20: 1024 x 1024 points; 2^21: 2048 x 1024; 2^22:
    2048 x 2048; 2^23: 4096 x 2048) on a few templates: every sample of the
    stored series within 1e-5 of the FP64 oracle, and the read-out inside the
    second pass equal to the read-out of the stored series, bit for bit,
    crossings included."""
    for n, fs, fl in ((1 << 20, 4096.0, 20.0), (1 << 21, 4096.0, 20.0), (1 << 22, 4096.0, 20.0),
                      (1 << 23, 4096.0, 10.0)):
        g = synth.make_grid(fs, n, fl)
        psd = synth.make_psd(g)
        xf = synth.noise(g, psd, seed=31 + n)
        tm = [(1.4, 1.3), (2.6, 1.9), (1.1, 1.0)]
        _say(f"two-pass mf n={n}")
        xf_d, psd_d = _dev(xf, torch.complex128), _dev(psd, torch.float64)
        z, sig = rf.mf_ref_snr(ctx, g, xf_d, psd_d, tm)
        thr = float(0.6 * z.abs().max().item())
        a = rf.mf_snr_peaks(ctx, g, xf_d, psd_d, tm, thr, trig_cap=1 << 18)
        b = rf.snr_peaks(ctx, z, thr, trig_cap=1 << 18)
        assert not a["overflow"] and not b["overflow"]
        _same_readout(rf, a, b)
        zc = z.cpu().numpy()
        for i, t in enumerate(tm):
            zo, no = omf.grid_snr_series(g, xf, psd, *t)
            assert np.abs(zc[i] - zo).max() <= TOL_SAME_KERNELS
            assert sig[i] == pytest.approx(no, rel=1e-12)


def test_direct_mf_of_neighbours(rf, ctx, small, small_gpu):
    w = small["w"]
    z, _ = rf.mf_ref_snr(ctx, w["grid"], small_gpu["xf"], small_gpu["psd"], w["nbrs"])
    z = z.cpu().numpy()
    err = max(np.abs(z[i] - small["direct"][i][0]).max() for i in range(len(w["nbrs"])))
    _say(f"direct mf small: max|dz| = {err:.3e}")
    assert err <= TOL_SAME_KERNELS


# ------------------------------------------------------------ kernel build

def _same_readout(rf, a, b):
    v1, i1 = rf.decode_peaks(a["peaks"])
    v2, i2 = rf.decode_peaks(b["peaks"])
    np.testing.assert_array_equal(i1, i2)
    np.testing.assert_array_equal(v1, v2)
    assert a["ntrig"] == b["ntrig"] > 0
    assert sorted(rf.decode_triggers(a["trig"], a["ntrig"])) == sorted(rf.decode_triggers(b["trig"], b["ntrig"]))


def test_direct_mf_readout_equals_stored_series(rf, ctx, small, small_gpu):
    """mf_snr_peaks reads the series out in its last transform pass: peaks and
    trigger set equal snr_peaks on the series mf_ref_snr stores, exactly."""
    w = small["w"]
    tm = [w["ref"]] + list(w["nbrs"])
    z, _ = rf.mf_ref_snr(ctx, w["grid"], small_gpu["xf"], small_gpu["psd"], tm, want_sigma=False)
    ref = rf.snr_peaks(ctx, z, 6.0, trig_cap=1 << 16)
    out = rf.mf_snr_peaks(ctx, w["grid"], small_gpu["xf"], small_gpu["psd"], tm, 6.0, trig_cap=1 << 16)
    _say(f"direct read-out: {out['ntrig']} triggers over {len(tm)} templates")
    _same_readout(rf, out, ref)
    g = rf.to_grid(w["grid"])
    assert ctx.lib.mf_snr_peaks(ctx.h, rf.ctypes.byref(g), rf._ptr(small_gpu["xf"]), rf._ptr(small_gpu["psd"]),
                                rf._tmpl_array(tm), len(tm), None) == rf.RF_E_INVAL


def test_kernel_build_matches_oracle(rf, ctx, small, small_gpu):
    K = small_gpu["K"]
    info = K.info()
    for k, kb in enumerate(small["kern"]):
        assert info["m_lo"][k] == kb["m_lo"]
        assert info["len"][k] == kb["taps"].size
        assert info["df_low"][k] == pytest.approx(kb["df_low"], rel=1e-12)
        taps = K.taps(k)
        assert np.abs(taps - kb["taps"]).max() <= 1e-12 * np.abs(kb["taps"]).max()
    nr = [small["nr"] / d[1] for d in small["direct"]]
    np.testing.assert_allclose(info["norm_ratio"], nr, rtol=1e-12)


# ------------------------------------------------------------ reconstruction

@pytest.mark.parametrize("prec", ["fp32", "split16"])
def test_reconstruct_matches_oracle(rf, ctx, small, small_gpu, prec):
    w = small["w"]
    _say(f"reconstruct small {prec}")
    out = rf.snr_reconstruct(ctx, small_gpu["K"], small_gpu["zref"], prec=prec)
    z = out["z"].cpu().numpy()
    e_same = e_direct = 0.0
    for k, kb in enumerate(small["kern"]):
        zo = orat.reconstruct(small["zr"], kb["m_lo"], kb["taps"], small["nr"] / small["direct"][k][1])
        e_same = max(e_same, np.abs(z[k] - zo).max())
        e_direct = max(e_direct, np.abs(z[k] - small["direct"][k][0]).max())
    _say(f"reconstruct small {prec}: vs same kernels {e_same:.3e}, vs direct MF {e_direct:.3e}")
    assert e_same <= TOL_SAME_KERNELS
    assert e_direct <= TOL_DIRECT


def test_reconstruct_is_deterministic(rf, ctx, small_gpu):
    a = rf.snr_reconstruct(ctx, small_gpu["K"], small_gpu["zref"], prec="split16")["z"]
    b = rf.snr_reconstruct(ctx, small_gpu["K"], small_gpu["zref"], prec="split16")["z"]
    assert torch.equal(a, b)


@pytest.mark.parametrize("prec", ["fp32", "split16"])
def test_fused_readout_equals_standalone(rf, ctx, small_gpu, prec):
    """Fused peaks/triggers equal snr_peaks on the stored series, exactly."""
    out = rf.snr_reconstruct(ctx, small_gpu["K"], small_gpu["zref"], prec=prec, fused_thr=6.0)
    ref = rf.snr_peaks(ctx, out["z"], 6.0)
    v1, i1 = rf.decode_peaks(out["peaks"])
    v2, i2 = rf.decode_peaks(ref["peaks"])
    np.testing.assert_array_equal(i1, i2)
    np.testing.assert_array_equal(v1, v2)
    assert out["ntrig"] == ref["ntrig"] > 0
    t1 = sorted(rf.decode_triggers(out["trig"], out["ntrig"]))
    t2 = sorted(rf.decode_triggers(ref["trig"], ref["ntrig"]))
    assert t1 == t2


def test_fused_only_readout_matches_oracle_peaks(rf, ctx, small, small_gpu):
    out = rf.snr_reconstruct(ctx, small_gpu["K"], small_gpu["zref"], prec="split16", store=False,
                             fused_thr=6.0)
    v, idx = rf.decode_peaks(out["peaks"])
    for k, kb in enumerate(small["kern"]):
        zo = orat.reconstruct(small["zr"], kb["m_lo"], kb["taps"], small["nr"] / small["direct"][k][1])
        pv, pi = opk.peak(zo)
        assert abs(v[k] - pv) <= TOL_SAME_KERNELS
        if pi != idx[k]:   # only a near-tie may flip the argmax
            assert abs(np.abs(zo[idx[k]]) - pv) <= 2 * TOL_SAME_KERNELS


# ------------------------------------------------------------ peaks

def _planted_series(nt, n, seed):
    rng = np.random.default_rng(seed)
    z = (rng.standard_normal((nt, n)) + 1j * rng.standard_normal((nt, n))).astype(np.complex64)
    z[0, 100] = 9.0 + 0j          # ties: first index wins
    z[0, 50000 % n] = 0 + 9.0j
    z[1, :] = 0                    # all-zero series: peak 0 at index 0
    z[2, n - 1] = 20.0
    return z


def _oracle_peaks_f32(z):
    """Oracle decisions in FP32: |z|^2 = re*re + im*im rounded per operation."""
    re = z.real.astype(np.float32)
    im = z.imag.astype(np.float32)
    a2 = (re * re) + (im * im)
    idx = a2.argmax(axis=1)
    return a2, idx


def test_snr_peaks_matches_oracle(rf, ctx):
    nt, n = 4, 65536 + 1000
    z = _planted_series(nt, n, 5)
    zt = torch.from_numpy(z).cuda()
    out = rf.snr_peaks(ctx, zt, 4.0, trig_cap=1 << 16)
    v, idx = rf.decode_peaks(out["peaks"])
    a2, oidx = _oracle_peaks_f32(z)
    np.testing.assert_array_equal(idx, oidx)
    np.testing.assert_allclose(v, np.sqrt(a2[np.arange(nt), oidx]), rtol=2e-7)
    assert idx[0] == 100 and idx[1] == 0 and idx[2] == n - 1
    thr2 = np.float32(4.0) * np.float32(4.0)
    expect = sorted((k, int(m)) for k in range(nt) for m in np.nonzero(a2[k] > thr2)[0])
    got = sorted((t[0], t[2]) for t in rf.decode_triggers(out["trig"], out["ntrig"]))
    assert out["ntrig"] == len(expect) and got == expect
    # the oracle's own definition in FP64 agrees on the values
    pv, pi = opk.peak(z[3].astype(np.complex128))
    assert abs(v[3] - pv) <= 1e-6 * pv


@pytest.mark.parametrize("n, offset", [(4097, 0), (4096, 1)])
def test_snr_peaks_unaligned_series(rf, ctx, n, offset):
    """Series whose rows are not 16-byte aligned (odd length, or a base pointer
    one element in) take the one-sample-per-load path: same decisions as the
    oracle's."""
    nt = 3
    z = _planted_series(nt, n, 13)
    flat = torch.zeros(nt * n + offset, dtype=torch.complex64, device="cuda")
    flat[offset:] = torch.from_numpy(z.reshape(-1)).cuda()
    zt = flat[offset:].view(nt, n)
    assert (zt.data_ptr() % 16 != 0) or (n % 2 == 1)
    out = rf.snr_peaks(ctx, zt, 4.0, trig_cap=1 << 14)
    v, idx = rf.decode_peaks(out["peaks"])
    a2, oidx = _oracle_peaks_f32(z)
    np.testing.assert_array_equal(idx, oidx)
    np.testing.assert_allclose(v, np.sqrt(a2[np.arange(nt), oidx]), rtol=2e-7)
    thr2 = np.float32(4.0) * np.float32(4.0)
    expect = sorted((k, int(m)) for k in range(nt) for m in np.nonzero(a2[k] > thr2)[0])
    got = sorted((t[0], t[2]) for t in rf.decode_triggers(out["trig"], out["ntrig"]))
    assert got == expect


def test_trigger_overflow_reports_true_count(rf, ctx):
    z = _planted_series(3, 4096, 9)
    out = rf.snr_peaks(ctx, torch.from_numpy(z).cuda(), 2.0, trig_cap=5)
    a2, _ = _oracle_peaks_f32(z)
    assert out["overflow"] and out["ntrig"] == int((a2 > np.float32(4.0)).sum())


# ------------------------------------------------------------ edge cases

def test_invalid_arguments_are_rejected(rf, ctx, small, small_gpu):
    w = small["w"]
    bad = synth.Grid(1024.0, 65536, 30.0, 500.0)       # f_high + 53 > fs / 2
    with pytest.raises(rf.RfError) as e:
        rf.mf_ref_snr(ctx, bad, small_gpu["xf"], small_gpu["psd"], [w["ref"]])
    assert e.value.code == rf.RF_E_INVAL
    with pytest.raises(rf.RfError):
        rf.ratio_kernel_build(ctx, w["grid"], small_gpu["psd"], w["ref"], w["nbrs"], n_build=3000)
    with pytest.raises(rf.RfError):
        rf.mf_ref_snr(ctx, w["grid"], small_gpu["xf"], small_gpu["psd"], [(1.4, -1.0)])


def test_empty_kernels_give_zero_series(rf, ctx, small, small_gpu):
    w = small["w"]
    K = rf.ratio_kernel_build(ctx, w["grid"], small_gpu["psd"], w["ref"], w["nbrs"][:3], thr=1e9)
    assert K.info()["len"] == [0, 0, 0]
    out = rf.snr_reconstruct(ctx, K, small_gpu["zref"], prec="fp32")
    assert torch.count_nonzero(out["z"]) == 0
    K.free()


@pytest.mark.parametrize("prec", ["split16", "fp32"])
def test_ragged_tiles_and_reference_delta(rf, ctx, small, small_gpu, prec):
    """130 kernels (four full tiles and a paired last tile holding 2) including
    the reference itself, whose kernel reproduces z_ref up to truncation; the
    fused read-out of the paired tile equals the read-out of its stored series."""
    w = small["w"]
    g = w["grid"]
    nbrs = (w["nbrs"] * 9)[:129] + [w["ref"]]
    K = rf.ratio_kernel_build(ctx, g, small_gpu["psd"], w["ref"], nbrs)
    out = rf.snr_reconstruct(ctx, K, small_gpu["zref"], prec=prec, fused_thr=4.0, trig_cap=1 << 16)
    ref = rf.snr_peaks(ctx, out["z"], 4.0, trig_cap=1 << 16)
    assert not out["overflow"] and not ref["overflow"]
    _same_readout(rf, out, ref)
    z = out["z"].cpu().numpy()
    for k in (0, 17, 127, 128, 129):
        kb = orat.build_kernel(g, w["ref"], nbrs[k])
        nk = omf.norm(g.fs, g.n, g.f_low, g.f_high, w["psd"], omf.template_spectrum(g.fs, g.n, *nbrs[k]))
        zo = orat.reconstruct(small["zr"], kb["m_lo"], kb["taps"], small["nr"] / nk)
        assert np.abs(z[k] - zo).max() <= TOL_SAME_KERNELS
    assert np.abs(z[129] - small["zr"]).max() <= TOL_DIRECT
    K.free()


def test_build_length_shorter_than_segment(rf, ctx, small, small_gpu):
    """n_build = n / 4: same kernel function sampled on a shorter period."""
    w = small["w"]
    g = w["grid"]
    nb = g.n // 4
    K = rf.ratio_kernel_build(ctx, g, small_gpu["psd"], w["ref"], w["nbrs"][:4], n_build=nb)
    info = K.info()
    for k in range(4):
        kb = orat.build_kernel(g, w["ref"], w["nbrs"][k], n_r=nb)
        assert info["m_lo"][k] == kb["m_lo"] and info["len"][k] == kb["taps"].size
        assert np.abs(K.taps(k) - kb["taps"]).max() <= 1e-12
    K.free()


# ------------------------------------------------------------ full size, sampled

@pytest.fixture(scope="module")
def realistic():
    return synth.workload_realistic()


def test_direct_mf_readout_full_size(rf, ctx, realistic):
    """The benchmark's comparator shape, 2^21 samples, with its 257 templates
    listed twice (513 series: two transform batches of at most 2^30 / n, so
    template offsets in the read-out), exactly as the stored series read out on
    their own."""
    w = realistic
    g = w["grid"]
    xf = _dev(w["xf"], torch.complex128)
    psd = _dev(w["psd"], torch.float64)
    tm = ([w["ref"]] + list(w["nbrs"])) * 2
    _say(f"full-size direct read-out: {len(tm)} templates, n = {g.n}")
    z, _ = rf.mf_ref_snr(ctx, g, xf, psd, tm, want_sigma=False)
    ref = rf.snr_peaks(ctx, z, 6.0, trig_cap=1 << 17)
    del z
    out = rf.mf_snr_peaks(ctx, g, xf, psd, tm, 6.0, trig_cap=1 << 17)
    _say(f"full-size direct read-out: {out['ntrig']} triggers")
    _same_readout(rf, out, ref)


def test_realistic_full_size_sampled(rf, ctx, realistic):
    """The 512 s / 4096 Hz / 256-neighbour workload in the benchmark's launch
    configuration: every sample of eight series (the four injected templates
    among them, |z| up to ~20) against the oracle and direct MF, and sampled
    times of every series against the oracle."""
    w = realistic
    g = w["grid"]
    _say("realistic: inputs to device")
    xf = _dev(w["xf"], torch.complex128)
    psd = _dev(w["psd"], torch.float64)
    zr_gpu, _ = rf.mf_ref_snr(ctx, g, xf, psd, [w["ref"]])
    zr_gpu = zr_gpu[0].contiguous()
    _say("realistic: kernel build (256)")
    K = rf.ratio_kernel_build(ctx, g, psd, w["ref"], w["nbrs"])
    info = K.info()
    _say(f"realistic: kernel lengths {min(info['len'])}..{max(info['len'])}")
    zr, nr = omf.grid_snr_series(g, w["xf"], w["psd"], *w["ref"])
    assert np.abs(zr_gpu.cpu().numpy() - zr).max() <= TOL_SAME_KERNELS
    picks = [0, 1, 100, 255] + [w["nbrs"].index((t[0], t[1])) for t in w["injections"]]
    full_o, full_d = {}, {}
    for k in picks:
        kb = orat.build_kernel(g, w["ref"], w["nbrs"][k])
        assert kb["m_lo"] == info["m_lo"][k] and kb["taps"].size == info["len"][k]
        full_d[k], nk = omf.grid_snr_series(g, w["xf"], w["psd"], *w["nbrs"][k])
        full_o[k] = orat.reconstruct(zr, kb["m_lo"], kb["taps"], nr / nk)
    rng = np.random.default_rng(77)
    idx = np.unique(rng.integers(0, g.n, 64))
    others = list(range(3, 256, 12))
    for prec in ("fp32", "split16"):
        _say(f"realistic: reconstruct {prec}")
        z = rf.snr_reconstruct(ctx, K, zr_gpu, prec=prec)["z"]
        zp = z[torch.tensor(picks, device=z.device)].cpu().numpy()
        zs = z[:, torch.from_numpy(idx).cuda()].cpu().numpy()
        del z
        e_same = max(np.abs(zp[i] - full_o[k]).max() for i, k in enumerate(picks))
        e_dir = max(np.abs(zp[i] - full_d[k]).max() for i, k in enumerate(picks))
        e_smp = 0.0
        for k in others:
            kb = orat.build_kernel(g, w["ref"], w["nbrs"][k])
            nk = omf.norm(g.fs, g.n, g.f_low, g.f_high, w["psd"], omf.template_spectrum(g.fs, g.n, *w["nbrs"][k]))
            e_smp = max(e_smp, np.abs(zs[k] - orat.reconstruct_samples(zr, kb["m_lo"], kb["taps"], nr / nk, idx)).max())
        _say(f"realistic {prec}: every sample of {len(picks)} series vs same kernels {e_same:.3e}, "
             f"vs direct MF {e_dir:.3e}; {len(others)} more series sampled {e_smp:.3e}")
        assert e_same <= TOL_SAME_KERNELS
        assert e_smp <= TOL_SAME_KERNELS
        assert e_dir <= TOL_DIRECT
    K.free()
