"""Next-generation-detector shape: 2048 s at 4096 Hz (n = 2^23, the largest
segment the library takes below its 2^24 limit), f_low = 10 Hz, kernels of
16k-28k taps; one 1+1 Msun reference with 48 lattice neighbours (a ragged
tile), an SNR-15 injection.  Split-FP16, FP32 and factored reconstruction
against direct matched filtering at every sample and against the FP64 oracle
at sampled outputs."""
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
def st(rf):
    w = synth.workload_stress(n_nbr=48, refs=((1.0, 1.0),))
    g = w["grid"]
    ref, nbrs = w["refs"][0], w["groups"][0]
    ctx = rf.Context(0)
    _say("stress: inputs to device, kernel build")
    xf = torch.from_numpy(w["xf"]).cuda()
    psd = torch.from_numpy(w["psd"]).cuda()
    K = rf.ratio_kernel_build(ctx, g, psd, ref, nbrs)
    z, _ = rf.mf_ref_snr(ctx, g, xf, psd, [ref])
    zd, _ = rf.mf_ref_snr(ctx, g, xf, psd, nbrs)
    _say("stress: oracle reference series and three kernels")
    zr, nr = omf.grid_snr_series(g, w["xf"], w["psd"], *ref)
    picks = (0, 23, 47)
    oks = {k: orat.build_kernel(g, ref, nbrs[k]) for k in picks}
    onr = {k: omf.norm(g.fs, g.n, g.f_low, g.f_high, w["psd"], omf.template_spectrum(g.fs, g.n, *nbrs[k]))
           for k in picks}
    rng = np.random.default_rng(9)
    t_inj = int(w["injections"][0][3] * g.fs)
    idx = np.unique(np.concatenate([rng.integers(0, g.n, 300), t_inj + np.arange(-64, 64)]))
    yield dict(w=w, g=g, ref=ref, nbrs=nbrs, ctx=ctx, xf=xf, psd=psd, K=K, z=z[0].contiguous(), zd=zd,
               zr=zr, nr=nr, oks=oks, onr=onr, idx=idx, picks=picks)
    torch.cuda.synchronize()
    K.free()
    ctx.close()


def test_kernels_match_the_oracle(rf, st):
    info = st["K"].info()
    assert max(info["len"]) <= 65536
    for k in st["picks"]:
        kb = st["oks"][k]
        assert info["m_lo"][k] == kb["m_lo"] and info["len"][k] == len(kb["taps"])
        assert np.abs(st["K"].taps(k) - kb["taps"]).max() <= 1e-9 * np.abs(kb["taps"]).max()


@pytest.mark.parametrize("prec", ["split16", "fp32"])
def test_reconstruction(rf, st, prec):
    out = rf.snr_reconstruct(st["ctx"], st["K"], st["z"], prec=prec, fused_thr=6.0, trig_cap=1 << 14)
    z = out["z"]
    ed = (z - st["zd"]).abs().max().item()
    zh = z.cpu().numpy()
    eo = 0.0
    for k in st["picks"]:
        kb = st["oks"][k]
        zo = orat.reconstruct_samples(st["zr"], kb["m_lo"], kb["taps"], st["nr"] / st["onr"][k], st["idx"])
        eo = max(eo, np.abs(zh[k, st["idx"]] - zo).max())
    _say(f"stress {prec}: vs direct MF {ed:.3e}, vs oracle (sampled) {eo:.3e}")
    assert eo <= 1e-5
    assert ed <= 2e-4
    ref = rf.snr_peaks(st["ctx"], z, 6.0, trig_cap=1 << 14)
    torch.cuda.synchronize()
    assert torch.equal(out["peaks"], ref["peaks"])
    del z, out


@pytest.mark.parametrize("prec", ["split16", "fp32"])
def test_factored(rf, st, prec):
    F = rf.Factored(st["ctx"], st["K"], st["g"], tol=2e-6, jmax=48)
    J = F.info()["J"]
    z = F.reconstruct(st["z"], prec=prec)["z"]
    ed = (z - st["zd"]).abs().max().item()
    _say(f"stress factored {prec}: J = {J}, vs direct MF {ed:.3e}")
    assert ed <= 2e-4
    del z
    F.free()


def test_ols(rf, st):
    """Kernels of 16k-28k taps: up to 8 partitions, spectra read per block."""
    O = rf.Ols(st["ctx"], st["K"], st["g"].n)
    info = O.info()
    assert info["pmax"] > 4
    z = O.reconstruct(st["z"])["z"]
    ed = (z - st["zd"]).abs().max().item()
    zh = z.cpu().numpy()
    eo = 0.0
    for k in st["picks"]:
        kb = st["oks"][k]
        zo = orat.reconstruct_samples(st["zr"], kb["m_lo"], kb["taps"], st["nr"] / st["onr"][k], st["idx"])
        eo = max(eo, np.abs(zh[k, st["idx"]] - zo).max())
    _say(f"stress ols: partitions up to {info['pmax']}, vs direct MF {ed:.3e}, vs oracle (sampled) {eo:.3e}")
    assert eo <= 1e-5
    assert ed <= 2e-4
    del z
    O.free()
