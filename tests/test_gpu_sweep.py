"""The SNR-loss study's measurement at one point (chirp mass 1.219, q = 0.3,
reference q = 0.6, threshold 1e-3 / s) against the FP64 oracle: kernel
support, direct and reconstructed peak SNR and their relative difference."""
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


@pytest.mark.parametrize("thr", [1e-3, 1e-2])
def test_sweep_point_against_the_oracle(rf, thr):
    w = synth.workload_sweep(1.219, 0.3)
    g = w["grid"]
    ctx = rf.Context(0)
    psd = torch.from_numpy(w["psd"]).cuda()
    xf = torch.from_numpy(w["xf"]).cuda()
    z, _ = rf.mf_ref_snr(ctx, g, xf, psd, [w["ref"], w["tgt"]], want_sigma=False)
    K = rf.ratio_kernel_build(ctx, g, psd, w["ref"], [w["tgt"]], thr=thr)
    zk = rf.snr_reconstruct(ctx, K, z[0].contiguous(), prec="split16")["z"][0]
    rho_m = z[1].abs().max().item()
    rho_r = zk.abs().max().item()
    info = K.info()
    _say(f"sweep point thr {thr}: GPU direct {rho_m:.6f}, reconstructed {rho_r:.6f}, taps {info['len'][0]}")
    # oracle: direct MF of the target, reference series, kernel, reconstruction
    zt, _ = omf.grid_snr_series(g, w["xf"], w["psd"], *w["tgt"])
    zr, nr = omf.grid_snr_series(g, w["xf"], w["psd"], *w["ref"])
    kb = orat.build_kernel(g, w["ref"], w["tgt"], threshold=thr)
    nt = omf.norm(g.fs, g.n, g.f_low, g.f_high, w["psd"], omf.template_spectrum(g.fs, g.n, *w["tgt"]))
    zo = orat.reconstruct(zr, kb["m_lo"], kb["taps"], nr / nt)
    po_m, _ = opk.peak(zt)
    po_r, _ = opk.peak(zo)
    _say(f"oracle direct {po_m:.6f}, reconstructed {po_r:.6f}, taps {len(kb['taps'])}")
    assert info["m_lo"][0] == kb["m_lo"] and info["len"][0] == len(kb["taps"])
    assert abs(rho_m - po_m) <= 1e-5 and abs(rho_r - po_r) <= 1e-5
    loss_gpu = abs(rho_r - rho_m) / rho_m
    loss_orc = abs(po_r - po_m) / po_m
    _say(f"loss GPU {loss_gpu:.3e}, oracle {loss_orc:.3e}")
    assert abs(loss_gpu - loss_orc) <= 2.5e-5 / po_m      # the two 1e-5 bars above, over the peak
    K.free()
    ctx.close()
