"""Where the split-FP16 reconstruction takes its correction products: the
granule flags the operand packing marks on the GPU, read back as step counts
(rf_kernels_split_steps), against the rule recomputed here from the kernels'
FP64 taps (integer counts, exact), for every window chunk size; and both
reconstruction forms against the FP64 oracle at every output sample."""
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


def _expected_steps(info, taps, chunk, n):
    """Tiles: kernels sorted by first tap (stable), 32 per tile, union support
    from a multiple of 4, rounded up to 128 taps; a tile of at most 16 kernels
    is paired: each kernel also sits in a second column 32 taps later, so its
    support reaches 32 taps further (if it then still fits the n-sample
    segment); a 256-tap granule is marked where a column has |w| s_k >= 1/2
    (s_k = 2^(14 - e), e the binary exponent of the largest |w| as an FP32
    value); a step takes the corrections when its 512-tap block holds a marked
    granule, whatever the window chunk.  Counts are in steps of a 32-kernel
    tile: a paired tile's step counts one half."""
    nk = len(info["len"])
    order = sorted(range(nk), key=lambda k: info["m_lo"][k])
    corr = total = 0
    for t in range(0, nk, 32):
        ks = [k for k in order[t:t + 32] if info["len"][k] > 0]
        if not ks:
            continue
        m0 = (min(info["m_lo"][k] for k in ks) // 4) * 4
        hi = max(info["m_lo"][k] + info["len"][k] for k in ks)
        shifts, per = [0], 1
        if len(order[t:t + 32]) <= 16 and -(-(hi + 32 - m0) // 128) * 128 <= n:
            shifts, hi, per = [0, 32], hi + 32, 2
        ntaps = -(-(hi - m0) // 128) * 128
        marked = np.zeros(ntaps // 256 + 1, bool)
        for k in ks:
            w = taps[k]
            e = np.frexp(np.float32(np.abs(w).max()))[1]
            s = 2.0 ** (14 - int(e))
            for sh in shifts:
                pos = np.nonzero(np.abs(w * s) >= 0.5)[0] + (info["m_lo"][k] - m0) + sh
                marked[np.unique(pos // 256)] = True
        total += ntaps // 16 // per
        for t0 in range(0, ntaps, 512):
            b = min(t0 + 512, ntaps)
            if marked[t0 // 256: -(-b // 256)].any():
                corr += (b - t0) // 16 // per
    return corr, total


def test_flags_and_step_counts_match_the_rule(rf):
    w = synth.workload_realistic(n_nbr=40, duration=64.0)        # a full and a paired tile
    g = w["grid"]
    ctx = rf.Context(0)
    psd = torch.from_numpy(w["psd"]).cuda()
    K = rf.ratio_kernel_build(ctx, g, psd, w["ref"], w["nbrs"])
    info = K.info()
    taps = [K.taps(k) for k in range(K.nk)]
    for chunk in (256, 512, 1024):
        got = K.split_steps(chunk)
        exp = _expected_steps(info, taps, chunk, g.n)
        _say(f"chunk {chunk}: correction steps {got[0]} of {got[1]} (expected {exp[0]} of {exp[1]})")
        assert got == exp
        assert got[0] < 0.6 * got[1]
    # invalid chunk sizes are rejected
    import ctypes
    c, a = ctypes.c_int64(), ctypes.c_int64()
    for bad in (0, 128, 384, 2048):
        assert ctx.lib.rf_kernels_split_steps(K.h, bad, ctypes.byref(c), ctypes.byref(a)) == rf.RF_E_INVAL
    # the reconstruction with these flags against the oracle at every sample of every
    # series (the SNR-20 injection puts |z| near 20, where FP32 partial sums round)
    xf = torch.from_numpy(w["xf"]).cuda()
    z, _ = rf.mf_ref_snr(ctx, g, xf, psd, [w["ref"]])
    zr, nr = omf.grid_snr_series(g, w["xf"], w["psd"], *w["ref"])
    zo = []
    for k in range(K.nk):
        kb = orat.build_kernel(g, w["ref"], w["nbrs"][k])
        nk = omf.norm(g.fs, g.n, g.f_low, g.f_high, w["psd"], omf.template_spectrum(g.fs, g.n, *w["nbrs"][k]))
        zo.append(orat.reconstruct(zr, kb["m_lo"], kb["taps"], nr / nk))
    zo = np.array(zo)
    for prec in ("split16", "fp32"):
        zh = rf.snr_reconstruct(ctx, K, z[0].contiguous(), prec=prec)["z"].cpu().numpy()
        err = np.abs(zh - zo).max()
        _say(f"{prec} vs oracle, every sample of {K.nk} series (max |z| {np.abs(zo).max():.1f}): {err:.3e}")
        assert err <= 1e-5
    K.free()
    torch.cuda.synchronize()
    ctx.close()
