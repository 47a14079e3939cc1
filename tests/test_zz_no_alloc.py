"""snr_reconstruct_noalloc (work buffers in the library's static device array)
against snr_reconstruct on the same kernels: identical series and read-out, on
two calls in a row, the second with a smaller input, for both precisions; and
the size limits rejected on the host."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

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


def _case(rf, ctx, w, nk):
    g = w["grid"]
    psd = torch.from_numpy(w["psd"]).cuda()
    xf = torch.from_numpy(w["xf"]).cuda()
    z, _ = rf.mf_ref_snr(ctx, g, xf, psd, [w["ref"]])
    K = rf.ratio_kernel_build(ctx, g, psd, w["ref"], w["nbrs"][:nk])
    return z[0].contiguous(), K


def _same(rf, a, b):
    assert torch.equal(a["z"], b["z"])
    va, ia = rf.decode_peaks(a["peaks"])
    vb, ib = rf.decode_peaks(b["peaks"])
    np.testing.assert_array_equal(va, vb)
    np.testing.assert_array_equal(ia, ib)
    assert a["ntrig"] == b["ntrig"]
    ta = sorted(rf.decode_triggers(a["trig"], a["ntrig"]))
    tb = sorted(rf.decode_triggers(b["trig"], b["ntrig"]))
    assert ta == tb


@pytest.mark.parametrize("prec", ["split16", "fp32"])
def test_noalloc_matches_allocating_call(rf, prec):
    ctx = rf.Context(0)
    big = synth.workload_realistic(n_nbr=64, duration=128.0)      # n = 2^19, 64 kernels
    small = synth.workload_small()                                 # n = 2^16, 16 kernels
    for name, w, nk in (("128 s, 64 kernels", big, 64), ("64 s, 12 kernels", small, 12)):
        _say(f"noalloc {prec}: {name}")
        zr, K = _case(rf, ctx, w, nk)
        a = rf.snr_reconstruct(ctx, K, zr, prec=prec, fused_thr=6.0, trig_cap=1 << 14)
        b = rf.snr_reconstruct(ctx, K, zr, prec=prec, fused_thr=6.0, trig_cap=1 << 14, noalloc=True)
        torch.cuda.synchronize()
        _same(rf, a, b)
        assert a["ntrig"] > 0 or name.startswith("64")
        K.free()
    ctx.close()


def test_noalloc_size_limits(rf):
    ctx = rf.Context(0)
    w = synth.workload_small()
    zr, K = _case(rf, ctx, w, 4)
    long = torch.zeros(1 << 22, dtype=torch.complex64, device="cuda")
    with pytest.raises(rf.RfError) as e:
        rf.snr_reconstruct(ctx, K, long, prec="split16", store=False, fused_thr=6.0, noalloc=True)
    assert e.value.code == rf.RF_E_INVAL and "2^21" in str(e.value)
    K.free()
    g = w["grid"]
    psd = torch.from_numpy(w["psd"]).cuda()
    many = synth.neighbour_lattice(*w["ref"], g.f_low, 4100)
    K = rf.ratio_kernel_build(ctx, g, psd, w["ref"], many, n_build=1 << 12)
    with pytest.raises(rf.RfError) as e:
        rf.snr_reconstruct(ctx, K, zr, prec="fp32", store=False, fused_thr=6.0, noalloc=True)
    assert e.value.code == rf.RF_E_INVAL and "4096" in str(e.value)
    K.free()
    ctx.close()
