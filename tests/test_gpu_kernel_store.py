"""Kernel sets stored and reused (rf_kernels_save / rf_kernels_load): the file
read back independently in the layout include/rf.h documents, a loaded set
equal to the built one field by field and tap by tap, reconstructions from it
equal bit for bit (split FP16 and FP32, a paired tile included), and damaged
or foreign files rejected."""
import ctypes
import struct
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


def _parse(raw):
    """The documented layout, read with struct/numpy (no library code)."""
    assert raw[:8] == b"RFKSET01"
    version, nk, n_build, fs, total = struct.unpack_from("<iiqdq", raw, 8)
    o = 8 + 32
    arr = {}
    for name, dt in (("m_lo", "<i8"), ("len", "<i4"), ("off", "<i8"), ("norm_ratio", "<f8"),
                     ("df_low", "<f8"), ("kscale", "<f8")):
        a = np.frombuffer(raw, dtype=dt, count=nk, offset=o)
        arr[name] = a
        o += a.nbytes
    taps = np.frombuffer(raw, dtype="<f8", count=total, offset=o)
    o += taps.nbytes
    (h,) = struct.unpack_from("<Q", raw, o)
    assert o + 8 == len(raw)
    x = 14695981039346656037
    for c in raw[8:o]:
        x = ((x ^ c) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    assert x == h
    return version, nk, n_build, fs, arr, taps


def test_save_load_roundtrip(rf, tmp_path):
    w = synth.workload_small()                      # 16 neighbours: one paired tile
    g = w["grid"]
    ctx = rf.Context(0)
    psd = torch.from_numpy(w["psd"]).cuda()
    xf = torch.from_numpy(w["xf"]).cuda()
    K = rf.ratio_kernel_build(ctx, g, psd, w["ref"], w["nbrs"])
    path = str(tmp_path / "set.rfk")
    rf.kernels_save(ctx, K, path)
    raw = open(path, "rb").read()
    version, nk, n_build, fs, arr, taps = _parse(raw)
    info = K.info()
    assert (version, nk, n_build, fs) == (1, K.nk, g.n, g.fs)
    np.testing.assert_array_equal(arr["m_lo"], info["m_lo"])
    np.testing.assert_array_equal(arr["len"], info["len"])
    np.testing.assert_array_equal(arr["norm_ratio"], info["norm_ratio"])
    for k in range(nk):
        np.testing.assert_array_equal(taps[arr["off"][k]:arr["off"][k] + arr["len"][k]], K.taps(k))
    _say(f"kernel set file: {len(raw)} bytes for {nk} kernels, {taps.size} taps")

    K2 = rf.kernels_load(ctx, path)
    info2 = K2.info()
    for key in ("m_lo", "len", "norm_ratio", "df_low"):
        assert info2[key] == info[key]
    for k in range(nk):
        np.testing.assert_array_equal(K2.taps(k), K.taps(k))
    assert K2.split_steps(1024) == K.split_steps(1024)
    z, _ = rf.mf_ref_snr(ctx, g, xf, psd, [w["ref"]])
    zr = z[0].contiguous()
    for prec in ("split16", "fp32"):
        a = rf.snr_reconstruct(ctx, K, zr, prec=prec, fused_thr=6.0)
        b = rf.snr_reconstruct(ctx, K2, zr, prec=prec, fused_thr=6.0)
        assert torch.equal(a["z"], b["z"]), prec
        assert torch.equal(a["peaks"], b["peaks"]), prec
        assert a["ntrig"] == b["ntrig"]

    # damaged and foreign files
    def load_status(p):
        h = ctypes.c_void_p(123)
        st = ctx.lib.rf_kernels_load(ctx.h, str(p).encode(), ctypes.byref(h))
        assert h.value is None
        return st
    bad = bytearray(raw)
    bad[len(raw) // 2] ^= 0x40                       # one bit inside the taps
    (tmp_path / "flip.rfk").write_bytes(bytes(bad))
    assert load_status(tmp_path / "flip.rfk") == rf.RF_E_INVAL
    (tmp_path / "short.rfk").write_bytes(raw[:-9])
    assert load_status(tmp_path / "short.rfk") == rf.RF_E_INVAL
    (tmp_path / "long.rfk").write_bytes(raw + b"\0")
    assert load_status(tmp_path / "long.rfk") == rf.RF_E_INVAL
    (tmp_path / "tag.rfk").write_bytes(b"RFKSET02" + raw[8:])
    assert load_status(tmp_path / "tag.rfk") == rf.RF_E_INVAL
    assert load_status(tmp_path / "missing.rfk") == rf.RF_E_INVAL
    assert ctx.lib.rf_kernels_save(ctx.h, K.h, str(tmp_path / "no_dir" / "x.rfk").encode()) == rf.RF_E_INVAL
    K2.free()
    K.free()
    torch.cuda.synchronize()
    ctx.close()
