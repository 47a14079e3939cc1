"""ctypes binding of librf (the C ABI declared in include/rf.h).

Argument marshalling only: every step runs in the HIP library.  PyTorch
provides device memory and the stream; tensors are passed by data pointer.
The library must have been built (paper_2511_12894_amd/build_lib.sh, or
__graft_entry__.build()); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librf.so")

RF_OK, RF_E_INVAL, RF_E_NOMEM, RF_E_HIP, RF_E_UNSUPPORTED, RF_E_OVERFLOW = range(6)
RF_THR_PER_SECOND, RF_THR_PER_TAP = 0, 1
RF_PREC_FP32, RF_PREC_SPLIT_FP16 = 0, 1
PREC = {"fp32": RF_PREC_FP32, "split16": RF_PREC_SPLIT_FP16}

EXPORTED = ("rf_ctx_create", "rf_ctx_destroy", "rf_last_error", "mf_ref_snr", "mf_snr_peaks", "ratio_kernel_build",
            "rf_kernels_info", "rf_kernels_taps_fp64", "rf_kernels_split_steps", "rf_kernels_free",
            "rf_kernels_save", "rf_kernels_load", "snr_reconstruct", "snr_reconstruct_noalloc",
            "snr_peaks", "rf_batch_create", "rf_batch_info", "rf_batch_set_chunks",
            "rf_batch_get_tuning", "rf_batch_set_tuning", "rf_batch_autotune", "rf_batch_run", "rf_batch_graph_stats", "rf_batch_free", "rf_surrogate_create",
            "rf_surrogate_info", "rf_surrogate_set_params", "rf_surrogate_get_params",
            "rf_surrogate_dataset", "rf_surrogate_grad", "rf_surrogate_train", "rf_surrogate_predict", "rf_surrogate_project",
            "rf_surrogate_encode", "rf_surrogate_decode",
            "rf_surrogate_kernels", "rf_factored_build", "rf_factored_info", "snr_reconstruct_factored",
            "snr_reconstruct_factored_batch",
            "rf_factored_free", "rf_ols_build", "rf_ols_info", "snr_reconstruct_ols", "rf_ols_free",
            "rf_template_durations", "rf_bank_organise", "rf_surrogate_free")


class RfGrid(ctypes.Structure):
    _fields_ = [("fs", ctypes.c_double), ("n", ctypes.c_int64), ("f_low", ctypes.c_double),
                ("f_high", ctypes.c_double), ("df_high", ctypes.c_double),
                ("df_low_max", ctypes.c_double)]


class RfTmpl(ctypes.Structure):
    _fields_ = [("m1", ctypes.c_double), ("m2", ctypes.c_double)]


class RfBatchTuning(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32 * 3), ("blocks", ctypes.c_int32 * 3), ("xcd_queues", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("bucket_hi", ctypes.c_int64 * 2)]


class RfPeak(ctypes.Structure):
    _fields_ = [("max_absz", ctypes.c_float), ("argmax", ctypes.c_int32)]


class RfTrigger(ctypes.Structure):
    _fields_ = [("tmpl", ctypes.c_int32), ("seg", ctypes.c_int32), ("idx", ctypes.c_int32),
                ("absz", ctypes.c_float), ("argz", ctypes.c_float)]


class RfPeakArgs(ctypes.Structure):
    _fields_ = [("thr", ctypes.c_float), ("peaks", ctypes.c_void_p), ("trig", ctypes.c_void_p),
                ("cap", ctypes.c_int64), ("ntrig", ctypes.POINTER(ctypes.c_int64))]


class RfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"librf status {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load librf.so (once).  Raises when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"librf.so not built at {path}; run paper_2511_12894_amd/build_lib.sh")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.rf_ctx_create.argtypes = [ctypes.c_int, vp, ctypes.POINTER(vp)]
    lib.rf_ctx_destroy.argtypes = [vp]
    lib.rf_last_error.argtypes = [vp]
    lib.rf_last_error.restype = ctypes.c_char_p
    lib.mf_ref_snr.argtypes = [vp, ctypes.POINTER(RfGrid), vp, vp, ctypes.POINTER(RfTmpl), i32, vp,
                               ctypes.POINTER(dbl)]
    lib.mf_snr_peaks.argtypes = [vp, ctypes.POINTER(RfGrid), vp, vp, ctypes.POINTER(RfTmpl), i32,
                                 ctypes.POINTER(RfPeakArgs)]
    lib.ratio_kernel_build.argtypes = [vp, ctypes.POINTER(RfGrid), vp, RfTmpl, ctypes.POINTER(RfTmpl),
                                       i32, dbl, ctypes.c_int, i64, ctypes.POINTER(vp)]
    lib.rf_kernels_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i32),
                                    ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    lib.rf_kernels_taps_fp64.argtypes = [vp, i32, ctypes.POINTER(dbl)]
    lib.rf_kernels_split_steps.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.rf_kernels_free.argtypes = [vp]
    lib.rf_kernels_save.argtypes = [vp, vp, ctypes.c_char_p]
    lib.rf_kernels_load.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(vp)]
    lib.snr_reconstruct.argtypes = [vp, vp, vp, i64, ctypes.c_int, vp, ctypes.POINTER(RfPeakArgs)]
    lib.snr_reconstruct_noalloc.argtypes = [vp, vp, vp, i64, ctypes.c_int, vp, ctypes.POINTER(RfPeakArgs)]
    lib.snr_peaks.argtypes = [vp, vp, i32, i64, ctypes.c_float, vp, vp, i64, ctypes.POINTER(i64)]
    lib.rf_batch_create.argtypes = [vp, ctypes.POINTER(RfGrid), vp, i32, ctypes.POINTER(RfTmpl),
                                    ctypes.POINTER(vp), i32, ctypes.POINTER(vp)]
    lib.rf_batch_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i32),
                                  ctypes.POINTER(i32)]
    lib.rf_batch_set_chunks.argtypes = [vp, ctypes.POINTER(i32)]
    lib.rf_batch_get_tuning.argtypes = [vp, ctypes.POINTER(RfBatchTuning)]
    lib.rf_batch_set_tuning.argtypes = [vp, ctypes.POINTER(RfBatchTuning)]
    lib.rf_batch_autotune.argtypes = [vp, vp, vp, ctypes.c_char_p]
    lib.rf_batch_run.argtypes = [vp, vp, vp, ctypes.c_float, vp, vp, i64, ctypes.POINTER(i64)]
    lib.rf_batch_graph_stats.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_float)]
    lib.rf_batch_free.argtypes = [vp]
    lib.rf_surrogate_create.argtypes = [vp, ctypes.POINTER(RfGrid), ctypes.POINTER(RfTmpl), ctypes.POINTER(RfTmpl),
                                        i32, i32, i32, vp, i32, ctypes.POINTER(vp)]
    lib.rf_surrogate_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                      ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    lib.rf_surrogate_set_params.argtypes = [vp, vp, vp]
    lib.rf_surrogate_get_params.argtypes = [vp, vp, vp]
    lib.rf_surrogate_dataset.argtypes = [vp, vp, vp, vp]
    lib.rf_surrogate_grad.argtypes = [vp, vp, vp, vp, i32, ctypes.POINTER(ctypes.c_float), vp]
    lib.rf_surrogate_train.argtypes = [vp, vp, vp, i32, i32, ctypes.c_float, ctypes.POINTER(ctypes.c_float)]
    lib.rf_surrogate_predict.argtypes = [vp, vp, RfTmpl, ctypes.POINTER(RfTmpl), i32, vp]
    lib.rf_surrogate_project.argtypes = [vp, vp, RfTmpl, ctypes.POINTER(RfTmpl), i32, vp]
    lib.rf_surrogate_encode.argtypes = [vp, vp, RfTmpl, ctypes.POINTER(RfTmpl), i32, i32, i32, vp, vp]
    lib.rf_surrogate_decode.argtypes = [vp, vp, RfTmpl, ctypes.POINTER(RfTmpl), i32, i32, i32, vp, vp, vp]
    lib.rf_surrogate_kernels.argtypes = [vp, vp, ctypes.POINTER(RfGrid), vp, RfTmpl, ctypes.POINTER(RfTmpl), i32,
                                         vp, dbl, ctypes.c_int, ctypes.POINTER(RfGrid), vp, vp, dbl,
                                         ctypes.POINTER(vp), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float)]
    lib.rf_surrogate_free.argtypes = [vp]
    lib.rf_factored_build.argtypes = [vp, vp, ctypes.POINTER(RfGrid), dbl, i32, ctypes.POINTER(vp)]
    lib.rf_factored_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i64),
                                     ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    lib.snr_reconstruct_factored.argtypes = [vp, vp, vp, i64, i32, vp, ctypes.POINTER(RfPeakArgs)]
    lib.snr_reconstruct_factored_batch.argtypes = [vp, ctypes.POINTER(RfGrid), vp, i32, vp, i32,
                                                   ctypes.POINTER(vp), ctypes.POINTER(RfTmpl), i32,
                                                   ctypes.POINTER(RfPeakArgs)]
    lib.rf_factored_free.argtypes = [vp]
    lib.rf_ols_build.argtypes = [vp, vp, i64, ctypes.POINTER(vp)]
    lib.rf_ols_info.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                ctypes.POINTER(i32), ctypes.POINTER(i64)]
    lib.snr_reconstruct_ols.argtypes = [vp, vp, vp, i64, vp, ctypes.POINTER(RfPeakArgs)]
    lib.rf_ols_free.argtypes = [vp]
    lib.rf_template_durations.argtypes = [ctypes.POINTER(RfTmpl), i64, dbl, ctypes.POINTER(dbl)]
    lib.rf_bank_organise.argtypes = [ctypes.POINTER(RfTmpl), ctypes.POINTER(dbl), i64, dbl, i32,
                                     ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i32)]
    for name in EXPORTED:
        if name != "rf_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def to_grid(g) -> RfGrid:
    return RfGrid(float(g.fs), int(g.n), float(g.f_low), float(g.f_high), float(g.df_high),
                  float(g.df_low_max))


def _tmpl_array(ts):
    arr = (RfTmpl * len(ts))()
    for i, (m1, m2) in enumerate(ts):
        arr[i] = RfTmpl(float(m1), float(m2))
    return arr


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _require(cond, msg):
    """Argument check that survives python -O (unlike assert)."""
    if not cond:
        raise ValueError(msg)


def _dev_tensor(t, dtype, numel=None, shape=None, what="tensor"):
    """A contiguous CUDA tensor of the given dtype and size, else ValueError."""
    _require(isinstance(t, torch.Tensor), f"{what}: expected a torch tensor")
    _require(t.dtype == dtype, f"{what}: expected dtype {dtype}, got {t.dtype}")
    _require(t.is_cuda, f"{what}: must be on a CUDA device")
    _require(t.is_contiguous(), f"{what}: must be contiguous")
    if numel is not None:
        _require(t.numel() == numel, f"{what}: expected {numel} elements, got {t.numel()}")
    if shape is not None:
        _require(tuple(t.shape) == tuple(shape), f"{what}: expected shape {tuple(shape)}, got {tuple(t.shape)}")


class Context:
    """rf_ctx on a device, enqueuing on a torch stream (default: current)."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.lib = load()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        st = self.lib.rf_ctx_create(device, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != RF_OK:
            raise RfError(st, "rf_ctx_create failed")
        self.h = h

    def check(self, st):
        if st != RF_OK:
            raise RfError(st, self.lib.rf_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.rf_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Kernels:
    ctx: Context
    h: ctypes.c_void_p
    nk: int

    def info(self):
        nk = self.nk
        m_lo = (ctypes.c_int64 * nk)()
        ln = (ctypes.c_int32 * nk)()
        nr = (ctypes.c_double * nk)()
        dfl = (ctypes.c_double * nk)()
        n = ctypes.c_int32()
        self.ctx.check(self.ctx.lib.rf_kernels_info(self.h, ctypes.byref(n), m_lo, ln, nr, dfl))
        return dict(m_lo=list(m_lo), len=list(ln), norm_ratio=list(nr), df_low=list(dfl))

    def split_steps(self, chunk: int = 1024):
        """(steps with the correction products, all steps) of the split-FP16 form."""
        c, a = ctypes.c_int64(), ctypes.c_int64()
        self.ctx.check(self.ctx.lib.rf_kernels_split_steps(self.h, int(chunk), ctypes.byref(c), ctypes.byref(a)))
        return c.value, a.value

    def taps(self, k: int):
        import numpy as np
        L = self.info()["len"][k]
        out = (ctypes.c_double * max(L, 1))()
        self.ctx.check(self.ctx.lib.rf_kernels_taps_fp64(self.h, k, out))
        return np.frombuffer(out, dtype=np.float64, count=L).copy()

    def free(self):
        if self.h:
            self.ctx.lib.rf_kernels_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def mf_ref_snr(ctx: Context, grid, xf: torch.Tensor, psd: torch.Tensor, templates, z=None,
               want_sigma: bool = True):
    """Complex SNR series of each template: z complex64 [nt, n] (device), sigma list."""
    n = int(grid.n)
    _dev_tensor(xf, torch.complex128, n // 2 + 1, what="xf")
    _dev_tensor(psd, torch.float64, n // 2 + 1, what="psd")
    nt = len(templates)
    if z is None:
        z = torch.empty((nt, n), dtype=torch.complex64, device=xf.device)
    _dev_tensor(z, torch.complex64, what="z")
    _require(z.numel() >= nt * n, "z: needs room for nt * n samples")
    g = to_grid(grid)
    sig = (ctypes.c_double * nt)() if want_sigma else None
    ctx.check(ctx.lib.mf_ref_snr(ctx.h, ctypes.byref(g), _ptr(xf), _ptr(psd), _tmpl_array(templates),
                                 nt, _ptr(z), sig))
    return z, (list(sig) if want_sigma else None)


def mf_snr_peaks(ctx: Context, grid, xf: torch.Tensor, psd: torch.Tensor, templates, thr: float,
                 trig_cap: int = 4096):
    """Direct matched filtering of each template with the read-out only (the
    series are not stored): peaks tensor of RfPeak bytes, triggers, count."""
    n = int(grid.n)
    _dev_tensor(xf, torch.complex128, n // 2 + 1, what="xf")
    _dev_tensor(psd, torch.float64, n // 2 + 1, what="psd")
    nt = len(templates)
    peaks = torch.empty((nt, 2), dtype=torch.int32, device=xf.device)
    trig = torch.empty((max(trig_cap, 1), 5), dtype=torch.int32, device=xf.device)
    cnt = ctypes.c_int64(0)
    args = RfPeakArgs(float(thr), peaks.data_ptr(), trig.data_ptr(), int(trig_cap), ctypes.pointer(cnt))
    g = to_grid(grid)
    st = ctx.lib.mf_snr_peaks(ctx.h, ctypes.byref(g), _ptr(xf), _ptr(psd), _tmpl_array(templates), nt,
                              ctypes.byref(args))
    if st not in (RF_OK, RF_E_OVERFLOW):
        ctx.check(st)
    return dict(peaks=peaks, trig=trig, ntrig=int(cnt.value), overflow=(st == RF_E_OVERFLOW))


def kernels_save(ctx: Context, kernels: "Kernels", path: str):
    """Write a kernel set to `path` (rf_kernels_save)."""
    ctx.check(ctx.lib.rf_kernels_save(ctx.h, kernels.h, os.fsencode(path)))


def kernels_load(ctx: Context, path: str) -> "Kernels":
    """Read a kernel set written by kernels_save onto ctx's device (rf_kernels_load)."""
    h = ctypes.c_void_p()
    ctx.check(ctx.lib.rf_kernels_load(ctx.h, os.fsencode(path), ctypes.byref(h)))
    nk = ctypes.c_int32()
    ctx.check(ctx.lib.rf_kernels_info(h, ctypes.byref(nk), None, None, None, None))
    return Kernels(ctx, h, nk.value)


def ratio_kernel_build(ctx: Context, grid, psd: torch.Tensor, ref, nbrs, thr: float = 1e-3,
                       unit: int = RF_THR_PER_SECOND, n_build: int = 0) -> Kernels:
    _dev_tensor(psd, torch.float64, int(grid.n) // 2 + 1, what="psd")
    g = to_grid(grid)
    h = ctypes.c_void_p()
    ctx.check(ctx.lib.ratio_kernel_build(ctx.h, ctypes.byref(g), _ptr(psd), RfTmpl(*map(float, ref)),
                                         _tmpl_array(nbrs), len(nbrs), float(thr), int(unit),
                                         int(n_build), ctypes.byref(h)))
    return Kernels(ctx, h, len(nbrs))


def snr_reconstruct(ctx: Context, kernels: Kernels, z_ref: torch.Tensor, prec: str = "split16",
                    z_out=None, store: bool = True, fused_thr: float | None = None,
                    trig_cap: int = 4096, noalloc: bool = False):
    """Reconstructed series [nk, n] (if store) and, with fused_thr, the fused
    read-out (peaks tensor of RfPeak bytes, triggers, count).  noalloc selects
    snr_reconstruct_noalloc (the library allocates nothing; the outputs are
    still the caller's)."""
    _dev_tensor(z_ref, torch.complex64, what="z_ref")
    n = z_ref.numel()
    if store and z_out is None:
        z_out = torch.empty((kernels.nk, n), dtype=torch.complex64, device=z_ref.device)
    if store:
        _dev_tensor(z_out, torch.complex64, shape=(kernels.nk, n), what="z_out")
    fused = None
    peaks = trig = None
    cnt = ctypes.c_int64(0)
    if fused_thr is not None:
        peaks = torch.empty((kernels.nk, 2), dtype=torch.int32, device=z_ref.device)
        trig = torch.empty((max(trig_cap, 1), 5), dtype=torch.int32, device=z_ref.device)
        fused = RfPeakArgs(float(fused_thr), peaks.data_ptr(), trig.data_ptr(), int(trig_cap),
                           ctypes.pointer(cnt))
    fn = ctx.lib.snr_reconstruct_noalloc if noalloc else ctx.lib.snr_reconstruct
    st = fn(ctx.h, kernels.h, _ptr(z_ref), n, PREC[prec], _ptr(z_out) if store else None,
            ctypes.byref(fused) if fused is not None else None)
    if st not in (RF_OK, RF_E_OVERFLOW):
        ctx.check(st)
    out = dict(z=z_out if store else None)
    if fused is not None:
        out.update(peaks=peaks, trig=trig, ntrig=int(cnt.value), overflow=(st == RF_E_OVERFLOW))
    return out


def snr_peaks(ctx: Context, z: torch.Tensor, thr: float, trig_cap: int = 4096):
    """Peaks and threshold crossings of series z [nt, n] (complex64, device)."""
    _dev_tensor(z, torch.complex64, what="z")
    _require(z.dim() == 2, "z: expected [nt, n]")
    nt, n = z.shape
    peaks = torch.empty((nt, 2), dtype=torch.int32, device=z.device)
    trig = torch.empty((max(trig_cap, 1), 5), dtype=torch.int32, device=z.device)
    cnt = ctypes.c_int64(0)
    st = ctx.lib.snr_peaks(ctx.h, _ptr(z), nt, n, ctypes.c_float(thr), _ptr(peaks), _ptr(trig),
                           int(trig_cap), ctypes.byref(cnt))
    if st not in (RF_OK, RF_E_OVERFLOW):
        ctx.check(st)
    return dict(peaks=peaks, trig=trig, ntrig=int(cnt.value), overflow=(st == RF_E_OVERFLOW))


def decode_peaks(peaks: torch.Tensor):
    """(max_absz float32 [nt], argmax int32 [nt]) from the RfPeak records."""
    p = peaks.cpu().contiguous()
    return p[:, 0].view(torch.float32).numpy().copy(), p[:, 1].numpy().copy()


def decode_triggers(trig: torch.Tensor, count: int):
    """List of (tmpl, seg, idx, absz, argz) for the first min(count, cap) records."""
    t = trig.cpu().contiguous()[: min(count, trig.shape[0])]
    ints = t[:, :3].numpy()
    fl = t[:, 3:].view(torch.float32).numpy()
    return [(int(a), int(b), int(c), float(d), float(e)) for (a, b, c), (d, e) in zip(ints, fl)]


class Batch:
    """rf_batch: nseg segments x len(refs) reference groups with their kernel
    sets, run as one captured graph with a persistent reconstruction launch.
    The context must enqueue on a non-default stream."""

    def __init__(self, ctx: Context, grid, psd: torch.Tensor, refs, ksets, nseg: int):
        self.ctx = ctx
        self.nseg = nseg
        self.nref = len(refs)
        self.n = int(grid.n)
        self.psd = psd                       # borrowed by the library: keep alive
        g = to_grid(grid)
        handles = (ctypes.c_void_p * len(ksets))(*[k.h.value for k in ksets])
        h = ctypes.c_void_p()
        ctx.check(ctx.lib.rf_batch_create(ctx.h, ctypes.byref(g), _ptr(psd), len(refs), _tmpl_array(refs),
                                          handles, int(nseg), ctypes.byref(h)))
        self.h = h
        self.ktotal = self.info()["ktotal"]

    def info(self):
        kt = ctypes.c_int32()
        ni = ctypes.c_int64()
        kb = (ctypes.c_int32 * self.nref)()
        ch = (ctypes.c_int32 * 3)()
        st = self.ctx.lib.rf_batch_info(self.h, ctypes.byref(kt), ctypes.byref(ni), kb, ch)
        self.ctx.check(st)
        return dict(ktotal=kt.value, nitems=ni.value, kbase=list(kb), chunks=list(ch))

    def set_chunks(self, chunks):
        arr = (ctypes.c_int32 * 3)(*chunks)
        st = self.ctx.lib.rf_batch_set_chunks(self.h, arr)
        if st != RF_OK:
            raise RfError(st, "rf_batch_set_chunks failed")

    def tuning(self):
        """Launch settings: chunk and blocks (per tile-length bucket), xcd_queues, bucket_hi."""
        t = RfBatchTuning()
        self.ctx.check(self.ctx.lib.rf_batch_get_tuning(self.h, ctypes.byref(t)))
        return dict(chunk=list(t.chunk), blocks=list(t.blocks), xcd_queues=int(t.xcd_queues),
                    bucket_hi=list(t.bucket_hi))

    def set_tuning(self, chunk=None, blocks=None, xcd_queues=None, bucket_hi=None):
        cur = self.tuning()
        t = RfBatchTuning()
        t.chunk = (ctypes.c_int32 * 3)(*(cur["chunk"] if chunk is None else chunk))
        t.blocks = (ctypes.c_int32 * 3)(*(cur["blocks"] if blocks is None else blocks))
        t.xcd_queues = int(cur["xcd_queues"] if xcd_queues is None else xcd_queues)
        t.bucket_hi = (ctypes.c_int64 * 2)(*(cur["bucket_hi"] if bucket_hi is None else bucket_hi))
        st = self.ctx.lib.rf_batch_set_tuning(self.h, ctypes.byref(t))
        if st != RF_OK:
            raise RfError(st, "rf_batch_set_tuning failed")

    def _inputs_ready(self, xf_segs):
        _dev_tensor(xf_segs, torch.complex128, shape=(self.nseg, self.n // 2 + 1), what="xf_segs")
        self.ctx.stream.wait_stream(torch.cuda.current_stream(xf_segs.device))

    def autotune(self, xf_segs: torch.Tensor, cache_path: str | None = None):
        self._inputs_ready(xf_segs)
        self.ctx.check(self.ctx.lib.rf_batch_autotune(self.ctx.h, self.h, _ptr(xf_segs),
                                                      cache_path.encode() if cache_path else None))
        return self.info()["chunks"]

    def run(self, xf_segs: torch.Tensor, thr: float, trig_cap: int = 1 << 16, peaks=None, trig=None):
        self._inputs_ready(xf_segs)
        dev = xf_segs.device
        if peaks is None:
            peaks = torch.empty((self.nseg, self.ktotal, 2), dtype=torch.int32, device=dev)
        if trig is None:
            trig = torch.empty((max(trig_cap, 1), 5), dtype=torch.int32, device=dev)
        _dev_tensor(peaks, torch.int32, numel=self.nseg * self.ktotal * 2, what="peaks")
        _dev_tensor(trig, torch.int32, what="trig")
        _require(trig.numel() >= 5 * trig_cap, "trig: needs room for trig_cap records")
        cnt = ctypes.c_int64(0)
        st = self.ctx.lib.rf_batch_run(self.ctx.h, self.h, _ptr(xf_segs), ctypes.c_float(thr), _ptr(peaks),
                                       _ptr(trig), int(trig_cap), ctypes.byref(cnt))
        if st not in (RF_OK, RF_E_OVERFLOW):
            self.ctx.check(st)
        return dict(peaks=peaks, trig=trig, ntrig=int(cnt.value), overflow=(st == RF_E_OVERFLOW))

    def graph_stats(self):
        """(captures, replays) of the batch's graphs since creation."""
        c, r = ctypes.c_int64(), ctypes.c_int64()
        self.ctx.check(self.ctx.lib.rf_batch_graph_stats(self.h, ctypes.byref(c), ctypes.byref(r), None))
        return c.value, r.value

    def last_recon_ms(self):
        """Duration of the last run's reconstruction graph (HIP events on the batch's stream)."""
        ms = ctypes.c_float()
        self.ctx.check(self.ctx.lib.rf_batch_graph_stats(self.h, None, None, ctypes.byref(ms)))
        return ms.value

    def free(self):
        if getattr(self, "h", None):
            self.ctx.lib.rf_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


N_MLP_PARAMS = 165760


class Surrogate:
    """rf_surrogate: SVD basis of exact analytic kernels + MLP (trained on the
    GPU by the library's own kernels).  The context must use a non-default
    stream for training (graph capture)."""

    def __init__(self, ctx: Context, grid, refs, nbrs, window: int, omega: torch.Tensor, rank: int = 64):
        self.ctx = ctx
        self.grid = grid
        _dev_tensor(omega, torch.float64, what="omega")
        _require(omega.dim() == 2 and omega.shape[0] == len(refs) == len(nbrs),
                 "omega: expected [npair, nomega] with one row per training pair")
        g = to_grid(grid)
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        ctx.check(ctx.lib.rf_surrogate_create(ctx.h, ctypes.byref(g), _tmpl_array(refs), _tmpl_array(nbrs),
                                              len(refs), int(window), int(rank), _ptr(omega), int(omega.shape[1]),
                                              ctypes.byref(h)))
        self.h = h
        self.rank = rank
        self.npair = len(refs)

    def info(self):
        w, r, kr = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        sc, st = ctypes.c_double(), ctypes.c_int64()
        self.ctx.check(self.ctx.lib.rf_surrogate_info(self.h, ctypes.byref(w), ctypes.byref(r), ctypes.byref(kr),
                                                      None, ctypes.byref(sc), ctypes.byref(st)))
        sv = (ctypes.c_double * max(kr.value, 1))()
        self.ctx.check(self.ctx.lib.rf_surrogate_info(self.h, None, None, None, sv, None, None))
        return dict(window=w.value, rank=r.value, numerical_rank=kr.value, svals=list(sv)[:kr.value],
                    out_scale=sc.value, steps=st.value)

    def set_params(self, theta: torch.Tensor):
        _dev_tensor(theta, torch.float32, N_MLP_PARAMS, what="theta")
        torch.cuda.synchronize()
        self.ctx.check(self.ctx.lib.rf_surrogate_set_params(self.ctx.h, self.h, _ptr(theta)))

    def get_params(self) -> torch.Tensor:
        out = torch.empty(N_MLP_PARAMS, dtype=torch.float32, device=f"cuda:{self.ctx.device}")
        torch.cuda.synchronize()
        self.ctx.check(self.ctx.lib.rf_surrogate_get_params(self.ctx.h, self.h, _ptr(out)))
        return out

    def dataset(self):
        """(x [npair, 4], t [npair, 128]) float32 device copies of the training rows."""
        dev = f"cuda:{self.ctx.device}"
        x = torch.empty((self.npair, 4), dtype=torch.float32, device=dev)
        t = torch.empty((self.npair, 2 * self.rank), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        self.ctx.check(self.ctx.lib.rf_surrogate_dataset(self.ctx.h, self.h, _ptr(x), _ptr(t)))
        return x, t

    def grad(self, x: torch.Tensor, t: torch.Tensor):
        _dev_tensor(x, torch.float32, what="x")
        _require(x.dim() == 2 and x.shape[1] == 4, "x: expected [rows, 4]")
        rows = x.shape[0]
        _dev_tensor(t, torch.float32, shape=(rows, 2 * self.rank), what="t")
        g = torch.empty(N_MLP_PARAMS, dtype=torch.float32, device=x.device)
        loss = ctypes.c_float()
        torch.cuda.synchronize()
        self.ctx.check(self.ctx.lib.rf_surrogate_grad(self.ctx.h, self.h, _ptr(x), _ptr(t), rows,
                                                      ctypes.byref(loss), _ptr(g)))
        return loss.value, g

    def train(self, order: torch.Tensor, lr: float):
        _dev_tensor(order, torch.int32, what="order")
        _require(order.dim() == 2, "order: expected [steps, batch]")
        steps, batch = order.shape
        _require(steps >= 1 and batch >= 1, "order: empty")
        lo, hi = int(order.min().item()), int(order.max().item())
        _require(0 <= lo and hi < self.npair, f"order: rows must lie in [0, {self.npair})")
        hist = (ctypes.c_float * steps)()
        torch.cuda.synchronize()
        self.ctx.check(self.ctx.lib.rf_surrogate_train(self.ctx.h, self.h, _ptr(order), steps, batch, float(lr), hist))
        return list(hist)

    def predict(self, ref, nbrs):
        c = torch.empty((len(nbrs), self.rank), dtype=torch.complex128, device=f"cuda:{self.ctx.device}")
        self.ctx.check(self.ctx.lib.rf_surrogate_predict(self.ctx.h, self.h, RfTmpl(*map(float, ref)),
                                                         _tmpl_array(nbrs), len(nbrs), _ptr(c)))
        return c

    def project(self, ref, nbrs):
        c = torch.empty((len(nbrs), self.rank), dtype=torch.complex128, device=f"cuda:{self.ctx.device}")
        self.ctx.check(self.ctx.lib.rf_surrogate_project(self.ctx.h, self.h, RfTmpl(*map(float, ref)),
                                                         _tmpl_array(nbrs), len(nbrs), _ptr(c)))
        return c

    def encode(self, ref, nbrs, bits: int = 16, network: bool = True):
        """Residual codes of the exact coefficients against the network's
        prediction (network=False: plain codes): (codes int8/int16 [nk, 2 rank],
        scales float32 [nk]) on the device."""
        _require(bits in (8, 16), "bits must be 8 or 16")
        dev = f"cuda:{self.ctx.device}"
        codes = torch.empty((len(nbrs), 2 * self.rank), dtype=torch.int8 if bits == 8 else torch.int16, device=dev)
        scales = torch.empty(len(nbrs), dtype=torch.float32, device=dev)
        torch.cuda.synchronize()
        self.ctx.check(self.ctx.lib.rf_surrogate_encode(self.ctx.h, self.h, RfTmpl(*map(float, ref)), _tmpl_array(nbrs),
                                                        len(nbrs), int(bits), int(bool(network)), _ptr(codes),
                                                        _ptr(scales)))
        return codes, scales

    def decode(self, ref, nbrs, codes: torch.Tensor, scales: torch.Tensor, network: bool = True):
        """Coefficients (complex128 [nk, rank], device) from residual codes."""
        bits = 8 if codes.dtype == torch.int8 else 16
        _dev_tensor(codes, torch.int8 if bits == 8 else torch.int16, shape=(len(nbrs), 2 * self.rank), what="codes")
        _dev_tensor(scales, torch.float32, len(nbrs), what="scales")
        c = torch.empty((len(nbrs), self.rank), dtype=torch.complex128, device=f"cuda:{self.ctx.device}")
        torch.cuda.synchronize()
        self.ctx.check(self.ctx.lib.rf_surrogate_decode(self.ctx.h, self.h, RfTmpl(*map(float, ref)), _tmpl_array(nbrs),
                                                        len(nbrs), bits, int(bool(network)), _ptr(codes), _ptr(scales),
                                                        _ptr(c)))
        return c

    def kernels(self, grid, psd, ref, nbrs, coeffs=None, thr=1e-3, unit=RF_THR_PER_SECOND, check=None, tol=2e-4):
        """Kernel set from the surrogate (network coefficients unless `coeffs`);
        check = (grid, xf, psd) of a check segment."""
        nk = len(nbrs)
        _dev_tensor(psd, torch.float64, int(grid.n) // 2 + 1, what="psd")
        if coeffs is not None:
            _dev_tensor(coeffs, torch.complex128, shape=(nk, self.rank), what="coeffs")
        if check:
            nc = int(check[0].n)
            _dev_tensor(check[1], torch.complex128, nc // 2 + 1, what="check xf")
            _dev_tensor(check[2], torch.float64, nc // 2 + 1, what="check psd")
        g = to_grid(grid)
        fb = (ctypes.c_int32 * nk)()
        err = (ctypes.c_float * nk)()
        h = ctypes.c_void_p()
        cg = to_grid(check[0]) if check else None
        torch.cuda.synchronize()
        self.ctx.check(self.ctx.lib.rf_surrogate_kernels(
            self.ctx.h, self.h, ctypes.byref(g), _ptr(psd), RfTmpl(*map(float, ref)), _tmpl_array(nbrs), nk,
            _ptr(coeffs) if coeffs is not None else None, float(thr), int(unit), ctypes.byref(cg) if check else None, _ptr(check[1]) if check else None,
            _ptr(check[2]) if check else None, float(tol), ctypes.byref(h), fb, err))
        return Kernels(self.ctx, h, nk), list(fb), list(err)

    def free(self):
        if getattr(self, "h", None):
            self.ctx.lib.rf_surrogate_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def factored_batch(ctx: Context, grid, xf_segs: torch.Tensor, psd: torch.Tensor, sets, refs, thr: float,
                   trig_cap: int = 1 << 16, prec: str = "split16"):
    """snr_reconstruct_factored_batch: every (segment, set) pair's reference matched
    filter and factored reconstruction with the fused read-out, one synchronisation.
    peaks [nseg, ktot, 2] int32 (RfPeak bytes; set r's kernels from the sum of the
    earlier sets' counts), triggers, count."""
    n = int(grid.n)
    _dev_tensor(xf_segs, torch.complex128, what="xf_segs")
    _require(xf_segs.dim() == 2 and xf_segs.shape[1] == n // 2 + 1, "xf_segs: expected [nseg, n/2+1]")
    _dev_tensor(psd, torch.float64, n // 2 + 1, what="psd")
    _require(len(sets) == len(refs) and len(sets) >= 1, "sets and refs: one reference per set")
    nseg = int(xf_segs.shape[0])
    ktot = sum(F.nk for F in sets)
    peaks = torch.empty((nseg, ktot, 2), dtype=torch.int32, device=xf_segs.device)
    trig = torch.empty((max(trig_cap, 1), 5), dtype=torch.int32, device=xf_segs.device)
    cnt = ctypes.c_int64(0)
    args = RfPeakArgs(float(thr), peaks.data_ptr(), trig.data_ptr(), int(trig_cap), ctypes.pointer(cnt))
    handles = (ctypes.c_void_p * len(sets))(*[F.h.value for F in sets])
    g = to_grid(grid)
    st = ctx.lib.snr_reconstruct_factored_batch(ctx.h, ctypes.byref(g), _ptr(xf_segs), nseg, _ptr(psd), len(sets),
                                                handles, _tmpl_array(refs), PREC[prec], ctypes.byref(args))
    if st not in (RF_OK, RF_E_OVERFLOW):
        ctx.check(st)
    return dict(peaks=peaks, trig=trig, ntrig=int(cnt.value), overflow=(st == RF_E_OVERFLOW))


class Factored:
    """rf_factored: a kernel set's leading basis for series of grid.n samples."""

    def __init__(self, ctx: Context, kernels: Kernels, grid, tol: float = 2e-6, jmax: int = 128):
        self.ctx = ctx
        self.nk = kernels.nk
        g = to_grid(grid)
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        ctx.check(ctx.lib.rf_factored_build(ctx.h, kernels.h, ctypes.byref(g), float(tol), int(jmax),
                                            ctypes.byref(h)))
        self.h = h

    def info(self):
        j = ctypes.c_int32()
        m0, ln = ctypes.c_int64(), ctypes.c_int64()
        lam = (ctypes.c_double * self.nk)()
        res = (ctypes.c_double * self.nk)()
        self.ctx.check(self.ctx.lib.rf_factored_info(self.h, ctypes.byref(j), ctypes.byref(m0), ctypes.byref(ln),
                                                     lam, res))
        return dict(J=j.value, m0=m0.value, len=ln.value, lam=list(lam), resid=list(res))

    def reconstruct(self, z_ref: torch.Tensor, z_out=None, store: bool = True, fused_thr: float | None = None,
                    trig_cap: int = 4096, prec: str = "split16"):
        _dev_tensor(z_ref, torch.complex64, what="z_ref")
        n = z_ref.numel()
        if store and z_out is None:
            z_out = torch.empty((self.nk, n), dtype=torch.complex64, device=z_ref.device)
        if store:
            _dev_tensor(z_out, torch.complex64, shape=(self.nk, n), what="z_out")
        fused = None
        peaks = trig = None
        cnt = ctypes.c_int64(0)
        if fused_thr is not None:
            peaks = torch.empty((self.nk, 2), dtype=torch.int32, device=z_ref.device)
            trig = torch.empty((max(trig_cap, 1), 5), dtype=torch.int32, device=z_ref.device)
            fused = RfPeakArgs(float(fused_thr), peaks.data_ptr(), trig.data_ptr(), int(trig_cap),
                               ctypes.pointer(cnt))
        st = self.ctx.lib.snr_reconstruct_factored(self.ctx.h, self.h, _ptr(z_ref), n, PREC[prec],
                                                   _ptr(z_out) if store else None,
                                                   ctypes.byref(fused) if fused is not None else None)
        if st not in (RF_OK, RF_E_OVERFLOW):
            self.ctx.check(st)
        out = dict(z=z_out if store else None)
        if fused is not None:
            out.update(peaks=peaks, trig=trig, ntrig=int(cnt.value), overflow=(st == RF_E_OVERFLOW))
        return out

    def free(self):
        if getattr(self, "h", None):
            self.ctx.lib.rf_factored_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Ols:
    """rf_ols: blocked frequency-domain (overlap-save) plan of a kernel set for
    series of n samples."""

    def __init__(self, ctx: Context, kernels: Kernels, n: int):
        self.ctx = ctx
        self.nk = kernels.nk
        self.n = int(n)
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        ctx.check(ctx.lib.rf_ols_build(ctx.h, kernels.h, self.n, ctypes.byref(h)))
        self.h = h

    def info(self):
        b, hop, pmax = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        parts = (ctypes.c_int32 * self.nk)()
        nbytes = ctypes.c_int64()
        self.ctx.check(self.ctx.lib.rf_ols_info(self.h, ctypes.byref(b), ctypes.byref(hop), ctypes.byref(pmax), parts,
                                                ctypes.byref(nbytes)))
        return dict(block=b.value, hop=hop.value, pmax=pmax.value, parts=list(parts), spectra_bytes=nbytes.value)

    def reconstruct(self, z_ref: torch.Tensor, z_out=None, store: bool = True, fused_thr: float | None = None,
                    trig_cap: int = 4096):
        _dev_tensor(z_ref, torch.complex64, what="z_ref")
        n = z_ref.numel()
        if store and z_out is None:
            z_out = torch.empty((self.nk, n), dtype=torch.complex64, device=z_ref.device)
        if store:
            _dev_tensor(z_out, torch.complex64, shape=(self.nk, n), what="z_out")
        fused = None
        peaks = trig = None
        cnt = ctypes.c_int64(0)
        if fused_thr is not None:
            peaks = torch.empty((self.nk, 2), dtype=torch.int32, device=z_ref.device)
            trig = torch.empty((max(trig_cap, 1), 5), dtype=torch.int32, device=z_ref.device)
            fused = RfPeakArgs(float(fused_thr), peaks.data_ptr(), trig.data_ptr(), int(trig_cap),
                               ctypes.pointer(cnt))
        st = self.ctx.lib.snr_reconstruct_ols(self.ctx.h, self.h, _ptr(z_ref), n, _ptr(z_out) if store else None,
                                              ctypes.byref(fused) if fused is not None else None)
        if st not in (RF_OK, RF_E_OVERFLOW):
            self.ctx.check(st)
        out = dict(z=z_out if store else None)
        if fused is not None:
            out.update(peaks=peaks, trig=trig, ntrig=int(cnt.value), overflow=(st == RF_E_OVERFLOW))
        return out

    def free(self):
        if getattr(self, "h", None):
            self.ctx.lib.rf_ols_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def template_durations(bank, f_low: float):
    """tau(f_low) of each (m1, m2) (host computation in the library)."""
    import numpy as np
    lib = load()
    n = len(bank)
    arr = (RfTmpl * max(n, 1))(*[RfTmpl(float(a), float(b)) for a, b in bank])
    out = np.zeros(n, dtype=np.float64)
    st = lib.rf_template_durations(arr, n, float(f_low), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    if st != RF_OK:
        raise RfError(st, "rf_template_durations failed")
    return out


def bank_organise(bank, tau, max_spread: float = 10.0, max_size: int = 500):
    """(group of each template, reference index of each group) from the library."""
    import numpy as np
    lib = load()
    n = len(bank)
    arr = (RfTmpl * max(n, 1))(*[RfTmpl(float(a), float(b)) for a, b in bank])
    tau = np.ascontiguousarray(tau, dtype=np.float64)
    group = np.zeros(n, dtype=np.int32)
    ref = np.zeros(max(n, 1), dtype=np.int64)
    ng = ctypes.c_int32()
    st = lib.rf_bank_organise(arr, tau.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n, float(max_spread),
                              int(max_size), group.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              ref.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(ng))
    if st != RF_OK:
        raise RfError(st, "rf_bank_organise failed")
    return group, ref[:ng.value].copy()
