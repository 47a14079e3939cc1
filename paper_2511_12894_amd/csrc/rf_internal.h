// Internal declarations of librf (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/rf.h"

namespace rf {

// ------------------------------------------------------------------ errors
struct Error {
  rf_status code;
  std::string msg;
};

#define RF_HIP(call)                                                            \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess)                                                       \
      throw ::rf::Error{RF_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define RF_CHECK(cond, msg)                                                     \
  do {                                                                          \
    if (!(cond)) throw ::rf::Error{RF_E_INVAL, (msg)};                          \
  } while (0)

// ------------------------------------------------------------------ device buffers
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void release();
  void* ensure(size_t n);  // grows, contents not preserved
};

}  // namespace rf

struct rf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string last_error;
  // workspace slots
  rf::DevBuf ws[16];
  std::vector<char> host_stage[16];
  hipEvent_t ev = nullptr;
};

namespace rf {

// Run f for an entry point: errors become the returned status, their message
// the context's last error.
template <typename F>
rf_status guarded(rf_ctx* ctx, F&& f) {
  try {
    if (ctx) {
      hipError_t e = hipSetDevice(ctx->device);
      if (e != hipSuccess) throw Error{RF_E_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e)};
    }
    f();
    return RF_OK;
  } catch (const Error& e) {
    if (ctx) ctx->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    if (ctx) ctx->last_error = "host allocation failed";
    return RF_E_NOMEM;
  } catch (...) {
    if (ctx) ctx->last_error = "unexpected exception";
    return RF_E_HIP;
  }
}

// Device allocation of `count` elements (at least one); RF_E_NOMEM on failure.
template <typename T>
T* dev_alloc(size_t count, const char* what = "device allocation failed") {
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(T) * (count > 0 ? count : 1)) != hipSuccess) {
    (void)hipGetLastError();
    throw Error{RF_E_NOMEM, what};
  }
  return static_cast<T*>(p);
}

// Copy on the context's stream (which need not synchronise with the null
// stream) and wait for it.
void copy_sync(rf_ctx* ctx, void* dst, const void* src, size_t bytes, hipMemcpyKind kind);

enum WsSlot {
  WS_FFT_A = 0, WS_FFT_B = 1, WS_RED = 2, WS_SPLIT = 3, WS_PEAK = 4, WS_COEF = 5, WS_BUILD = 6,
  WS_Y = 7, WS_SCALAR = 8, WS_SCAN = 9, WS_TGT = 10, WS_ZREF = 11
};

inline bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }
inline int ilog2(int64_t n) {
  int l = 0;
  while ((int64_t(1) << l) < n) ++l;
  return l;
}

void validate_grid(const rf_grid* g);

// ------------------------------------------------------------------ TaylorF2 (host)
// Per-template constants of the stationary-phase phase series, in the form
// Psi(f) = -pi/4 + pref * v^-5 * [1 + v^2 (a2 + v (a3 + v (a4 + v ((a5c + a5l ln v)
//          + v ((a6c + a6l ln v) + v a7)))))],  v = (pi M f)^(1/3).
struct Tf2Coef {
  double piM;      // pi * M  [s]
  double pref;     // 3 / (128 eta)
  double a2, a3, a4, a5c, a5l, a6c, a6l, a7;
  double amp;      // Mc^(5/6)
  double cbrt_piM; // (pi M)^(1/3)
  double ln_cbrt_piM, inv_cbrt_piM;   // ln and reciprocal of (pi M)^(1/3)
  // the same phase in powers of x = f^(1/3) and ln f (v = (pi M)^(1/3) x):
  // Psi = e0 + e5 x^-5 + e3 x^-3 + e2 x^-2 + e1 x^-1 + el ln f + ex x + exl x ln f + exx x^2
  double e0, e5, e3, e2, e1, el, ex, exl, exx;
};
Tf2Coef tf2_coef(const rf_tmpl& t);

// Psi at v = (pi M f)^(1/3) with lv = ln v and iv = 1 / v supplied, FP64 (the
// phase reaches ~1e5 rad in band).
__device__ inline double tf2_phase_v(const Tf2Coef& c, double v, double lv, double iv) {
  const double v2 = v * v;
  const double iv5 = iv * iv * iv * iv * iv;
  const double poly =
      1.0 + v2 * (c.a2 + v * (c.a3 + v * (c.a4 + v * ((c.a5c + c.a5l * lv) +
                                                       v * ((c.a6c + c.a6l * lv) + v * c.a7)))));
  return -0.25 * 3.14159265358979323846 + c.pref * poly * iv5;
}
__device__ inline double tf2_phase(const Tf2Coef& c, double v) { return tf2_phase_v(c, v, log(v), 1.0 / v); }
double tf2_dtdf(const Tf2Coef& c, double f);   // t'(f) = Psi''(f) / (2 pi)
double tf2_t(const Tf2Coef& c, double f);      // t(f)  = Psi'(f) / (2 pi)

// ------------------------------------------------------------------ launchers
// Inverse (exp +) unnormalised complex DFT of `batch` contiguous series of n
// points, in -> out (out may not alias in).  Uses ctx workspace slots A/B.
// wsa/wsb: caller-owned scratch of n * batch elements each (both NULL: the
// context's growable workspace, which a captured graph must not reference).
void fft_inverse_f32(rf_ctx* ctx, const float2* in, float2* out, int64_t n, int batch,
                     float2* wsa = nullptr, float2* wsb = nullptr);
void fft_inverse_f64(rf_ctx* ctx, const double2* in, double2* out, int64_t n, int batch);
// The same (FP32) for `batch` inputs formed on the fly, input y being
// conj(Q[f]) Ub[y][f - b0] * inv_n on the bins f in [b0, b0 + nb) and zero
// elsewhere (Ub: [batch][nb]); nothing else is read.
void fft_inverse_band_f32(rf_ctx* ctx, const float2* Q, const float2* Ub, int64_t b0, int64_t nb, float inv_n,
                          float2* out, int64_t n, int batch);

// Matched-filter series of `batch` templates, the first pass forming its input on
// the fly (the template spectrum is never stored): input y is
// sqrt(4 df / I) f^(-7/6) q[y / nt][f - jlo] exp(+i Psi_t(f)) on the band bins
// f in [jlo, jhi] and zero elsewhere, with t = y % nt, coef[t] its phase series
// and I = *moment; q: [batch / nt][jhi - jlo + 1] (condition_data).
void fft_inverse_tmpl_f32(rf_ctx* ctx, const rf_grid* g, const float2* q, const Tf2Coef* coef, int nt,
                          const double* moment, float2* out, int batch, float2* wsa = nullptr,
                          float2* wsb = nullptr);
// Conditioned data q[seg][j - jlo] = x~_j / S_j on the band bins (FP64
// arithmetic, complex64 store) for nseg segments (xf: [nseg][n/2+1]).
void condition_data(rf_ctx* ctx, const rf_grid* g, const double2* xf, const double* psd, float2* q,
                    int nseg = 1);

// sum over the band of f^(-7/3) / S(f) -> *moment (device double), FP64, fixed order
void band_moment(rf_ctx* ctx, const rf_grid* g, const double* psd, double* moment);
// band bins j with f_low <= j fs / n <= f_high: [jlo, jhi]
void band_limits(const rf_grid* g, int64_t* jlo, int64_t* jhi);


// One-sided ratio spectra for nb-point kernels, nk targets (FP64), scaled by c_j / nb.
struct RatioParam {
  double amp_ratio;   // (Mc_k / Mc_ref)^(5/6)
  double df_low;      // lower taper width
};
void ratio_spectrum(rf_ctx* ctx, const rf_grid* g, int64_t nb, const Tf2Coef* ref_dev,
                    const Tf2Coef* tgt_dev, const RatioParam* par_dev, double2* out, int nk);

// support scan on the real parts of nk complex series of nb points
void support_scan(rf_ctx* ctx, const double2* w, int64_t nb, int nk, double thr_tap,
                  int32_t* lo, int32_t* hi, uint32_t* maxabs_bits);

// copy taps Re(w[(m_lo + l) mod nb]), l < len, into dst (contiguous per kernel)
void gather_taps(rf_ctx* ctx, const double2* w, int64_t nb, int nk, const int64_t* off_dev,
                 const int32_t* mlo_dev, const int32_t* len_dev, double* dst);

// generic fill (graph-safe replacement for memset)
void fill_u64(rf_ctx* ctx, uint64_t* p, uint64_t v, int64_t n);
void fill_u32(rf_ctx* ctx, uint32_t* p, uint32_t v, int64_t n);

}  // namespace rf
struct rf_kernels;
namespace rf {
void finalize_kernel_set(rf_ctx* ctx, rf_kernels* K, const std::vector<double>& taps_host);
void free_kernel_set(rf_kernels* k);

}  // namespace rf

// ------------------------------------------------------------------ kernel set
namespace rf {
struct TileDev {
  int64_t m0;       // first tap (signed) of the tile's union support
  int64_t ksteps;   // 16-tap steps covering it
  int64_t b32_off;  // offsets of the tile in the packed operand buffers
  int64_t b16_off;
  int64_t gflag_off; // offset of the tile's granule flags (one per 256 taps; bit 1 corrections, bit 2 folds)
  int32_t first;    // first slot of the tile in the slot arrays
  int32_t count;    // live kernels in the tile
  int32_t pair;     // 1: at most 16 kernels, operand columns 16..31 repeating columns 0..15
                    // 32 taps later (their outputs are 32 times later), so one 32 x 32
                    // product per plane covers a wave's 64 output times
  int32_t pad;
};
}  // namespace rf

struct rf_kernels {
  int device = 0;
  int32_t nk = 0;
  int64_t n_build = 0;
  double fs = 0;
  std::vector<int64_t> m_lo;         // signed first tap of each kernel
  std::vector<int32_t> len;          // taps kept
  std::vector<int64_t> off;          // offset of each kernel's taps in taps64
  std::vector<double> norm_ratio;    // N_ref / N_k
  std::vector<double> df_low;        // lower taper width used
  std::vector<double> kscale;        // power-of-two FP16 scale s_k
  double* taps64 = nullptr;          // device, concatenated FP64 taps
  int64_t total_taps = 0;
  // reconstruction tiles (kernels sorted by first tap, 32 per tile)
  std::vector<rf::TileDev> tiles;
  int64_t max_ksteps = 0;
  rf::TileDev* tiles_dev = nullptr;
  float* b32 = nullptr;              // FP32 operand fragments
  __half* b16 = nullptr;             // FP16 hi/lo operand fragments
  float* colscale32 = nullptr;       // per slot: N_ref / N_k
  float* colscale16 = nullptr;       // per slot: N_ref / N_k / s_k
  int32_t* slot_kernel = nullptr;    // per slot: kernel index (-1 empty)
  // per tile and 256-tap granule: 1 if some kernel of the tile has a tap there of at
  // least half an FP16 unit after its scale s_k (|w| s_k >= 1/2, i.e. above 2^-15..2^-14
  // of its largest tap), else 0; the split form's correction products are skipped in
  // window chunks without such a granule
  uint32_t* gflag = nullptr;
  int64_t gflag_total = 0;
};
