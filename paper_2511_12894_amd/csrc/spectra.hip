// FP64 frequency-domain work: the TaylorF2 phase coefficients (the template
// spectra themselves are formed inside the first transform pass of the matched
// filter), data conditioning x~ / S and the band moment for the template norms
// (section II.A), windowed ratio spectra (sections II.B-II.C), and the kernel
// support scan and tap gather of the truncation (section II.D).
#include <algorithm>
#include <cmath>

#include "rf_internal.h"

namespace rf {

// ---------------------------------------------------------------- host side

namespace {
constexpr double kTsun = 4.925490947641267e-6;  // G M_sun / c^3 [s]
constexpr double kPi = 3.14159265358979323846;
constexpr double kEuler = 0.57721566490153286061;
}  // namespace

// Non-spinning TaylorF2 phase series to 3.5PN (the paper's TaylorF2 model,
// sections II.B and III.B; stationary-phase form of appendix A), coefficients
// written as rationals in eta with t_c = phi_c = 0.
Tf2Coef tf2_coef(const rf_tmpl& t) {
  Tf2Coef c{};
  const double m = (t.m1 + t.m2) * kTsun;
  const double eta = t.m1 * t.m2 / ((t.m1 + t.m2) * (t.m1 + t.m2));
  const double mc = m * std::pow(eta, 0.6);
  const double e2 = eta * eta, e3 = e2 * eta;
  c.piM = kPi * m;
  c.pref = 3.0 / (128.0 * eta);
  c.a2 = 3715.0 / 756.0 + 55.0 / 9.0 * eta;
  c.a3 = -16.0 * kPi;
  c.a4 = 15293365.0 / 508032.0 + 27145.0 / 504.0 * eta + 3085.0 / 72.0 * e2;
  const double a5 = kPi * (38645.0 / 756.0 - 65.0 / 9.0 * eta);
  // a5 (1 + 3 ln(v / v_lso)), v_lso = 6^(-1/2)
  c.a5c = a5 * (1.0 + 1.5 * std::log(6.0));
  c.a5l = 3.0 * a5;
  // psi_6 = const - 6848/21 ln(4 v)
  c.a6l = -6848.0 / 21.0;
  c.a6c = 11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * kPi * kPi - 6848.0 / 21.0 * kEuler +
          (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * kPi * kPi) * eta + 76055.0 / 1728.0 * e2 -
          127825.0 / 1296.0 * e3 + c.a6l * std::log(4.0);
  c.a7 = kPi * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta - 74045.0 / 756.0 * e2);
  c.amp = std::pow(mc, 5.0 / 6.0);
  c.cbrt_piM = std::cbrt(c.piM);
  c.ln_cbrt_piM = std::log(c.cbrt_piM);
  c.inv_cbrt_piM = 1.0 / c.cbrt_piM;
  // pref [v^-5 + a2 v^-3 + a3 v^-2 + a4 v^-1 + (a5c + a5l ln v) + (a6c + a6l ln v) v + a7 v^2]
  // with v = k x, ln v = ln k + ln(f) / 3
  const double k = c.cbrt_piM, lk = c.ln_cbrt_piM, ik = c.inv_cbrt_piM;
  c.e0 = -0.25 * kPi + c.pref * (c.a5c + c.a5l * lk);
  c.e5 = c.pref * ik * ik * ik * ik * ik;
  c.e3 = c.pref * c.a2 * ik * ik * ik;
  c.e2 = c.pref * c.a3 * ik * ik;
  c.e1 = c.pref * c.a4 * ik;
  c.el = c.pref * c.a5l / 3.0;
  c.ex = c.pref * (c.a6c + c.a6l * lk) * k;
  c.exl = c.pref * c.a6l * k / 3.0;
  c.exx = c.pref * c.a7 * k * k;
  return c;
}

namespace {
// P(v) = pref [v^-5 + a2 v^-3 + a3 v^-2 + a4 v^-1 + (a5c + a5l ln v) + (a6c + a6l ln v) v + a7 v^2]
void series_derivs(const Tf2Coef& c, double v, double* d1, double* d2) {
  const double lv = std::log(v);
  const double iv = 1.0 / v;
  const double iv2 = iv * iv, iv3 = iv2 * iv, iv4 = iv3 * iv, iv5 = iv4 * iv, iv6 = iv5 * iv,
               iv7 = iv6 * iv;
  *d1 = c.pref * (-5.0 * iv6 - 3.0 * c.a2 * iv4 - 2.0 * c.a3 * iv3 - c.a4 * iv2 + c.a5l * iv +
                  (c.a6c + c.a6l * lv + c.a6l) + 2.0 * c.a7 * v);
  *d2 = c.pref * (30.0 * iv7 + 12.0 * c.a2 * iv5 + 6.0 * c.a3 * iv4 + 2.0 * c.a4 * iv3 -
                  c.a5l * iv2 + c.a6l * iv + 2.0 * c.a7);
}
}  // namespace

double tf2_t(const Tf2Coef& c, double f) {
  const double v = std::cbrt(c.piM * f);
  double d1, d2;
  series_derivs(c, v, &d1, &d2);
  return d1 * (v / (3.0 * f)) / (2.0 * kPi);
}

double tf2_dtdf(const Tf2Coef& c, double f) {
  const double v = std::cbrt(c.piM * f);
  double d1, d2;
  series_derivs(c, v, &d1, &d2);
  const double dv = v / (3.0 * f);
  const double d2v = -2.0 * v / (9.0 * f * f);
  return (d2 * dv * dv + d1 * d2v) / (2.0 * kPi);
}

// ---------------------------------------------------------------- device side

namespace {


constexpr int kRedThreads = 256;
constexpr int kRedBlocks = 1024;

// Partial sums of f^(-7/3) / S(f) over the band, one per block (grid-stride),
// then a single-block fixed-order sum: deterministic.
__global__ __launch_bounds__(kRedThreads) void k_moment_partial(const double* __restrict__ psd,
                                                                int64_t jlo, int64_t jhi,
                                                                double df, double* partial) {
  __shared__ double sh[kRedThreads];
  double acc = 0.0;
  for (int64_t j = jlo + int64_t(blockIdx.x) * kRedThreads + threadIdx.x; j <= jhi;
       j += int64_t(gridDim.x) * kRedThreads) {
    const double f = double(j) * df;
    const double cf = cbrt(f);
    acc += 1.0 / (f * f * cf * psd[j]);   // f^(-7/3) / S
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kRedThreads) void k_sum_partials(const double* __restrict__ partial,
                                                              int np, double* out) {
  __shared__ double sh[kRedThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += kRedThreads) acc += partial[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kRedThreads / 2; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// q[seg][j - jlo] = x~_j / S_j on the band bins (the data conditioning of
// section II.A, shared by every template filtered against the segment).
__global__ __launch_bounds__(256) void k_condition(const double2* __restrict__ xf,
                                                   const double* __restrict__ psd, float2* q,
                                                   int64_t n, int64_t jlo, int64_t nb) {
  xf += int64_t(blockIdx.y) * (n / 2 + 1);
  q += int64_t(blockIdx.y) * nb;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nb;
       i += int64_t(gridDim.x) * blockDim.x) {
    const double2 x = xf[jlo + i];
    const double s = 1.0 / psd[jlo + i];
    q[i] = make_float2(float(x.x * s), float(x.y * s));
  }
}

// One-sided ratio spectrum on nb points: A_j = c_j / nb * W(f_j) R e^{-i dPsi(f_j)}
// for j <= nb/2 (c_0 = c_{nb/2} = 1, else 2), 0 for j > nb/2; Re of its
// exp(+) DFT is the inverse real DFT of R~.
__global__ __launch_bounds__(256) void k_ratio_spectrum(const Tf2Coef* __restrict__ refc,
                                                        const Tf2Coef* __restrict__ tgtc,
                                                        const RatioParam* __restrict__ par,
                                                        double2* out, int64_t nb, double dfb,
                                                        double f_low, double f_high, double df_high) {
  const Tf2Coef cr = *refc;
  const Tf2Coef ct = tgtc[blockIdx.y];
  const RatioParam p = par[blockIdx.y];
  double2* o = out + int64_t(blockIdx.y) * nb;
  const double lo_edge = f_low - p.df_low, hi_edge = f_high + df_high;
  for (int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < nb;
       j += int64_t(gridDim.x) * blockDim.x) {
    double2 r = make_double2(0.0, 0.0);
    const double f = double(j) * dfb;
    if (j <= nb / 2 && f > lo_edge && f < hi_edge) {
      double w;
      if (f < f_low)
        w = 0.5 * (1.0 + cospi((f - f_low) / p.df_low));
      else if (f <= f_high)
        w = 1.0;
      else
        w = 0.5 * (1.0 - cospi((f - hi_edge) / df_high));
      const double cbf = cbrt(f);
      const double dpsi = tf2_phase(ct, ct.cbrt_piM * cbf) - tf2_phase(cr, cr.cbrt_piM * cbf);
      double sn, cs;
      sincos(dpsi, &sn, &cs);
      const double cj = (j == 0 || j == nb / 2) ? 1.0 : 2.0;
      const double a = cj / double(nb) * w * p.amp_ratio;
      r.x = a * cs;
      r.y = -a * sn;
    }
    o[j] = r;
  }
}

// Signed support of |Re w| >= thr and max |Re w| per series (blockIdx.y).
__global__ __launch_bounds__(256) void k_support_scan(const double2* __restrict__ w, int64_t nb,
                                                      double thr, int32_t* lo, int32_t* hi,
                                                      uint32_t* maxbits) {
  const double2* x = w + int64_t(blockIdx.y) * nb;
  int32_t mlo = INT32_MAX, mhi = INT32_MIN;
  float mx = 0.f;
  for (int64_t m = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; m < nb;
       m += int64_t(gridDim.x) * blockDim.x) {
    const double a = fabs(x[m].x);
    mx = fmaxf(mx, float(a));
    if (a >= thr) {
      const int32_t s = int32_t(m > nb / 2 ? m - nb : m);
      mlo = min(mlo, s);
      mhi = max(mhi, s);
    }
  }
  // wave reduction, then block reduction, then one atomic per block
  for (int o = 32; o > 0; o >>= 1) {
    mlo = min(mlo, __shfl_xor(mlo, o));
    mhi = max(mhi, __shfl_xor(mhi, o));
    mx = fmaxf(mx, __shfl_xor(mx, o));
  }
  __shared__ int32_t slo[4], shi[4];
  __shared__ float smx[4];
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    slo[wv] = mlo;
    shi[wv] = mhi;
    smx[wv] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < 4; ++i) {
      mlo = min(mlo, slo[i]);
      mhi = max(mhi, shi[i]);
      mx = fmaxf(mx, smx[i]);
    }
    if (mlo != INT32_MAX) {
      atomicMin(&lo[blockIdx.y], mlo);
      atomicMax(&hi[blockIdx.y], mhi);
    }
    atomicMax(&maxbits[blockIdx.y], __float_as_uint(mx));
  }
}

__global__ void k_gather_taps(const double2* __restrict__ w, int64_t nb, const int64_t* off,
                              const int32_t* mlo, const int32_t* len, double* dst) {
  const int k = blockIdx.y;
  const double2* x = w + int64_t(k) * nb;
  const int32_t L = len[k];
  const int64_t o = off[k];
  const int64_t m0 = mlo[k];
  for (int64_t l = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; l < L;
       l += int64_t(gridDim.x) * blockDim.x) {
    const int64_t m = (m0 + l) & (nb - 1);
    dst[o + l] = x[m].x;
  }
}

__global__ void k_fill_u64(uint64_t* p, uint64_t v, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

inline unsigned blocks_for(int64_t n, int per = 256, unsigned cap = 8192) {
  int64_t b = (n + per - 1) / per;
  if (b < 1) b = 1;
  return unsigned(b > cap ? cap : b);
}

}  // namespace

void band_limits(const rf_grid* g, int64_t* jlo, int64_t* jhi) {
  const double df = g->fs / double(g->n);
  *jlo = int64_t(std::ceil(g->f_low / df));
  *jhi = int64_t(std::floor(g->f_high / df));
}

void band_moment(rf_ctx* ctx, const rf_grid* g, const double* psd, double* moment) {
  int64_t jlo, jhi;
  band_limits(g, &jlo, &jhi);
  const double df = g->fs / double(g->n);
  double* part = static_cast<double*>(ctx->ws[WS_RED].ensure(sizeof(double) * kRedBlocks));
  hipLaunchKernelGGL(k_moment_partial, dim3(kRedBlocks), dim3(kRedThreads), 0, ctx->stream, psd,
                     jlo, jhi, df, part);
  RF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kRedThreads), 0, ctx->stream, part, kRedBlocks,
                     moment);
  RF_HIP(hipGetLastError());
}

void condition_data(rf_ctx* ctx, const rf_grid* g, const double2* xf, const double* psd, float2* q,
                    int nseg) {
  int64_t jlo, jhi;
  band_limits(g, &jlo, &jhi);
  const int64_t nb = jhi - jlo + 1;
  dim3 grid(blocks_for(nb, 256, unsigned(std::max(64, 2048 / nseg))), unsigned(nseg));
  hipLaunchKernelGGL(k_condition, grid, dim3(256), 0, ctx->stream, xf, psd, q, g->n, jlo, nb);
  RF_HIP(hipGetLastError());
}

void ratio_spectrum(rf_ctx* ctx, const rf_grid* g, int64_t nb, const Tf2Coef* ref_dev,
                    const Tf2Coef* tgt_dev, const RatioParam* par_dev, double2* out, int nk) {
  dim3 grid(blocks_for(nb, 256, 4096), unsigned(nk));
  hipLaunchKernelGGL(k_ratio_spectrum, grid, dim3(256), 0, ctx->stream, ref_dev, tgt_dev, par_dev,
                     out, nb, g->fs / double(nb), g->f_low, g->f_high, g->df_high);
  RF_HIP(hipGetLastError());
}

void support_scan(rf_ctx* ctx, const double2* w, int64_t nb, int nk, double thr_tap, int32_t* lo,
                  int32_t* hi, uint32_t* maxabs_bits) {
  dim3 grid(blocks_for(nb, 256, 256), unsigned(nk));
  hipLaunchKernelGGL(k_support_scan, grid, dim3(256), 0, ctx->stream, w, nb, thr_tap, lo, hi,
                     maxabs_bits);
  RF_HIP(hipGetLastError());
}

void gather_taps(rf_ctx* ctx, const double2* w, int64_t nb, int nk, const int64_t* off_dev,
                 const int32_t* mlo_dev, const int32_t* len_dev, double* dst) {
  dim3 grid(blocks_for(nb, 256, 256), unsigned(nk));
  hipLaunchKernelGGL(k_gather_taps, grid, dim3(256), 0, ctx->stream, w, nb, off_dev, mlo_dev,
                     len_dev, dst);
  RF_HIP(hipGetLastError());
}

void fill_u64(rf_ctx* ctx, uint64_t* p, uint64_t v, int64_t n) {
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks_for(n, 256, 1024)), dim3(256), 0, ctx->stream, p, v, n);
  RF_HIP(hipGetLastError());
}
void fill_u32(rf_ctx* ctx, uint32_t* p, uint32_t v, int64_t n) {
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks_for(n, 256, 1024)), dim3(256), 0, ctx->stream, p, v, n);
  RF_HIP(hipGetLastError());
}

}  // namespace rf
