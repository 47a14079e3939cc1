// Stockham auto-sort inverse DFT (exp +2 pi i j m / n, unnormalised) for
// power-of-two n, in FP32 (the SNR series) and FP64 (the ratio-kernel build).
//
// The n-point transform is factored as n = P_1 P_2 ... P_s with every P_i <= 256
// and performed in s global passes.  Pass i treats the data as n / P_i columns
// j, each contributing the P_i elements x[j + r n / P_i]; after the twiddle
// w_{Ns P}^{r (j mod Ns)} (Ns = P_1 ... P_{i-1}) it takes a P-point DFT of
// every column and writes element q to (j / Ns) Ns P + (j mod Ns) + q Ns.
// A workgroup owns 16 consecutive columns, so each global read and write is a
// run of 16 consecutive complex values; the P-point DFT of a column runs in
// LDS as a short in-workgroup Stockham sequence of radix-8/4/2 register
// butterflies.  Twiddles come from sincospi of exact dyadic arguments.  A
// first pass may form its input on the fly instead of reading it: the
// band-limited products of the factored reconstruction, or a matched filter's
// weighted template spectrum (FP64 phase), so neither is ever stored.
#include <type_traits>

#include "recon.h"

namespace rf {
namespace {

template <typename T> struct C2;
template <> struct C2<float> { using t = float2; };
template <> struct C2<double> { using t = double2; };

__device__ inline void sc_pi(float x, float* s, float* c) { sincospif(x, s, c); }
__device__ inline void sc_pi(double x, double* s, double* c) { sincospi(x, s, c); }

template <typename V> __device__ inline V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ inline V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <typename V> __device__ inline V cmul(V a, V b) {
  return V{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename V> __device__ inline V mul_i(V a) { return V{-a.y, a.x}; }  // * (+i)

// In-register DFT of size R with kernel exp(+2 pi i / R).
template <typename V, int R> struct Dft;

template <typename V> struct Dft<V, 2> {
  __device__ static void run(V* v) {
    V a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <typename V> struct Dft<V, 4> {
  __device__ static void run(V* v) {
    V t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    V t2 = cadd(v[1], v[3]), t3 = mul_i(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <typename V> struct Dft<V, 8> {
  __device__ static void run(V* v) {
    using T = decltype(v[0].x);
    V e[4] = {v[0], v[2], v[4], v[6]};
    V o[4] = {v[1], v[3], v[5], v[7]};
    Dft<V, 4>::run(e);
    Dft<V, 4>::run(o);
    const T h = T(0.70710678118654752440084436210485);
    // o[k] *= exp(+i pi k / 4)
    V o1 = V{h * (o[1].x - o[1].y), h * (o[1].x + o[1].y)};
    V o2 = mul_i(o[2]);
    V o3 = V{-h * (o[3].x + o[3].y), h * (o[3].x - o[3].y)};
    v[0] = cadd(e[0], o[0]);
    v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], o1);
    v[5] = csub(e[1], o1);
    v[2] = cadd(e[2], o2);
    v[6] = csub(e[2], o2);
    v[3] = cadd(e[3], o3);
    v[7] = csub(e[3], o3);
  }
};

constexpr int kThreads = 256;
constexpr int kCols = 16;

// One in-LDS Stockham stage of radix R on every column (sub-length NS done).
template <typename T, int P, int NS, int R>
__device__ inline void inner_stage(typename C2<T>::t (*s)[P + 1], const typename C2<T>::t* tw) {
  using V = typename C2<T>::t;
  constexpr int NBF = kCols * P / R;                 // butterflies in the block
  constexpr int PER = (NBF + kThreads - 1) / kThreads;
  constexpr int Q = P / R;
  V v[PER][R];
  int cc[PER], jj[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int b = threadIdx.x + i * kThreads;
    cc[i] = b / Q;
    jj[i] = b % Q;
    if (NBF % kThreads == 0 || b < NBF) {
      const int kk = jj[i] % NS;
#pragma unroll
      for (int q = 0; q < R; ++q) v[i][q] = s[cc[i]][jj[i] + q * Q];
      if (NS > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) v[i][q] = cmul(v[i][q], tw[q * kk * (P / (NS * R))]);
      }
      Dft<V, R>::run(v[i]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int b = threadIdx.x + i * kThreads;
    if (NBF % kThreads == 0 || b < NBF) {
      const int kk = jj[i] % NS;
      const int d = (jj[i] / NS) * NS * R + kk;
#pragma unroll
      for (int q = 0; q < R; ++q) s[cc[i]][d + q * NS] = v[i][q];
    }
  }
  __syncthreads();
}

template <typename T, int P, int NS>
__device__ inline void inner_dft(typename C2<T>::t (*s)[P + 1], const typename C2<T>::t* tw) {
  if constexpr (NS < P) {
    constexpr int REM = P / NS;
    constexpr int R = REM >= 8 ? 8 : REM;
    inner_stage<T, P, NS, R>(s, tw);
    inner_dft<T, P, NS * R>(s, tw);
  }
}

// Input of a first pass formed on the fly: transform y of the batch reads
// conj(Q[f]) Ub[y][f - b0] / n on the band bins f in [b0, b0 + nb), zero elsewhere.
struct BandIn {
  const float2* Q;
  const float2* Ub;
  int64_t b0, nb;
  float inv_n;
};

// Input of a first pass formed from a template's phase series: transform y
// reads sqrt(4 df / I) f^(-7/6) q[y / nt][f - jlo] exp(+i Psi_{y % nt}(f)) on the
// band bins f in [jlo, jhi] (FP64 phase and weighting), zero elsewhere.
struct TmplIn {
  const float2* q;
  const Tf2Coef* coef;
  const double* moment;
  int64_t jlo, jhi;
  double df;
  int nt;
};

enum PassInput { kPlain = 0, kBand = 1, kTmpl = 2 };

// RO (a pass after the first, FP32): the outputs are not stored but read out
// (running peak and threshold crossings of series tmpl0 + blockIdx.y).
template <typename T, int P, int MODE, bool RO = false>
__global__ __launch_bounds__(kThreads) void k_fft_pass(const typename C2<T>::t* __restrict__ in,
                                                       typename C2<T>::t* __restrict__ out,
                                                       int64_t n, int64_t ns, BandIn bin, TmplIn tin,
                                                       PeakOut po) {
  using V = typename C2<T>::t;
  __shared__ V s[kCols][P + 1];
  __shared__ V tw[P];
  const int64_t ncols = n / P;
  const int64_t j0 = int64_t(blockIdx.x) * kCols;
  in += int64_t(blockIdx.y) * n;
  out += int64_t(blockIdx.y) * n;

  for (int m = threadIdx.x; m < P; m += kThreads) {
    T sn, cs;
    sc_pi(T(2 * m) / T(P), &sn, &cs);
    tw[m] = V{cs, sn};
  }
  Tf2Coef tc{};
  double tg = 0.0;
  if constexpr (MODE == kTmpl) {
    tc = tin.coef[blockIdx.y % tin.nt];
    tg = sqrt(4.0 * tin.df / *tin.moment);
  }
  // load 16 columns, apply the inter-pass twiddle exp(+2 pi i r k / (ns P))
  const int64_t L = ns * P;
  for (int e = threadIdx.x; e < kCols * P; e += kThreads) {
    const int c = e % kCols, r = e / kCols;
    const int64_t j = j0 + c;
    V v;
    if constexpr (MODE == kTmpl) {
      const int64_t fj = j + int64_t(r) * ncols;
      v = V{0, 0};
      if (fj >= tin.jlo && fj <= tin.jhi) {
        const double f = double(fj) * tin.df;
        // f^(1/3): the FP32 root refined by one Newton step (about 46 bits)
        double cf = double(cbrtf(float(f)));
        const float cf32 = float(cf);
        cf -= double(float(cf * cf * cf - f) / (3.0f * cf32 * cf32));
        // the phase in FP64 (it reaches ~1e5 rad), reduced to [-pi, pi] in FP64; the
        // exponential of the reduced angle and the amplitude need only FP32
        const double psi = tf2_phase(tc, tc.cbrt_piM * cf);
        const double k = rint(psi * 0.15915494309189533577);
        const float ang = float(fma(-k, 6.28318530717958647693, psi));
        float sn, cs;
        sincosf(ang, &sn, &cs);
        // f^(-7/6) = 1 / (f sqrt(f^(1/3)))
        const float a = float(tg) / (float(f) * sqrtf(float(cf)));
        const float2 q = tin.q[int64_t(blockIdx.y / tin.nt) * (tin.jhi - tin.jlo + 1) + (fj - tin.jlo)];
        v = V{a * (q.x * cs - q.y * sn), a * (q.x * sn + q.y * cs)};
      }
    } else if constexpr (MODE == kBand) {
      const int64_t i = j + int64_t(r) * ncols - bin.b0;
      v = V{0, 0};
      if (i >= 0 && i < bin.nb) {
        const float2 q = bin.Q[bin.b0 + i];
        const float2 u = bin.Ub[int64_t(blockIdx.y) * bin.nb + i];
        const float xr = q.x * bin.inv_n, xi = -q.y * bin.inv_n;
        v = V{xr * u.x - xi * u.y, xr * u.y + xi * u.x};
      }
    } else {
      v = in[j + int64_t(r) * ncols];
    }
    if (ns > 1) {
      const int64_t k = j & (ns - 1);
      T sn, cs;
      sc_pi(T(2 * ((int64_t(r) * k) & (L - 1))) / T(L), &sn, &cs);
      v = cmul(v, V{cs, sn});
    }
    s[c][r] = v;
  }
  __syncthreads();
  inner_dft<T, P, 1>(s, tw);
  if constexpr (RO) {
    static_assert(std::is_same<T, float>::value && MODE == kPlain, "read-out: FP32 passes after the first");
    // output m = (j / ns) ns P + j mod ns + q ns, as in the store below
    Best best{-1.f, INT32_MAX};
    for (int e = threadIdx.x; e < kCols * P; e += kThreads) {
      const int c = e % kCols, q = e / kCols;
      const int64_t j = j0 + c;
      peak_visit(best, s[c][q].x, s[c][q].y, (j / ns) * ns * P + (j & (ns - 1)) + int64_t(q) * ns, po);
    }
    peak_commit(best, po);
    return;
  }
  if (ns == 1) {
    // out[j P + q]: the block's 16 columns are one contiguous run
    for (int e = threadIdx.x; e < kCols * P; e += kThreads) {
      const int q = e % P, c = e / P;
      out[(j0 + c) * P + q] = s[c][q];
    }
  } else {
    for (int e = threadIdx.x; e < kCols * P; e += kThreads) {
      const int c = e % kCols, q = e / kCols;
      const int64_t j = j0 + c;
      out[(j / ns) * ns * P + (j & (ns - 1)) + int64_t(q) * ns] = s[c][q];
    }
  }
}

// Split log2(n) into at least two passes of at most 8 bits each, as even as
// possible (16 columns per workgroup need n / P >= 16 in every pass).
std::vector<int> plan_passes(int lg) {
  int s = (lg + 7) / 8;
  if (s < 2) s = 2;
  std::vector<int> bits(s, lg / s);
  for (int i = 0; i < lg % s; ++i) bits[i] += 1;
  return bits;
}

template <typename T, int MODE = kPlain, bool RO = false>
void launch_pass(int bits, const typename C2<T>::t* in, typename C2<T>::t* out, int64_t n,
                 int64_t ns, int batch, hipStream_t st, BandIn bin = BandIn{}, TmplIn tin = TmplIn{},
                 PeakOut po = PeakOut{}) {
  const int64_t P = int64_t(1) << bits;
  dim3 grid(unsigned((n / P) / kCols), unsigned(batch));
  switch (bits) {
#define RF_FFT_CASE(B)                                                                            \
  case B:                                                                                         \
    hipLaunchKernelGGL((k_fft_pass<T, (1 << B), MODE, RO>), grid, dim3(kThreads), 0, st, in, out, n, \
                       ns, bin, tin, po);                                                         \
    break;
    RF_FFT_CASE(4)
    RF_FFT_CASE(5)
    RF_FFT_CASE(6)
    RF_FFT_CASE(7)
    RF_FFT_CASE(8)
#undef RF_FFT_CASE
    default:
      throw Error{RF_E_UNSUPPORTED, "fft: unsupported pass size"};
  }
  RF_HIP(hipGetLastError());
}

template <typename T>
void fft_inverse(rf_ctx* ctx, const typename C2<T>::t* in, typename C2<T>::t* out, int64_t n,
                 int batch, typename C2<T>::t* wsa_in, typename C2<T>::t* wsb_in, const BandIn* band = nullptr,
                 const TmplIn* tmpl = nullptr, const PeakOut* ro = nullptr) {
  using V = typename C2<T>::t;
  RF_CHECK(is_pow2(n) && n >= 256 && n <= (int64_t(1) << 24), "fft: n must be a power of two in [2^8, 2^24]");
  const int lg = ilog2(n);
  std::vector<int> bits = plan_passes(lg);
  const int s = int(bits.size());
  V* wa = nullptr;
  V* wb = nullptr;
  if (wsa_in) {
    wa = wsa_in;
    wb = wsb_in;
  } else {
    if (s > 1) wa = static_cast<V*>(ctx->ws[WS_FFT_A].ensure(sizeof(V) * size_t(n) * batch));
    if (s > 2) wb = static_cast<V*>(ctx->ws[WS_FFT_B].ensure(sizeof(V) * size_t(n) * batch));
  }
  const V* src = in;
  int64_t ns = 1;
  for (int i = 0; i < s; ++i) {
    V* dst = (i == s - 1) ? out : ((i % 2 == 0) ? wa : wb);
    if constexpr (std::is_same<T, float>::value) {
      if (i == 0 && (band || tmpl)) {
        if (band)
          launch_pass<T, kBand>(bits[i], nullptr, dst, n, ns, batch, ctx->stream, *band);
        else
          launch_pass<T, kTmpl>(bits[i], nullptr, dst, n, ns, batch, ctx->stream, BandIn{}, *tmpl);
        ns <<= bits[i];
        src = dst;
        continue;
      }
    }
    if constexpr (std::is_same<T, float>::value) {
      if (i == s - 1 && ro) {          // the last pass reads the outputs out instead
        launch_pass<T, kPlain, true>(bits[i], src, nullptr, n, ns, batch, ctx->stream, BandIn{}, TmplIn{}, *ro);
        break;
      }
    }
    launch_pass<T>(bits[i], src, dst, n, ns, batch, ctx->stream);
    ns <<= bits[i];
    src = dst;
  }
}

}  // namespace

void fft_inverse_f32(rf_ctx* ctx, const float2* in, float2* out, int64_t n, int batch, float2* wsa,
                     float2* wsb) {
  fft_inverse<float>(ctx, in, out, n, batch, wsa, wsb);
}
void fft_inverse_f64(rf_ctx* ctx, const double2* in, double2* out, int64_t n, int batch) {
  fft_inverse<double>(ctx, in, out, n, batch, nullptr, nullptr);
}
void fft_inverse_tmpl_f32(rf_ctx* ctx, const rf_grid* g, const float2* q, const Tf2Coef* coef, int nt,
                          const double* moment, float2* out, int batch, float2* wsa, float2* wsb) {
  RF_CHECK(nt >= 1 && batch % nt == 0, "fft: batch must be a multiple of the template count");
  TmplIn t{};
  t.q = q;
  t.coef = coef;
  t.moment = moment;
  band_limits(g, &t.jlo, &t.jhi);
  t.df = g->fs / double(g->n);
  t.nt = nt;
  RF_CHECK(t.jlo >= 1 && t.jhi < g->n, "fft: band outside the transform");
  fft_inverse<float>(ctx, nullptr, out, g->n, batch, wsa, wsb, nullptr, &t);
}
void fft_inverse_tmpl_peaks_f32(rf_ctx* ctx, const rf_grid* g, const float2* q, const Tf2Coef* coef, int nt,
                                const double* moment, int batch, const PeakOut& po) {
  RF_CHECK(nt >= 1 && batch % nt == 0, "fft: batch must be a multiple of the template count");
  TmplIn t{};
  t.q = q;
  t.coef = coef;
  t.moment = moment;
  band_limits(g, &t.jlo, &t.jhi);
  t.df = g->fs / double(g->n);
  t.nt = nt;
  RF_CHECK(t.jlo >= 1 && t.jhi < g->n, "fft: band outside the transform");
  fft_inverse<float>(ctx, nullptr, nullptr, g->n, batch, nullptr, nullptr, nullptr, &t, &po);
}
void fft_inverse_band_f32(rf_ctx* ctx, const float2* Q, const float2* Ub, int64_t b0, int64_t nb, float inv_n,
                          float2* out, int64_t n, int batch) {
  RF_CHECK(b0 >= 0 && nb >= 0 && b0 + nb <= n, "fft: band outside the transform");
  const BandIn band{Q, Ub, b0, nb, inv_n};
  fft_inverse<float>(ctx, nullptr, out, n, batch, nullptr, nullptr, &band);
}

}  // namespace rf
