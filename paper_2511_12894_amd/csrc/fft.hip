// Stockham auto-sort inverse DFT (exp +2 pi i j m / n, unnormalised) for
// power-of-two n, in FP32 (the SNR series) and FP64 (the ratio-kernel build).
//
// The n-point transform is factored as n = P_1 P_2 ... P_s with every P_i <= 256
// and performed in s global passes.  Pass i treats the data as n / P_i columns
// j, each contributing the P_i elements x[j + r n / P_i]; after the twiddle
// w_{Ns P}^{r (j mod Ns)} (Ns = P_1 ... P_{i-1}) it takes a P-point DFT of
// every column and writes element q to (j / Ns) Ns P + (j mod Ns) + q Ns.
// A workgroup owns 16 consecutive columns, so each global read and write is a
// run of 16 consecutive complex values.
//
// FP32 passes split P = R1 R2 into two register radices: a thread loads the R1
// inputs of its first butterfly straight from memory (elements u + i P / R1 of
// its column), the inter-pass twiddles advancing by one complex product per
// element from two sin/cos values of exact dyadic arguments; one exchange
// through LDS then gives it the R2 inputs of its second butterfly, whose
// outputs (elements u + q R1) it stores, or reads out, from registers.  A
// first pass may form its input on the fly instead of reading it: the
// band-limited products of the factored reconstruction, or a matched filter's
// weighted template spectrum (FP64 phase), so neither is ever stored.  Matched
// filters of 2^20 to 2^23 samples take two passes instead of three (a 1024- to
// 4096-point first pass of one column per workgroup, then 1024- or 2048-point
// columns, 16 or 8 a workgroup, in 135 KB of LDS), so their intermediate crosses
// HBM once.
// FP64 passes (kernel builds) run the P-point DFT in LDS as a short
// in-workgroup Stockham sequence of radix-8/4/2 butterflies.
#include <type_traits>

#include "recon.h"

namespace rf {
namespace {

template <typename T> struct C2;
template <> struct C2<float> { using t = float2; };
template <> struct C2<double> { using t = double2; };

// sin(pi x) and cos(pi x) in FP32 for |x| <= 2^22: the nearest quarter turn
// q = rint(2x), the remainder f = x - q/2 in [-1/4, 1/4] (exact), theta = pi f
// with pi split into two floats, then an odd degree-7 and an even degree-8
// polynomial on [-pi/4, pi/4] (coefficients fitted here by weighted least
// squares: relative error 3.6e-9 for sin, absolute 5.4e-11 for cos, in exact
// arithmetic; about 0.6 ulp of 1 in FP32 with fused multiply-adds), rotated by
// the quarter turn.
__device__ inline void sincospi_f32(float x, float* s, float* c) {
  const float q = rintf(2.f * x);
  const float f = fmaf(-0.5f, q, x);
  const float th = fmaf(f, 3.14159274101257324f, f * -8.74227766e-08f);
  const float u = th * th;
  float ps = fmaf(-1.9517e-04f, u, 8.33218e-03f);
  ps = fmaf(ps, u, -0.16666655f);
  const float sn = fmaf(th * u, ps, th);
  float pc = fmaf(2.43904474e-05f, u, -1.38867638e-03f);
  pc = fmaf(pc, u, 4.16666233e-02f);
  pc = fmaf(pc, u, -0.499999997f);
  const float cs = fmaf(u, pc, 1.f);
  const int qi = int(q) & 3;
  const float s0 = (qi & 1) ? cs : sn, c0 = (qi & 1) ? sn : cs;
  *s = (qi & 2) ? -s0 : s0;
  *c = ((qi + 1) & 2) ? -c0 : c0;
}
__device__ inline void sc_pi(double x, double* s, double* c) { sincospi(x, s, c); }

// sin and cos of a template phase psi (FP64, up to ~1e5 rad): psi reduced in FP64
// to psi / (2 pi) - k in [-1/2, 1/2] turns, then the hardware sine and cosine of
// an angle in turns (measured here at most 1.3e-7 from the exact values over
// that range, about two units in the last place of 1).
__device__ inline void phase_exp(double psi, float* s, float* c) {
  const double k = rint(psi * 0.15915494309189533577);
  const float x = float(fma(psi, 0.15915494309189533577, -k));
  *s = __builtin_amdgcn_sinf(x);
  *c = __builtin_amdgcn_cosf(x);
}

template <typename V> __device__ inline V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <typename V> __device__ inline V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
// Complex product with the fused multiply-adds written out, and butterflies
// compiled without contraction (below): a pass rounds the same way whether its
// outputs are stored or read out.
__device__ inline float2 cmul(float2 a, float2 b) {
  return float2{fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x)};
}
__device__ inline double2 cmul(double2 a, double2 b) {
  return double2{fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x)};
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
#pragma clang fp contract(off)
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

// 16 = 4 x 4: DFTs of the four residue classes m (inputs m + 4 p), the twiddles
// w16^(m k1), then DFTs over m; output k1 + 4 k2.
template <typename V> struct Dft<V, 16> {
  __device__ static void run(V* v) {
#pragma clang fp contract(off)
    using T = decltype(v[0].x);
    const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);
    const T h = T(0.70710678118654752440084436210485);
    V y[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
      for (int p = 0; p < 4; ++p) y[m][p] = v[m + 4 * p];
      Dft<V, 4>::run(y[m]);
    }
    // w16^e for e = m k1: 1 = (c1, s1), 2 = (h, h), 3 = (s1, c1), 4 = i, 6 = (-h, h), 9 = (-c1, -s1)
    y[1][1] = cmul(y[1][1], V{c1, s1});
    y[1][2] = V{h * (y[1][2].x - y[1][2].y), h * (y[1][2].x + y[1][2].y)};
    y[1][3] = cmul(y[1][3], V{s1, c1});
    y[2][1] = V{h * (y[2][1].x - y[2][1].y), h * (y[2][1].x + y[2][1].y)};
    y[2][2] = mul_i(y[2][2]);
    y[2][3] = V{-h * (y[2][3].x + y[2][3].y), h * (y[2][3].x - y[2][3].y)};
    y[3][1] = cmul(y[3][1], V{s1, c1});
    y[3][2] = V{-h * (y[3][2].x + y[3][2].y), h * (y[3][2].x - y[3][2].y)};
    y[3][3] = cmul(y[3][3], V{-c1, -s1});
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      V z[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
      Dft<V, 4>::run(z);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = z[k2];
    }
  }
};

constexpr int kThreads = 256;
constexpr int kCols = 16;
static_assert(kThreads % kCols == 0, "a thread keeps one column through every loop of a pass");

// LDS layout of a block's columns: element x of a column at x + x / 32 (one
// pad slot every 32 elements), columns lds_stride apart.  With 64 banks of 4
// bytes this spreads the column-strided loads and the radix-8 stage writes
// over the banks (a column stride of P + 1 put up to 4 lanes on a bank).
__device__ constexpr int sw(int x) { return x + (x >> 5); }
template <typename T, int P> struct Lds;
template <int P> struct Lds<float, P> {
  static constexpr int stride = P == 16 ? 18 : P == 32 ? 37 : P == 64 ? 70 : P == 128 ? 138 : 266;
};
template <int P> struct Lds<double, P> {
  static constexpr int stride = P == 16 ? 17 : P == 32 ? 35 : P == 64 ? 67 : P == 128 ? 131 : 263;
};
template <typename T, int P> using LdsRow = typename C2<T>::t[Lds<T, P>::stride];

// FP32 passes: P = R1 x R2, the radices of a thread's two register butterflies.
template <int P> struct Radix;
template <> struct Radix<16> { static constexpr int R1 = 4, R2 = 4; };
template <> struct Radix<32> { static constexpr int R1 = 4, R2 = 8; };
template <> struct Radix<64> { static constexpr int R1 = 8, R2 = 8; };
template <> struct Radix<128> { static constexpr int R1 = 8, R2 = 16; };
template <> struct Radix<256> { static constexpr int R1 = 16, R2 = 16; };

// Columns per workgroup of the FP32 passes: 32 (256-byte runs of every row)
// where the pass has a multiple of 32 columns, else 16; the workgroup has one
// thread per butterfly of the larger of its two stages (P / R1 or R1 per column).
template <int P, int C> constexpr int threads32() {
  return C * (P / Radix<P>::R1 > Radix<P>::R1 ? P / Radix<P>::R1 : Radix<P>::R1);
}

// One in-LDS Stockham stage of radix R on every column (sub-length NS done).
template <typename T, int P, int NS, int R>
__device__ inline void inner_stage(LdsRow<T, P>* s, const typename C2<T>::t* tw) {
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
      for (int q = 0; q < R; ++q) v[i][q] = s[cc[i]][sw(jj[i] + q * Q)];
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
      for (int q = 0; q < R; ++q) s[cc[i]][sw(d + q * NS)] = v[i][q];
    }
  }
  __syncthreads();
}

template <typename T, int P, int NS>
__device__ inline void inner_dft(LdsRow<T, P>* s, const typename C2<T>::t* tw) {
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

enum PassInput { kPlain = 0, kBand = 1 };

// FP64 pass (plain input, stored output): columns through LDS, the P-point DFT
// as in-LDS radix-8/4/2 stages, inter-pass twiddles from sincospi.
template <typename T, int P>
__global__ __launch_bounds__(kThreads) void k_fft_pass(const typename C2<T>::t* __restrict__ in,
                                                       typename C2<T>::t* __restrict__ out, int64_t n,
                                                       int64_t ns) {
  using V = typename C2<T>::t;
  __shared__ V s[kCols][Lds<T, P>::stride];
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
  // load 16 columns, apply the inter-pass twiddle exp(+2 pi i r k / (ns P)); r k < ns P <= 2^24
  // is exact in 32 bits and as a float, 2 / (ns P) a power of two
  const int64_t L = ns * P;
  const T two_over_L = T(2) / T(L);
  for (int e = threadIdx.x; e < kCols * P; e += kThreads) {
    const int c = e % kCols, r = e / kCols;
    const int64_t j = j0 + c;
    V v = in[j + int64_t(r) * ncols];
    if (ns > 1) {
      const uint32_t k = uint32_t(j) & uint32_t(ns - 1);
      T sn, cs;
      sc_pi(T(uint32_t(r) * k) * two_over_L, &sn, &cs);
      v = cmul(v, V{cs, sn});
    }
    s[c][sw(r)] = v;
  }
  __syncthreads();
  inner_dft<T, P, 1>(s, tw);
  if (ns == 1) {
    // out[j P + q]: the block's 16 columns are one contiguous run
    for (int e = threadIdx.x; e < kCols * P; e += kThreads) {
      const int q = e % P, c = e / P;
      out[(j0 + c) * P + q] = s[c][sw(q)];
    }
  } else {
    for (int e = threadIdx.x; e < kCols * P; e += kThreads) {
      const int c = e % kCols, q = e / kCols;
      const int64_t j = j0 + c;
      out[(j / ns) * ns * P + (j & (ns - 1)) + int64_t(q) * ns] = s[c][sw(q)];
    }
  }
}

// Inter-pass twiddles w_L^(r k) of a thread's R1 inputs r = u + i Q1 (i < R1),
// k = j mod ns, L = ns P: sin/cos of the exact arguments 2 (u + i0 Q1) k / L
// (every 8 elements) and 2 Q1 k / L (r k < L <= 2^24 is exact in 32 bits and as
// a float, 2 / L a power of two), the twiddle advancing by one complex product
// per element in between (at most 7 products: about 7 units in the last place).
template <int R1, int Q1>
__device__ inline void apply_twiddles(float2* v, uint32_t u, uint32_t k, float two_over_L) {
  float sn, cs;
  sincospi_f32(float(uint32_t(Q1) * k) * two_over_L, &sn, &cs);
  const float2 b{cs, sn};
#pragma unroll
  for (int i0 = 0; i0 < R1; i0 += 8) {
    sincospi_f32(float((u + uint32_t(i0 * Q1)) * k) * two_over_L, &sn, &cs);
    float2 t{cs, sn};
#pragma unroll
    for (int i = i0; i < i0 + 8 && i < R1; ++i) {
      v[i] = cmul(v[i], t);
      if (i + 1 < i0 + 8 && i + 1 < R1) t = cmul(t, b);
    }
  }
}

// Twiddles w_P^(q u) and radix-R2 DFT of a thread's second butterfly (inputs
// v[q] = stage-one output u + q R1 of its column, u < R1); its outputs are the
// column's elements u + q R1.
template <int P>
__device__ inline void second_butterfly(const float2* tw, int u, float2* v) {
  constexpr int R2 = Radix<P>::R2;
#pragma unroll
  for (int q = 1; q < R2; ++q) v[q] = cmul(v[q], tw[q * u]);
  Dft<float2, R2>::run(v);
}

// Second register butterfly of an FP32 pass: thread u < R1 of column c takes the
// stage-one outputs u + q R1 (q < R2) from LDS.
template <int P>
__device__ inline void second_stage(const LdsRow<float, P>* s, const float2* tw, int c, int u, float2* v) {
  constexpr int R1 = Radix<P>::R1, R2 = Radix<P>::R2;
#pragma unroll
  for (int q = 0; q < R2; ++q) v[q] = s[c][sw(u + q * R1)];
  second_butterfly<P>(tw, u, v);
}

// FP32 pass.  Thread (c, u) = (threadIdx % C, threadIdx / C) of column j =
// C blockIdx.x + c: for u < P / R1 its first butterfly on elements u + i P / R1
// (loaded, or formed from the band products for MODE kBand on a first pass),
// outputs to LDS at u R1 + i; for u < R1 its second butterfly.  RO (a pass after
// the first): the outputs are read out (running peak and threshold crossings of
// series tmpl0 + blockIdx.y) instead of stored.
template <int P, int C, int MODE, bool RO>
__global__ __launch_bounds__((threads32<P, C>())) void k_pass32(const float2* __restrict__ in,
                                                              float2* __restrict__ out, int32_t n, int32_t ns,
                                                              BandIn bin, PeakOut po) {
  using V = float2;
  constexpr int R1 = Radix<P>::R1, R2 = Radix<P>::R2, Q1 = P / R1, NT = threads32<P, C>();
  constexpr int RM = R1 > R2 ? R1 : R2;
  __shared__ V s[C][Lds<float, P>::stride];
  __shared__ V tw[P];
  const int32_t ncols = n / P;
  const int c = int(threadIdx.x) % C, u = int(threadIdx.x) / C;
  const int32_t j0 = int32_t(blockIdx.x) * C, j = j0 + c;
  in += int64_t(blockIdx.y) * n;
  out += int64_t(blockIdx.y) * n;
  for (int m = threadIdx.x; m < P; m += NT) {
    float sn, cs;
    sincospi_f32(float(2 * m) / float(P), &sn, &cs);
    tw[m] = V{cs, sn};
  }
  V v[RM];
  if (u < Q1) {
#pragma unroll
    for (int i = 0; i < R1; ++i) {
      const int32_t x = j + (u + i * Q1) * ncols;
      if constexpr (MODE == kBand) {
        const int64_t b = int64_t(x) - bin.b0;
        v[i] = V{0.f, 0.f};
        if (b >= 0 && b < bin.nb) {
          const float2 q = bin.Q[x];
          const float2 w = bin.Ub[int64_t(blockIdx.y) * bin.nb + b];
          const float xr = q.x * bin.inv_n, xi = -q.y * bin.inv_n;
          v[i] = V{xr * w.x - xi * w.y, xr * w.y + xi * w.x};
        }
      } else {
        v[i] = in[x];
      }
    }
    if (ns > 1) apply_twiddles<R1, Q1>(v, uint32_t(u), uint32_t(j) & uint32_t(ns - 1), 2.f / float(ns * P));
    Dft<V, R1>::run(v);
  }
  if (u < Q1) {
#pragma unroll
    for (int q = 0; q < R1; ++q) s[c][sw(u * R1 + q)] = v[q];
  }
  __syncthreads();
  if (u < R1) second_stage<P>(s, tw, c, u, v);
  const int32_t base = (j / ns) * ns * P + (j & (ns - 1));   // output m = base + element * ns
  if constexpr (RO) {
    static_assert(MODE == kPlain, "read-out: passes after the first");
    Best best{-1.f, INT32_MAX};
    if (u < R1) {
#pragma unroll
      for (int q = 0; q < R2; ++q) peak_visit_rising_raw(best, v[q].x, v[q].y, base + (u + q * R1) * ns, po);
    }
    peak_commit(best, po);
    return;
  }
  if (ns == 1) {
    // out[j P + q] through LDS: the block's C columns are one contiguous run
    __syncthreads();
    if (u < R1) {
#pragma unroll
      for (int q = 0; q < R2; ++q) s[c][sw(u + q * R1)] = v[q];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < C * P; e += NT) {
      const int q = e % P, cc = e / P;
      out[(j0 + cc) * P + q] = s[cc][sw(q)];
    }
  } else if (u < R1) {
#pragma unroll
    for (int q = 0; q < R2; ++q) out[base + (u + q * R1) * ns] = v[q];
  }
}

// First pass of the matched filters of TPW templates sharing one workgroup.  The
// phase of a template is a fixed combination of nine functions of the bin,
// Psi = e0 + e5 x^-5 + e3 x^-3 + e2 x^-2 + e1 x^-1 + el ln f + ex x + exl x ln f
// + exx x^2 with x = f^(1/3) (the TaylorF2 series in v = (pi M)^(1/3) x); the
// functions of every bin (FP64) and f^(-7/6) are computed once per workgroup
// and kept in registers (all eight where a thread has at most four bins, else
// x, 1 / x and ln f), so a template's phase costs eight FP64 multiply-adds per
// bin.  Each template forms its weighted spectrum in the registers of the first
// butterflies (bins j + (u + i P / R1) n / P), transforms its columns as
// k_pass32 does and stores them.
template <int P, int C, int TPW>
__global__ __launch_bounds__((threads32<P, C>())) void k_fft_tmpl_pass(float2* __restrict__ out, int32_t n,
                                                                     int batch, TmplIn tin) {
  using V = float2;
  constexpr int R1 = Radix<P>::R1, R2 = Radix<P>::R2, Q1 = P / R1, NT = threads32<P, C>();
  constexpr int RM = R1 > R2 ? R1 : R2;
  constexpr bool kAll = R1 <= 4;              // keep all eight bin functions
  constexpr int NG = kAll ? 8 : 3;
  __shared__ V s[C][Lds<float, P>::stride];
  __shared__ V tw[P];
  const int32_t ncols = n / P;
  const int c = int(threadIdx.x) % C, u = int(threadIdx.x) / C;
  const int32_t j0 = int32_t(blockIdx.x) * C, j = j0 + c;
  for (int m = threadIdx.x; m < P; m += NT) {
    float sn, cs;
    sincospi_f32(float(2 * m) / float(P), &sn, &cs);
    tw[m] = V{cs, sn};
  }
  const double tg = sqrt(4.0 * tin.df / *tin.moment);
  // per-bin functions: kAll: x^-5, x^-3, x^-2, x^-1, ln f, x, x ln f, x^2; else x, 1 / x, ln f
  // (in band: g[0] != 0; out of band all zero)
  double g[NG][R1];
  float a0[R1];
#pragma unroll
  for (int i = 0; i < R1; ++i) {
#pragma unroll
    for (int q = 0; q < NG; ++q) g[q][i] = 0.0;
    a0[i] = 0.f;
    const int32_t fj = j + (u + i * Q1) * ncols;
    if (u < Q1 && fj >= tin.jlo && fj <= tin.jhi) {
      const double f = double(fj) * tin.df;
      // f^(1/3): the FP32 root refined by one Newton step (about 46 bits)
      double x = double(cbrtf(float(f)));
      const float x32 = float(x);
      x -= double(float(x * x * x - f) / (3.0f * x32 * x32));
      const double ix = 1.0 / x, lf = log(f);
      if constexpr (kAll) {
        const double ix2 = ix * ix, ix3 = ix2 * ix;
        g[0][i] = ix3 * ix2;
        g[1][i] = ix3;
        g[2][i] = ix2;
        g[3][i] = ix;
        g[4][i] = lf;
        g[5][i] = x;
        g[6][i] = x * lf;
        g[7][i] = x * x;
      } else {
        g[0][i] = x;
        g[1][i] = ix;
        g[2][i] = lf;
      }
      // f^(-7/6) = 1 / (f sqrt(f^(1/3)))
      a0[i] = float(tg) / (float(f) * sqrtf(float(x)));
    }
  }
  const int y0 = int(blockIdx.y) * TPW;
#pragma unroll 1
  for (int t = 0; t < TPW && y0 + t < batch; ++t) {
    const int y = y0 + t;
    const Tf2Coef tc = tin.coef[y % tin.nt];
    const float2* qs = tin.q + int64_t(y / tin.nt) * (tin.jhi - tin.jlo + 1);
    V v[RM];
    if (u < Q1) {
#pragma unroll
      for (int i = 0; i < R1; ++i) {
        v[i] = V{0.f, 0.f};
        if (g[0][i] != 0.0) {
          const int32_t fj = j + (u + i * Q1) * ncols;
          // the phase in FP64 (it reaches ~1e5 rad), reduced in FP64 to psi / pi - 2k in
          // [-1, 1]; the exponential of the reduced angle and the amplitude need only FP32
          double psi;
          if constexpr (kAll) {
            psi = fma(tc.e5, g[0][i], tc.e0);
            psi = fma(tc.e3, g[1][i], psi);
            psi = fma(tc.e2, g[2][i], psi);
            psi = fma(tc.e1, g[3][i], psi);
            psi = fma(tc.el, g[4][i], psi);
            psi = fma(tc.ex, g[5][i], psi);
            psi = fma(tc.exl, g[6][i], psi);
            psi = fma(tc.exx, g[7][i], psi);
          } else {
            const double x = g[0][i], ix = g[1][i], lf = g[2][i];
            const double ix2 = ix * ix, ix3 = ix2 * ix;
            psi = fma(tc.e5, ix3 * ix2, tc.e0);
            psi = fma(tc.e3, ix3, psi);
            psi = fma(tc.e2, ix2, psi);
            psi = fma(tc.e1, ix, psi);
            psi = fma(tc.el, lf, psi);
            psi = fma(tc.ex, x, psi);
            psi = fma(tc.exl, x * lf, psi);
            psi = fma(tc.exx, x * x, psi);
          }
          float sn, cs;
          phase_exp(psi, &sn, &cs);
          const float2 q = qs[fj - tin.jlo];
          v[i] = V{a0[i] * (q.x * cs - q.y * sn), a0[i] * (q.x * sn + q.y * cs)};
        }
      }
      Dft<V, R1>::run(v);
#pragma unroll
      for (int q = 0; q < R1; ++q) s[c][sw(u * R1 + q)] = v[q];
    }
    __syncthreads();
    if (u < R1) second_stage<P>(s, tw, c, u, v);
    __syncthreads();
    if (u < R1) {
#pragma unroll
      for (int q = 0; q < R2; ++q) s[c][sw(u + q * R1)] = v[q];
    }
    __syncthreads();
    // out[j P + q]: the block's 16 columns are one contiguous run
    float2* o = out + int64_t(y) * n;
    for (int e = threadIdx.x; e < C * P; e += NT) {
      const int q = e % P, cc = e / P;
      o[(j0 + cc) * P + q] = s[cc][sw(q)];
    }
    __syncthreads();
  }
}

// first pass of matched filters: templates per workgroup
constexpr int kTmplPerBlock = 16;

// ---------------------------------------------------------------- two-pass form
// Matched filters of n = P_A P_B <= 2^23 samples in two passes (P_B = 1024 up to
// 2^21, then 2048): pass A (k_tmpl_wide) forms each template's spectrum and takes
// P_A-point DFTs of single columns through LDS; pass B (k_pass_wide) takes P_B-point
// DFTs of 16 or 8 columns (135 KB of LDS) and stores or reads out its outputs.  The intermediate
// is written and read once, as a transform too large for the chip must.

// Stockham stage (NS done, radix R) on C columns of P points in LDS: butterfly
// beta = threadIdx.x + k NT (beta < C P / R) is column beta % C, index b = beta / C;
// it takes elements b + q P / R, the twiddles w_P^(q (b mod NS) P / (NS R)), a
// radix-R DFT, and writes elements (b / NS) NS R + b mod NS + q NS.
template <int P, int C, int NT, int NS, int R, int ST>
__device__ inline void lds_stage(float2 (*s)[ST], const float2* tw) {
  constexpr int NB = C * P / R, K = (NB + NT - 1) / NT, Q = P / R;
  float2 v[K][R];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int beta = int(threadIdx.x) + k * NT;
    if (NB % NT == 0 || beta < NB) {
      const int c = beta % C, b = beta / C, kk = b % NS;
#pragma unroll
      for (int q = 0; q < R; ++q) v[k][q] = s[c][sw(b + q * Q)];
      if (NS > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) v[k][q] = cmul(v[k][q], tw[q * kk * (P / (NS * R))]);
      }
      Dft<float2, R>::run(v[k]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int beta = int(threadIdx.x) + k * NT;
    if (NB % NT == 0 || beta < NB) {
      const int c = beta % C, b = beta / C, kk = b % NS;
      const int d = (b / NS) * NS * R + kk;
#pragma unroll
      for (int q = 0; q < R; ++q) s[c][sw(d + q * NS)] = v[k][q];
    }
  }
  __syncthreads();
}

// Radices of pass A: a radix-4 first butterfly (four bins a thread keep their
// phase functions in registers at four waves per SIMD), then 8, 8 and 4 or 8;
// at 4096 points 16, 8 and 8 (the order that fits 128 registers a thread).
template <int PA> struct WideA;
template <> struct WideA<1024> { static constexpr int R1 = 4, R2 = 8, R3 = 8, R4 = 4; };
template <> struct WideA<2048> { static constexpr int R1 = 4, R2 = 8, R3 = 8, R4 = 8; };
template <> struct WideA<4096> { static constexpr int R1 = 4, R2 = 16, R3 = 8, R4 = 8; };

// Pass A of the two-pass matched filter: one column j (of n / PA) per workgroup,
// PA / R1 threads; thread u forms bins j + (u + i PA / R1) n / PA (i < R1) of each
// of TPW templates from x = f^(1/3), 1 / x and ln f computed once per bin (the
// phase basis of k_fft_tmpl_pass), its first butterfly in registers, two stages
// in LDS (radices R2, R3), and a last stage whose outputs b + q NS it stores from
// registers: out[j PA + e].
template <int PA, int TPW>
__global__ __launch_bounds__(PA / WideA<PA>::R1) void k_tmpl_wide(float2* __restrict__ out, int32_t n, int batch,
                                                                  TmplIn tin) {
  using V = float2;
  using W = WideA<PA>;
  constexpr int R1 = W::R1, R2 = W::R2, R3 = W::R3, R4 = W::R4;
  constexpr int NT = PA / R1, QA = PA / R1;
  constexpr int NS4 = R1 * R2 * R3;                 // done before the last stage
  constexpr int NL = PA / R4;                       // last-stage butterflies
  constexpr int KL = (NL + NT - 1) / NT;            // per thread
  static_assert(R1 * R2 * R3 * R4 == PA, "pass A radices");
  constexpr int ST = PA + PA / 32 + 1;
  __shared__ V s[1][ST];
  __shared__ V tw[PA];
  const int32_t ncols = n / PA;
  const int u = int(threadIdx.x);
  // workgroups go to the 8 XCDs in turn: give each XCD a contiguous range of
  // columns, so the workgroups running together on one XCD read neighbouring
  // bins of the conditioned data and share its cache lines in that XCD's L2
  const int32_t j = int32_t(blockIdx.x % 8u) * (ncols / 8) + int32_t(blockIdx.x / 8u);
  for (int m = u; m < PA; m += NT) {
    float sn, cs;
    sincospi_f32(float(2 * m) / float(PA), &sn, &cs);
    tw[m] = V{cs, sn};
  }
  const double tg = sqrt(4.0 * tin.df / *tin.moment);
  double gx[R1], gi[R1], gl[R1];                    // x, 1 / x, ln f (in band: gx > 0)
#pragma unroll
  for (int i = 0; i < R1; ++i) {
    gx[i] = 0.0;
    gi[i] = 0.0;
    gl[i] = 0.0;
    const int32_t fj = j + (u + i * QA) * ncols;
    if (fj >= tin.jlo && fj <= tin.jhi) {
      const double f = double(fj) * tin.df;
      double x = double(cbrtf(float(f)));
      const float x32 = float(x);
      x -= double(float(x * x * x - f) / (3.0f * x32 * x32));
      gx[i] = x;
      gi[i] = 1.0 / x;
      gl[i] = log(f);
    }
  }
  const int y0 = int(blockIdx.y) * TPW;
  // the conditioned data times f^(-7/6) of the thread's bins, for the segment of
  // the templates in hand (read again only when the segment changes)
  V aq[R1];
  int seg = -1;
#pragma unroll 1
  for (int t = 0; t < TPW && y0 + t < batch; ++t) {
    const int y = y0 + t;
    const Tf2Coef tc = tin.coef[y % tin.nt];
    if (y / tin.nt != seg) {
      seg = y / tin.nt;
      const float2* qs = tin.q + int64_t(seg) * (tin.jhi - tin.jlo + 1);
#pragma unroll
      for (int i = 0; i < R1; ++i) {
        aq[i] = V{0.f, 0.f};
        if (gx[i] > 0.0) {
          const int32_t fj = j + (u + i * QA) * ncols;
          const float2 q = qs[fj - tin.jlo];
          const float a0 = float(tg) / (float(double(fj) * tin.df) * sqrtf(float(gx[i])));
          aq[i] = V{a0 * q.x, a0 * q.y};
        }
      }
    }
    V v[R1];
#pragma unroll
    for (int i = 0; i < R1; ++i) {
      v[i] = V{0.f, 0.f};
      if (gx[i] > 0.0) {
        double x = gx[i], ix = gi[i], lf = gl[i];
        // at 4096 points the products of x, 1 / x and ln f are formed again for
        // every template rather than held across the loop: 1024 threads a
        // workgroup leave 128 registers a thread
        if constexpr (PA >= 4096) asm volatile("" : "+v"(x), "+v"(ix), "+v"(lf));
        const double ix2 = ix * ix, ix3 = ix2 * ix;
        double psi = fma(tc.e5, ix3 * ix2, tc.e0);
        psi = fma(tc.e3, ix3, psi);
        psi = fma(tc.e2, ix2, psi);
        psi = fma(tc.e1, ix, psi);
        psi = fma(tc.el, lf, psi);
        psi = fma(tc.ex, x, psi);
        psi = fma(tc.exl, x * lf, psi);
        psi = fma(tc.exx, x * x, psi);
        float sn, cs;
        phase_exp(psi, &sn, &cs);
        v[i] = cmul(aq[i], V{cs, sn});
      }
    }
    Dft<V, R1>::run(v);
#pragma unroll
    for (int q = 0; q < R1; ++q) s[0][sw(R1 * u + q)] = v[q];
    __syncthreads();
    lds_stage<PA, 1, NT, R1, R2, ST>(s, tw);
    lds_stage<PA, 1, NT, R1 * R2, R3, ST>(s, tw);
    // last stage (NS = NS4, radix R4): butterflies b = u + k NT, outputs b + q NS4
    float2* o = out + int64_t(y) * n + int64_t(j) * PA;
#pragma unroll
    for (int k = 0; k < KL; ++k) {
      const int b = u + k * NT;
      if (NL % NT != 0 && b >= NL) break;
      V w[R4];
#pragma unroll
      for (int q = 0; q < R4; ++q) w[q] = s[0][sw(b + q * NS4)];
#pragma unroll
      for (int q = 1; q < R4; ++q) w[q] = cmul(w[q], tw[q * b]);
      Dft<V, R4>::run(w);
#pragma unroll
      for (int q = 0; q < R4; ++q) o[b + q * NS4] = w[q];
    }
    __syncthreads();
  }
}

// Pass B of the two-pass form (ns = n / P columns of P = 1024 or 2048 points):
// C = 16 or 8 columns j per workgroup, 1024 threads; thread (c, u) = (threadIdx %
// C, threadIdx / C), u < U = P / 16, loads elements u + U i (i < 16) of column j,
// applies the inter-pass twiddles, a radix-16 butterfly, one radix-16 stage in
// LDS and a radix-(P / 256) last stage whose outputs u + U k + 256 q it stores to
// out[j + e ns], or reads out (RO, trigger records raw until trig_finish).  With
// 8 columns (64 bytes of a row) per workgroup, each XCD takes a contiguous range
// of column groups, so the two halves of a 128-byte line go to one L2 together.
template <int P> struct WideB {
  static constexpr int C = 16384 / P, U = P / 16, R3 = P / 256, K = 256 / U;
  static constexpr int ST = P + P / 32 + 1;
};
template <int P, bool RO>
__global__ __launch_bounds__(1024) void k_pass_wide(const float2* __restrict__ in, float2* __restrict__ out,
                                                    int32_t n, PeakOut po) {
  using V = float2;
  using W = WideB<P>;
  constexpr int C = W::C, U = W::U, R3 = W::R3, K = W::K, NT = 1024;
  static_assert(C * U == NT && U * K == 256 && 256 * R3 == P, "pass B shape");
  __shared__ V s[C][W::ST];
  __shared__ V tw[P];
  const int32_t ns = n / P;                          // = columns of this pass
  const int c = int(threadIdx.x) % C, u = int(threadIdx.x) / C;
  int32_t grp = int32_t(blockIdx.x);
  if (C < 16) grp = int32_t(blockIdx.x % 8u) * int32_t(gridDim.x / 8u) + int32_t(blockIdx.x / 8u);
  const int32_t j = grp * C + c;
  in += int64_t(blockIdx.y) * n;
  if (!RO) out += int64_t(blockIdx.y) * n;
  for (int m = int(threadIdx.x); m < P; m += NT) {
    float sn, cs;
    sincospi_f32(float(2 * m) / float(P), &sn, &cs);
    tw[m] = V{cs, sn};
  }
  V v[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = in[j + (u + i * U) * ns];
  // w_n^(r j), r = u + U i; j < ns so j mod ns = j; 2 / n is exact
  apply_twiddles<16, U>(v, uint32_t(u), uint32_t(j), 2.f / float(n));
  Dft<V, 16>::run(v);
#pragma unroll
  for (int q = 0; q < 16; ++q) s[c][sw(16 * u + q)] = v[q];
  __syncthreads();
  lds_stage<P, C, NT, 16, 16, W::ST>(s, tw);
  // last stage (NS = 256, radix R3): butterflies b = u + U k (k < K) of column c
  V w[K][R3];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int b = u + U * k;
#pragma unroll
    for (int q = 0; q < R3; ++q) w[k][q] = s[c][sw(b + q * 256)];
#pragma unroll
    for (int q = 1; q < R3; ++q) w[k][q] = cmul(w[k][q], tw[q * b]);
    Dft<V, R3>::run(w[k]);
  }
  if constexpr (RO) {
    Best best{-1.f, INT32_MAX};
#pragma unroll
    for (int q = 0; q < R3; ++q)
#pragma unroll
      for (int k = 0; k < K; ++k)
        peak_visit_rising_raw(best, w[k][q].x, w[k][q].y, j + (u + U * k + 256 * q) * ns, po);
    peak_commit(best, po);
  } else {
#pragma unroll
    for (int q = 0; q < R3; ++q)
#pragma unroll
      for (int k = 0; k < K; ++k) out[j + (u + U * k + 256 * q) * ns] = w[k][q];
  }
}

// the two-pass form applies to n = 2^20 ... 2^23
bool wide_tmpl(int64_t n) { return n >= (int64_t(1) << 20) && n <= (int64_t(1) << 23); }

// second-pass length: 1024 points up to n = 2^21, 2048 above
int64_t wide_pb(int64_t n) { return n <= (int64_t(1) << 21) ? 1024 : 2048; }

void launch_tmpl_wide(float2* mid, const float2* mid_in, float2* out, int64_t n, int batch, hipStream_t st,
                      const TmplIn& tin, const PeakOut* ro) {
  const int64_t PB = wide_pb(n), PA = n / PB;
  RF_CHECK(PB % 8 == 0 && (PA / WideB<2048>::C) % 8 == 0, "fft: two-pass form needs a multiple of 8 columns");
  dim3 ga(unsigned(PB), unsigned((batch + kTmplPerBlock - 1) / kTmplPerBlock));
  switch (PA) {
#define RF_WIDE_CASE(P)                                                                                 \
  case P:                                                                                               \
    hipLaunchKernelGGL((k_tmpl_wide<P, kTmplPerBlock>), ga, dim3(P / WideA<P>::R1), 0, st, mid, int32_t(n), \
                       batch, tin);                                                                     \
    break;
    RF_WIDE_CASE(1024)
    RF_WIDE_CASE(2048)
    RF_WIDE_CASE(4096)
#undef RF_WIDE_CASE
    default:
      throw Error{RF_E_UNSUPPORTED, "fft: unsupported two-pass size"};
  }
  RF_HIP(hipGetLastError());
  if (PB == 1024) {
    dim3 gb(unsigned(PA / WideB<1024>::C), unsigned(batch));
    if (ro)
      hipLaunchKernelGGL((k_pass_wide<1024, true>), gb, dim3(1024), 0, st, mid_in, nullptr, int32_t(n), *ro);
    else
      hipLaunchKernelGGL((k_pass_wide<1024, false>), gb, dim3(1024), 0, st, mid_in, out, int32_t(n), PeakOut{});
  } else {
    dim3 gb(unsigned(PA / WideB<2048>::C), unsigned(batch));
    if (ro)
      hipLaunchKernelGGL((k_pass_wide<2048, true>), gb, dim3(1024), 0, st, mid_in, nullptr, int32_t(n), *ro);
    else
      hipLaunchKernelGGL((k_pass_wide<2048, false>), gb, dim3(1024), 0, st, mid_in, out, int32_t(n), PeakOut{});
  }
  RF_HIP(hipGetLastError());
}

// Split log2(n) into at least two passes of at most 8 bits each (16 columns per
// workgroup need n / P >= 16 in every pass).  FP64: as even as possible.  FP32:
// as many 256-point passes as fit, the remainder in the first pass (where the
// matched filters form their spectra: fewer elements per thread there keep the
// per-bin phase parts in registers at full occupancy), at least 16 points.
std::vector<int> plan_passes(int lg, bool small_first) {
  int s = (lg + 7) / 8;
  if (s < 2) s = 2;
  std::vector<int> bits(s, lg / s);
  if (!small_first) {
    for (int i = 0; i < lg % s; ++i) bits[i] += 1;
    return bits;
  }
  for (int i = 0; i < s; ++i) bits[i] = 8;
  int excess = 8 * s - lg;
  for (int i = 0; excess > 0; i = (i + 1) % s) {
    const int d = std::min(excess, bits[i] - 4);
    bits[i] -= d;
    excess -= d;
  }
  return bits;
}

void launch_pass64(int bits, const double2* in, double2* out, int64_t n, int64_t ns, int batch,
                   hipStream_t st) {
  const int64_t P = int64_t(1) << bits;
  dim3 grid(unsigned((n / P) / kCols), unsigned(batch));
  switch (bits) {
#define RF_FFT_CASE(B)                                                                                  \
  case B:                                                                                               \
    hipLaunchKernelGGL((k_fft_pass<double, (1 << B)>), grid, dim3(kThreads), 0, st, in, out, n, ns);   \
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

template <int MODE = kPlain, bool RO = false>
void launch_pass32(int bits, const float2* in, float2* out, int64_t n, int64_t ns, int batch, hipStream_t st,
                   BandIn bin = BandIn{}, PeakOut po = PeakOut{}) {
  const int64_t cols = n >> bits;
  const bool wide = cols % 32 == 0;
  RF_CHECK(cols % 16 == 0, "fft: fewer columns than a workgroup takes");
  dim3 grid(unsigned(cols / (wide ? 32 : 16)), unsigned(batch));
  switch (bits * 2 + (wide ? 1 : 0)) {
#define RF_FFT_CASE(B, C)                                                                               \
  case B * 2 + (C == 32 ? 1 : 0):                                                                       \
    hipLaunchKernelGGL((k_pass32<(1 << B), C, MODE, RO>), grid, dim3(threads32<(1 << B), C>()), 0, st,  \
                       in, out, int32_t(n), int32_t(ns), bin, po);                                      \
    break;
    RF_FFT_CASE(4, 16)
    RF_FFT_CASE(5, 16)
    RF_FFT_CASE(6, 16)
    RF_FFT_CASE(7, 16)
    RF_FFT_CASE(8, 16)
    RF_FFT_CASE(4, 32)
    RF_FFT_CASE(5, 32)
    RF_FFT_CASE(6, 32)
    RF_FFT_CASE(7, 32)
    RF_FFT_CASE(8, 32)
#undef RF_FFT_CASE
    default:
      throw Error{RF_E_UNSUPPORTED, "fft: unsupported pass size"};
  }
  RF_HIP(hipGetLastError());
}


void launch_tmpl_pass(int bits, float2* out, int64_t n, int batch, hipStream_t st, const TmplIn& tin) {
  const int64_t cols = n >> bits;
  const bool wide = cols % 32 == 0;
  RF_CHECK(cols % 16 == 0, "fft: fewer columns than a workgroup takes");
  dim3 grid(unsigned(cols / (wide ? 32 : 16)), unsigned((batch + kTmplPerBlock - 1) / kTmplPerBlock));
  switch (bits * 2 + (wide ? 1 : 0)) {
#define RF_TMPL_CASE(B, C)                                                                              \
  case B * 2 + (C == 32 ? 1 : 0):                                                                       \
    hipLaunchKernelGGL((k_fft_tmpl_pass<(1 << B), C, kTmplPerBlock>), grid, dim3(threads32<(1 << B), C>()), \
                       0, st, out, int32_t(n), batch, tin);                                             \
    break;
    RF_TMPL_CASE(4, 16)
    RF_TMPL_CASE(5, 16)
    RF_TMPL_CASE(6, 16)
    RF_TMPL_CASE(7, 16)
    RF_TMPL_CASE(8, 16)
    RF_TMPL_CASE(4, 32)
    RF_TMPL_CASE(5, 32)
    RF_TMPL_CASE(6, 32)
    RF_TMPL_CASE(7, 32)
    RF_TMPL_CASE(8, 32)
#undef RF_TMPL_CASE
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
  if constexpr (std::is_same<T, float>::value) {
    if (tmpl && wide_tmpl(n)) {        // two passes through one intermediate
      V* mid = wsa_in ? wsa_in : static_cast<V*>(ctx->ws[WS_FFT_A].ensure(sizeof(V) * size_t(n) * batch));
      launch_tmpl_wide(mid, mid, out, n, batch, ctx->stream, *tmpl, ro);
      return;
    }
  }
  std::vector<int> bits = plan_passes(lg, std::is_same<T, float>::value);
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
      if (i == 0 && band) {
        launch_pass32<kBand>(bits[i], nullptr, dst, n, ns, batch, ctx->stream, *band);
      } else if (i == 0 && tmpl) {
        launch_tmpl_pass(bits[i], dst, n, batch, ctx->stream, *tmpl);
      } else if (i == s - 1 && ro) {   // the last pass reads the outputs out instead
        launch_pass32<kPlain, true>(bits[i], src, nullptr, n, ns, batch, ctx->stream, BandIn{}, *ro);
        break;
      } else {
        launch_pass32(bits[i], src, dst, n, ns, batch, ctx->stream);
      }
    } else {
      launch_pass64(bits[i], src, dst, n, ns, batch, ctx->stream);
    }
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
