// Learned ratio kernels: a small MLP maps the chirp-time coordinates of a
// (reference, neighbour) pair to the coefficients of the pair's analytic ratio
// kernel in a basis built from exact kernels; the exact FP64 build is both the
// training data and the fallback.
//
//   analytic kernel  h[m] = (1/nb) sum_{j <= nb/2} c_j R~_j e^{2 pi i j m / nb},
//                    c_0 = c_{nb/2} = 1, else 2, so that w = Re h is the real
//                    ratio kernel of sections II.B-II.C;
//   basis            U: the leading left singular vectors of [h_1 ... h_P] on the
//                    tap window (-L/2, L/2] (randomized range finder, Gaussian
//                    draws supplied by the caller, twice-applied Cholesky-QR);
//   coefficients     c_p = U^H h_p (rank complex values);
//   network          x (4 standardised features) -> 3 x 256 GELU -> 2 rank reals;
//   inference        w_k = Re(U c_k) on the window, truncated like the exact
//                    kernel, with a check segment deciding the fallback.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <functional>
#include <numeric>

#include "recon.h"

namespace rf {
namespace mlpdef {
constexpr int kIn = 4, kHid = 256, kOut = 128;
// packed parameter offsets: W [out][in] row-major then b [out], per layer
constexpr int kW0 = 0, kB0 = kW0 + kHid * kIn;
constexpr int kW1 = kB0 + kHid, kB1 = kW1 + kHid * kHid;
constexpr int kW2 = kB1 + kHid, kB2 = kW2 + kHid * kHid;
constexpr int kW3 = kB2 + kHid, kB3 = kW3 + kOut * kHid;
constexpr int kParams = kB3 + kOut;
static_assert(kParams == 165760, "parameter count");
}  // namespace mlpdef
}  // namespace rf

struct rf_surrogate {
  int device = 0;
  rf_grid grid{};                 // training grid (grid.n = training build length)
  int32_t window = 0, rank = 0, npair = 0, kr = 0;   // kr: numerical rank kept
  double2* U = nullptr;           // device [window][rank], rows in FFT order of m
  double feat_mean[4] = {0, 0, 0, 0}, feat_std[4] = {1, 1, 1, 1};
  double out_scale = 1.0;
  std::vector<double> svals;      // singular values of the training kernels (kr)
  float* X = nullptr;             // [npair][4]
  float* T = nullptr;             // [npair][2 rank]
  float* theta = nullptr;         // parameters, gradient, Adam moments
  float* grad = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  // training state
  int32_t B = 0;
  float* xb = nullptr;            // [B][4]
  float* tb = nullptr;            // [B][128]
  float* pre[3] = {nullptr, nullptr, nullptr};   // [B][256]
  float* act[3] = {nullptr, nullptr, nullptr};   // [B][256]
  float* out = nullptr;           // [B][128]
  float* d0 = nullptr;            // [B][256] scratch gradients
  float* d1 = nullptr;
  float* lpart = nullptr;         // loss partial sums
  float* loss_hist = nullptr;
  int64_t hist_cap = 0;
  int32_t* counter = nullptr;     // training step (device)
  const int32_t* order = nullptr; // borrowed batch order of the current training call
  hipGraphExec_t exec = nullptr;
  int32_t graph_steps = 0, graph_batch = 0;   // shape the training graph was captured for
  int64_t steps_total = 0;        // Adam steps since the parameters were last set
  float lr = 0.f;
};

namespace rf {
namespace {

inline unsigned gblocks(int64_t n, unsigned cap = 4096) {
  int64_t b = (n + 255) / 256;
  return unsigned(std::max<int64_t>(1, std::min<int64_t>(b, cap)));
}

// ------------------------------------------------------------ complex FP64 GEMM
// C[M][N] = sum_k opA(i, k) opB(k, j).  opA(i, k) = A[i*lda + k] (ta = 0) or
// A[k*lda + i] (ta = 1), conjugated when ca; likewise opB(k, j) = B[k*ldb + j]
// (tb = 0) or B[j*ldb + k] (tb = 1), conjugated when cb.  32 x 32 tiles.
__global__ __launch_bounds__(256) void k_zgemm(const double2* __restrict__ A, int64_t lda, int ta, int ca,
                                               const double2* __restrict__ Bm, int64_t ldb, int tb, int cb,
                                               double2* __restrict__ C, int64_t ldc, int64_t M, int64_t N,
                                               int64_t K) {
  __shared__ double2 as[16][33];
  __shared__ double2 bs[16][33];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t i0 = int64_t(blockIdx.y) * 32, j0 = int64_t(blockIdx.x) * 32;
  double2 acc[2][2] = {{{0, 0}, {0, 0}}, {{0, 0}, {0, 0}}};
  for (int64_t k0 = 0; k0 < K; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 32; e += 256) {
      const int kk = e / 32, r = e % 32;
      const int64_t i = i0 + r, k = k0 + kk;
      double2 a = {0, 0};
      if (i < M && k < K) a = ta ? A[k * lda + i] : A[i * lda + k];
      if (ca) a.y = -a.y;
      as[kk][r] = a;
      const int64_t j = j0 + r;
      double2 b = {0, 0};
      if (j < N && k < K) b = tb ? Bm[j * ldb + k] : Bm[k * ldb + j];
      if (cb) b.y = -b.y;
      bs[kk][r] = b;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const double2 a = as[kk][ty * 2 + x];
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const double2 b = bs[kk][tx * 2 + y];
          acc[x][y].x += a.x * b.x - a.y * b.y;
          acc[x][y].y += a.x * b.y + a.y * b.x;
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int64_t i = i0 + ty * 2 + x, j = j0 + tx * 2 + y;
      if (i < M && j < N) C[i * ldc + j] = acc[x][y];
    }
}

void zgemm(rf_ctx* ctx, const double2* A, int64_t lda, int ta, int ca, const double2* B, int64_t ldb,
           int tb, int cb, double2* C, int64_t ldc, int64_t M, int64_t N, int64_t K) {
  RF_CHECK(M <= int64_t(65535) * 32, "zgemm: M too large");
  dim3 grid(unsigned((N + 31) / 32), unsigned((M + 31) / 32));
  hipLaunchKernelGGL(k_zgemm, grid, dim3(256), 0, ctx->stream, A, lda, ta, ca, B, ldb, tb, cb, C, ldc, M,
                     N, K);
  RF_HIP(hipGetLastError());
}

// ------------------------------------------------------------ FP32 GEMM (MLP)
// C[M][N] = op(A)[M][K] op(B)[K][N]; op(A) = A [M][K] (ta = 0) or A^T with A
// stored [K][M]; op(B) = B [K][N] (tb = 0) or B^T with B stored [N][K].
// Epilogue: bias[N] added when bias != NULL; when act != NULL, C holds the
// pre-activation and act = gelu(C).  64 x 64 tiles staged through LDS in
// 16-deep slices; each wavefront owns a 32 x 32 quarter on the FP32 matrix
// cores (v_mfma_f32_32x32x2f32: FP32 products and sums, two k per
// instruction).
__device__ inline float gelu_f(float u) { return 0.5f * u * (1.f + erff(u * 0.70710678118654752f)); }
__device__ inline float gelu_grad_f(float u) {
  return 0.5f * (1.f + erff(u * 0.70710678118654752f)) + u * 0.39894228040143268f * expf(-0.5f * u * u);
}

__global__ __launch_bounds__(256) void k_sgemm(const float* __restrict__ A, int ta, const float* __restrict__ Bm,
                                               int tb, float* __restrict__ C, const float* __restrict__ bias,
                                               float* __restrict__ act, int M, int N, int K) {
  __shared__ float as[16][68];
  __shared__ float bs[16][68];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;   // the wave's quarter
  const int i0 = blockIdx.y * 64, j0 = blockIdx.x * 64;
  floatx16 acc = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int kk = e / 64, r = e % 64;
      const int i = i0 + r, k = k0 + kk, j = j0 + r;
      as[kk][r] = (i < M && k < K) ? (ta ? A[size_t(k) * M + i] : A[size_t(i) * K + k]) : 0.f;
      bs[kk][r] = (j < N && k < K) ? (tb ? Bm[size_t(j) * K + k] : Bm[size_t(k) * N + j]) : 0.f;
    }
    __syncthreads();
    // lane l supplies A[wr + l % 32][kk + l / 32] and B[kk + l / 32][wc + l % 32]
#pragma unroll
    for (int kk = 0; kk < 16; kk += 2)
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(as[kk + (lane >> 5)][wr + (lane & 31)],
                                                 bs[kk + (lane >> 5)][wc + (lane & 31)], acc, 0, 0, 0);
    __syncthreads();
  }
  // accumulator element e of lane l: row acc_row(e, l), column l % 32 of the quarter
  const int j = j0 + wc + (lane & 31);
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int i = i0 + wr + acc_row(e, lane);
    if (i < M && j < N) {
      const float v = acc[e] + (bias ? bias[j] : 0.f);
      C[size_t(i) * N + j] = v;
      if (act) act[size_t(i) * N + j] = gelu_f(v);
    }
  }
}

void sgemm(rf_ctx* ctx, const float* A, int ta, const float* B, int tb, float* C, const float* bias,
           float* act, int M, int N, int K) {
  dim3 grid(unsigned((N + 63) / 64), unsigned((M + 63) / 64));
  hipLaunchKernelGGL(k_sgemm, grid, dim3(256), 0, ctx->stream, A, ta, B, tb, C, bias, act, M, N, K);
  RF_HIP(hipGetLastError());
}

// d[i] *= gelu'(pre[i])
__global__ void k_gelu_back(float* __restrict__ d, const float* __restrict__ pre, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    d[i] *= gelu_grad_f(pre[i]);
}

// gb[j] = sum_b d[b][j]
__global__ void k_colsum(const float* __restrict__ d, float* __restrict__ gb, int rows, int cols) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= cols) return;
  float s = 0.f;
  for (int b = 0; b < rows; ++b) s += d[size_t(b) * cols + j];
  gb[j] = s;
}

// dout = 2 (out - t) / (rows * cols); per-block partial sums of (out - t)^2
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ out, const float* __restrict__ t,
                                             float* __restrict__ dout, float* __restrict__ part, int64_t n) {
  __shared__ float sh[256];
  float s = 0.f;
  const float sc = 2.f / float(n);
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const float e = out[i] - t[i];
    if (dout) dout[i] = sc * e;
    s += e * e;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (int(threadIdx.x) < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

constexpr int kMseBlocks = 64;

// loss = sum(part) / n, written to hist[*counter] (and hist_base[0] when no counter)
__global__ void k_loss_final(const float* __restrict__ part, int np, int64_t n, float* hist,
                             const int32_t* counter) {
  __shared__ float sh[64];
  sh[threadIdx.x] = int(threadIdx.x) < np ? part[threadIdx.x] : 0.f;
  __syncthreads();
  for (int k = 32; k > 0; k >>= 1) {
    if (int(threadIdx.x) < k) sh[threadIdx.x] += sh[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) hist[counter ? *counter : 0] = sh[0] / float(n);
}

// gather the batch of the current step: rows order[step * B + b] of X and T
__global__ void k_gather(const float* __restrict__ X, const float* __restrict__ T,
                         const int32_t* __restrict__ order, const int32_t* __restrict__ counter, int B,
                         float* __restrict__ xb, float* __restrict__ tb) {
  const int b = blockIdx.x;
  const int64_t row = order[int64_t(*counter) * B + b];
  for (int j = threadIdx.x; j < mlpdef::kOut; j += blockDim.x) tb[size_t(b) * mlpdef::kOut + j] = T[row * mlpdef::kOut + j];
  if (threadIdx.x < mlpdef::kIn) xb[size_t(b) * mlpdef::kIn + threadIdx.x] = X[row * mlpdef::kIn + threadIdx.x];
}

// Adam with bias correction and a cosine learning-rate schedule over `total` steps
__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, const int32_t* __restrict__ counter, int64_t n, float lr0,
                       int64_t total) {
  // counter[0]: step within this schedule; counter[1]: Adam steps since the moments were reset
  const float lr = lr0 * 0.5f * (1.f + cospif(float(counter[0]) / float(total)));
  const int t = counter[1] + 1;
  const float c1 = 1.f - powf(0.9f, float(t)), c2 = 1.f - powf(0.999f, float(t));
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
  }
}

__global__ void k_count(int32_t* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    counter[0] += 1;
    counter[1] += 1;
  }
}

// ------------------------------------------------------------ dataset helpers
// rows of the complex FFT output (FFT order, nb points) gathered on the tap window
// (-L/2, L/2] in the same wrapped order: H[p][q] holds signed tap q for q <= L/2 and
// tap q - L above (the signed-tap convention of the support scan)
__global__ void k_window(const double2* __restrict__ out, int64_t nb, int L, double2* __restrict__ H) {
  const int p = blockIdx.y;
  for (int q = blockIdx.x * 256 + threadIdx.x; q < L; q += gridDim.x * 256) {
    const int64_t m = q <= L / 2 ? q : int64_t(q) - L;         // signed tap
    H[int64_t(p) * L + q] = out[int64_t(p) * nb + (m & (nb - 1))];
  }
}

// coefficients (complex [n][rank]) -> targets [n][2 rank] (re..., im...) / scale
__global__ void k_to_targets(const double2* __restrict__ c, int n, int rank, double inv_scale,
                             float* __restrict__ T) {
  const int p = blockIdx.x;
  if (p >= n) return;
  for (int j = threadIdx.x; j < rank; j += blockDim.x) {
    const double2 v = c[int64_t(p) * rank + j];
    T[int64_t(p) * 2 * rank + j] = float(v.x * inv_scale);
    T[int64_t(p) * 2 * rank + rank + j] = float(v.y * inv_scale);
  }
}

// network outputs [n][2 rank] -> complex coefficients [n][rank] * scale
__global__ void k_from_outputs(const float* __restrict__ o, int n, int rank, double scale,
                               double2* __restrict__ c) {
  const int p = blockIdx.x;
  if (p >= n) return;
  for (int j = threadIdx.x; j < rank; j += blockDim.x)
    c[int64_t(p) * rank + j] = make_double2(double(o[int64_t(p) * 2 * rank + j]) * scale,
                                            double(o[int64_t(p) * 2 * rank + rank + j]) * scale);
}

// Residual codes of one kernel's coefficients (one block per kernel):
// r = c - p (p the network's prediction, or zero), scale = max |Re r|, |Im r|
// over the kernel's 2 rank reals / qmax (as float), code = round(r / scale)
// clamped to [-qmax, qmax]; real parts first, then imaginary parts.
template <typename Q>
__global__ __launch_bounds__(128) void k_encode(const double2* __restrict__ c, const double2* __restrict__ p,
                                                int rank, int qmax, Q* __restrict__ codes,
                                                float* __restrict__ scales) {
  __shared__ double sh[128];
  const int k = blockIdx.x;
  double mx = 0.0;
  for (int j = threadIdx.x; j < rank; j += blockDim.x) {
    double2 r = c[int64_t(k) * rank + j];
    if (p) {
      r.x -= p[int64_t(k) * rank + j].x;
      r.y -= p[int64_t(k) * rank + j].y;
    }
    mx = fmax(mx, fmax(fabs(r.x), fabs(r.y)));
  }
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 64; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  const float sc = float(sh[0] / double(qmax));
  if (threadIdx.x == 0) scales[k] = sc;
  const double inv = sc > 0.f ? 1.0 / double(sc) : 0.0;
  for (int j = threadIdx.x; j < rank; j += blockDim.x) {
    double2 r = c[int64_t(k) * rank + j];
    if (p) {
      r.x -= p[int64_t(k) * rank + j].x;
      r.y -= p[int64_t(k) * rank + j].y;
    }
    const double qa = fmin(fmax(rint(r.x * inv), -double(qmax)), double(qmax));
    const double qb = fmin(fmax(rint(r.y * inv), -double(qmax)), double(qmax));
    codes[int64_t(k) * 2 * rank + j] = Q(qa);
    codes[int64_t(k) * 2 * rank + rank + j] = Q(qb);
  }
}

// c = p + code * scale (p the prediction, or zero)
template <typename Q>
__global__ void k_decode(const Q* __restrict__ codes, const float* __restrict__ scales,
                         const double2* __restrict__ p, int rank, double2* __restrict__ c) {
  const int k = blockIdx.x;
  const double sc = double(scales[k]);
  for (int j = threadIdx.x; j < rank; j += blockDim.x) {
    double2 v = make_double2(double(codes[int64_t(k) * 2 * rank + j]) * sc,
                             double(codes[int64_t(k) * 2 * rank + rank + j]) * sc);
    if (p) {
      v.x += p[int64_t(k) * rank + j].x;
      v.y += p[int64_t(k) * rank + j].y;
    }
    c[int64_t(k) * rank + j] = v;
  }
}

// max_m |a[k][m] - b[k][m]| per row (complex64), one block per row
__global__ __launch_bounds__(256) void k_rowmaxdiff(const float2* __restrict__ a, const float2* __restrict__ b,
                                                    int64_t n, float* __restrict__ out) {
  __shared__ float sh[256];
  const int64_t off = int64_t(blockIdx.x) * n;
  float mx = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const float2 x = a[off + i], y = b[off + i];
    mx = fmaxf(mx, hypotf(x.x - y.x, x.y - y.y));
  }
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (int(threadIdx.x) < k) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

// ------------------------------------------------------------ host linear algebra
using cd = std::complex<double>;

// Eigen-decomposition of a Hermitian n x n matrix (row-major) by cyclic complex
// Jacobi rotations: A = V diag(w) V^H, eigenvalues descending.
void herm_eig(std::vector<cd> A, int n, std::vector<double>& w, std::vector<cd>& V) {
  V.assign(size_t(n) * n, cd(0, 0));
  for (int i = 0; i < n; ++i) V[size_t(i) * n + i] = 1.0;
  auto a = [&](int i, int j) -> cd& { return A[size_t(i) * n + j]; };
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0, tot = 0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        const double v = std::norm(a(i, j));
        tot += v;
        if (i != j) off += v;
      }
    if (off <= 1e-30 * tot || off == 0) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        const cd apq = a(p, q);
        const double r = std::abs(apq);
        if (r == 0.0) continue;
        const cd ph = apq / r;                                  // e^{i phi}
        const double app = a(p, p).real(), aqq = a(q, q).real();
        // real symmetric 2x2 [[app, r], [r, aqq]] after the phase change of column q
        const double theta = 0.5 * std::atan2(2.0 * r, aqq - app);
        const double c = std::cos(theta), s = std::sin(theta);
        // G acts on columns p, q: col_p' = c col_p - s conj(ph) col_q ... built so that (G^H A G)_pq = 0
        const cd gpp = c, gpq = s * ph, gqp = -s * std::conj(ph), gqq = c;
        for (int k = 0; k < n; ++k) {        // A <- A G (columns)
          const cd akp = a(k, p), akq = a(k, q);
          a(k, p) = akp * gpp + akq * gqp;
          a(k, q) = akp * gpq + akq * gqq;
        }
        for (int k = 0; k < n; ++k) {        // A <- G^H A (rows)
          const cd apk = a(p, k), aqk = a(q, k);
          a(p, k) = std::conj(gpp) * apk + std::conj(gqp) * aqk;
          a(q, k) = std::conj(gpq) * apk + std::conj(gqq) * aqk;
        }
        for (int k = 0; k < n; ++k) {        // V <- V G
          const cd vkp = V[size_t(k) * n + p], vkq = V[size_t(k) * n + q];
          V[size_t(k) * n + p] = vkp * gpp + vkq * gqp;
          V[size_t(k) * n + q] = vkp * gpq + vkq * gqq;
        }
      }
  }
  std::vector<int> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  std::vector<double> d(n);
  for (int i = 0; i < n; ++i) d[i] = a(i, i).real();
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] > d[y]; });
  w.resize(n);
  std::vector<cd> Vs(size_t(n) * n);
  for (int c = 0; c < n; ++c) {
    w[c] = d[idx[c]];
    for (int k = 0; k < n; ++k) Vs[size_t(k) * n + c] = V[size_t(k) * n + idx[c]];
  }
  V.swap(Vs);
}

std::vector<cd> to_host(rf_ctx* ctx, const double2* d, size_t n) {
  std::vector<double2> h(n);
  copy_sync(ctx, h.data(), d, sizeof(double2) * n, hipMemcpyDeviceToHost);
  std::vector<cd> out(n);
  for (size_t i = 0; i < n; ++i) out[i] = cd(h[i].x, h[i].y);
  return out;
}
double2* to_dev(rf_ctx* ctx, const std::vector<cd>& v) {
  std::vector<double2> h(v.size());
  for (size_t i = 0; i < v.size(); ++i) h[i] = make_double2(v[i].real(), v[i].imag());
  double2* d = dev_alloc<double2>(v.size(), "surrogate: device allocation failed");
  copy_sync(ctx, d, h.data(), sizeof(double2) * v.size(), hipMemcpyHostToDevice);
  return d;
}

// chirp-time features of a pair: (tau0_ref, tau3_ref, tau0_k - tau0_ref, tau3_k - tau3_ref) at f0
void features(const rf_tmpl& ref, const rf_tmpl& k, double f0, double* x) {
  auto ct = [&](const rf_tmpl& t, double* t0, double* t3) {
    const double mt = (t.m1 + t.m2) * 4.925490947641267e-6;
    const double eta = t.m1 * t.m2 / ((t.m1 + t.m2) * (t.m1 + t.m2));
    const double v = 3.14159265358979323846 * mt * f0;
    *t0 = 5.0 / (256.0 * 3.14159265358979323846 * f0 * eta) * std::pow(v, -5.0 / 3.0);
    *t3 = 1.0 / (8.0 * f0 * eta) * std::pow(v, -2.0 / 3.0);
  };
  double r0, r3, k0, k3;
  ct(ref, &r0, &r3);
  ct(k, &k0, &k3);
  x[0] = r0;
  x[1] = r3;
  x[2] = k0 - r0;
  x[3] = k3 - r3;
}

// Exact analytic kernels h of the pairs (refs[p], nbrs[p]) built on `grid`
// (FP64 ratio spectrum, one-sided complex inverse FFT of length grid->n) and
// gathered on the tap window: H [npair][L].
void window_kernels(rf_ctx* ctx, const rf_grid* grid, const rf_tmpl* refs, const rf_tmpl* nbrs, int npair,
                    int L, double2* H) {
  const int64_t nb = grid->n;
  const int per = int(std::max<int64_t>(1, std::min<int64_t>(npair, (int64_t(1) << 25) / nb)));
  double2* spec = static_cast<double2*>(ctx->ws[WS_BUILD].ensure(sizeof(double2) * size_t(nb) * per));
  double2* wout = static_cast<double2*>(ctx->ws[WS_Y].ensure(sizeof(double2) * size_t(nb) * per));
  Tf2Coef* cdev = static_cast<Tf2Coef*>(ctx->ws[WS_TGT].ensure((sizeof(Tf2Coef) * 2 + sizeof(RatioParam)) * per));
  Tf2Coef* tdev = cdev + per;
  RatioParam* pdev = reinterpret_cast<RatioParam*>(tdev + per);
  std::vector<Tf2Coef> rc(per), tc(per);
  std::vector<RatioParam> pr(per);
  for (int p0 = 0; p0 < npair; p0 += per) {
    const int cnt = std::min(per, npair - p0);
    for (int i = 0; i < cnt; ++i) {
      RF_CHECK(refs[p0 + i].m1 > 0 && refs[p0 + i].m2 > 0 && nbrs[p0 + i].m1 > 0 && nbrs[p0 + i].m2 > 0,
               "surrogate: masses must be positive");
      rc[i] = tf2_coef(refs[p0 + i]);
      tc[i] = tf2_coef(nbrs[p0 + i]);
      const double d = std::fabs(tf2_dtdf(tc[i], grid->f_low) - tf2_dtdf(rc[i], grid->f_low));
      const double dfl = d > 0 ? 1.0 / std::sqrt(d) : grid->df_low_max;
      pr[i].df_low = std::min(dfl, grid->df_low_max);
      pr[i].amp_ratio = tc[i].amp / rc[i].amp;
    }
    copy_sync(ctx, cdev, rc.data(), sizeof(Tf2Coef) * cnt, hipMemcpyHostToDevice);
    copy_sync(ctx, tdev, tc.data(), sizeof(Tf2Coef) * cnt, hipMemcpyHostToDevice);
    copy_sync(ctx, pdev, pr.data(), sizeof(RatioParam) * cnt, hipMemcpyHostToDevice);
    // the spectrum kernel takes one reference per launch: one launch per pair
    for (int i = 0; i < cnt; ++i)
      ratio_spectrum(ctx, grid, nb, cdev + i, tdev + i, pdev + i, spec + int64_t(i) * nb, 1);
    fft_inverse_f64(ctx, spec, wout, nb, cnt);
    hipLaunchKernelGGL(k_window, dim3(gblocks(L, 256), unsigned(cnt)), dim3(256), 0, ctx->stream, wout, nb, L,
                       H + int64_t(p0) * L);
    RF_HIP(hipGetLastError());
    RF_HIP(hipStreamSynchronize(ctx->stream));   // host parameter arrays are reused
  }
}

void free_surrogate(rf_surrogate* s) {
  if (!s) return;
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  for (void* p : {(void*)s->U, (void*)s->X, (void*)s->T, (void*)s->theta, (void*)s->grad, (void*)s->m1,
                  (void*)s->m2, (void*)s->xb, (void*)s->tb, (void*)s->pre[0], (void*)s->pre[1],
                  (void*)s->pre[2], (void*)s->act[0], (void*)s->act[1], (void*)s->act[2], (void*)s->out,
                  (void*)s->d0, (void*)s->d1, (void*)s->lpart, (void*)s->loss_hist, (void*)s->counter})
    if (p) (void)hipFree(p);
  delete s;
}

// forward pass over `rows` inputs x [rows][4] with caller-provided buffers
void mlp_forward(rf_ctx* ctx, const float* th, const float* x, int rows, float* const pre[3],
                 float* const act[3], float* out) {
  using namespace mlpdef;
  sgemm(ctx, x, 0, th + kW0, 1, pre[0], th + kB0, act[0], rows, kHid, kIn);
  sgemm(ctx, act[0], 0, th + kW1, 1, pre[1], th + kB1, act[1], rows, kHid, kHid);
  sgemm(ctx, act[1], 0, th + kW2, 1, pre[2], th + kB2, act[2], rows, kHid, kHid);
  sgemm(ctx, act[2], 0, th + kW3, 1, out, th + kB3, nullptr, rows, kOut, kHid);
}

// backward pass from dout [rows][128] (overwritten) into grad (packed like theta)
void mlp_backward(rf_ctx* ctx, const float* th, const float* x, int rows, float* const pre[3],
                  float* const act[3], float* dout, float* d0, float* d1, float* g) {
  using namespace mlpdef;
  // layer 3 (output, linear)
  sgemm(ctx, dout, 1, act[2], 0, g + kW3, nullptr, nullptr, kOut, kHid, rows);
  hipLaunchKernelGGL(k_colsum, dim3((kOut + 255) / 256), dim3(256), 0, ctx->stream, dout, g + kB3, rows, kOut);
  sgemm(ctx, dout, 0, th + kW3, 0, d0, nullptr, nullptr, rows, kHid, kOut);
  hipLaunchKernelGGL(k_gelu_back, dim3(gblocks(int64_t(rows) * kHid)), dim3(256), 0, ctx->stream, d0, pre[2],
                     int64_t(rows) * kHid);
  // layer 2
  sgemm(ctx, d0, 1, act[1], 0, g + kW2, nullptr, nullptr, kHid, kHid, rows);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, ctx->stream, d0, g + kB2, rows, kHid);
  sgemm(ctx, d0, 0, th + kW2, 0, d1, nullptr, nullptr, rows, kHid, kHid);
  hipLaunchKernelGGL(k_gelu_back, dim3(gblocks(int64_t(rows) * kHid)), dim3(256), 0, ctx->stream, d1, pre[1],
                     int64_t(rows) * kHid);
  // layer 1
  sgemm(ctx, d1, 1, act[0], 0, g + kW1, nullptr, nullptr, kHid, kHid, rows);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, ctx->stream, d1, g + kB1, rows, kHid);
  sgemm(ctx, d1, 0, th + kW1, 0, d0, nullptr, nullptr, rows, kHid, kHid);
  hipLaunchKernelGGL(k_gelu_back, dim3(gblocks(int64_t(rows) * kHid)), dim3(256), 0, ctx->stream, d0, pre[0],
                     int64_t(rows) * kHid);
  // layer 0
  sgemm(ctx, d0, 1, x, 0, g + kW0, nullptr, nullptr, kHid, kIn, rows);
  hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, ctx->stream, d0, g + kB0, rows, kHid);
  RF_HIP(hipGetLastError());
}

void ensure_batch(rf_surrogate* s, int B) {
  using namespace mlpdef;
  if (s->B >= B) return;
  for (float** p : {&s->xb, &s->tb, &s->pre[0], &s->pre[1], &s->pre[2], &s->act[0], &s->act[1], &s->act[2],
                    &s->out, &s->d0, &s->d1})
    if (*p) {
      (void)hipFree(*p);
      *p = nullptr;
    }
  s->xb = dev_alloc<float>(size_t(B) * kIn, "surrogate: device allocation failed");
  s->tb = dev_alloc<float>(size_t(B) * kOut, "surrogate: device allocation failed");
  for (int i = 0; i < 3; ++i) {
    s->pre[i] = dev_alloc<float>(size_t(B) * kHid, "surrogate: device allocation failed");
    s->act[i] = dev_alloc<float>(size_t(B) * kHid, "surrogate: device allocation failed");
  }
  s->out = dev_alloc<float>(size_t(B) * kOut, "surrogate: device allocation failed");
  s->d0 = dev_alloc<float>(size_t(B) * kHid, "surrogate: device allocation failed");
  s->d1 = dev_alloc<float>(size_t(B) * kHid, "surrogate: device allocation failed");
  s->B = B;
  if (s->exec) {
    (void)hipGraphExecDestroy(s->exec);
    s->exec = nullptr;
  }
}

// network prediction of the coefficients of (ref, nbr[k]) into c [nk][rank]
void predict_into(rf_ctx* ctx, rf_surrogate* s, const rf_tmpl& ref, const rf_tmpl* nbr, int nk, double2* c) {
  ensure_batch(s, nk);
  std::vector<float> xs(size_t(nk) * 4);
  for (int k = 0; k < nk; ++k) {
    RF_CHECK(nbr[k].m1 > 0 && nbr[k].m2 > 0, "surrogate: masses must be positive");
    double f[4];
    features(ref, nbr[k], s->grid.f_low, f);
    for (int j = 0; j < 4; ++j) xs[size_t(k) * 4 + j] = float((f[j] - s->feat_mean[j]) / s->feat_std[j]);
  }
  copy_sync(ctx, s->xb, xs.data(), sizeof(float) * xs.size(), hipMemcpyHostToDevice);
  mlp_forward(ctx, s->theta, s->xb, nk, s->pre, s->act, s->out);
  hipLaunchKernelGGL(k_from_outputs, dim3(unsigned(nk)), dim3(64), 0, ctx->stream, s->out, nk, s->rank,
                     s->out_scale, c);
  RF_HIP(hipGetLastError());
}

}  // namespace
}  // namespace rf

using namespace rf;

extern "C" {

rf_status rf_surrogate_create(rf_ctx* ctx, const rf_grid* grid, const rf_tmpl* refs, const rf_tmpl* nbrs,
                              int32_t npair, int32_t window, int32_t rank, const double* omega,
                              int32_t nomega, rf_surrogate** out) {
  if (!ctx) return RF_E_INVAL;
  rf_surrogate* s = nullptr;
  rf_status st = guarded(ctx, [&] {
    validate_grid(grid);
    RF_CHECK(refs && nbrs && omega && out, "rf_surrogate_create: null pointer");
    RF_CHECK(npair >= 8, "rf_surrogate_create: need at least 8 pairs");
    RF_CHECK(is_pow2(window) && window >= 256 && window <= grid->n, "rf_surrogate_create: window must be a power of two in [256, n]");
    RF_CHECK(rank >= 1 && 2 * rank == mlpdef::kOut, "rf_surrogate_create: rank must be 64");
    RF_CHECK(nomega >= rank && nomega <= 256, "rf_surrogate_create: need rank <= nomega <= 256 draws per pair");
    *out = nullptr;
    s = new rf_surrogate();
    s->device = ctx->device;
    s->grid = *grid;
    s->window = window;
    s->rank = rank;
    s->npair = npair;
    const int L = window;
    // features
    std::vector<double> feat(size_t(npair) * 4);
    for (int p = 0; p < npair; ++p) {
      RF_CHECK(refs[p].m1 > 0 && refs[p].m2 > 0 && nbrs[p].m1 > 0 && nbrs[p].m2 > 0, "rf_surrogate_create: bad masses");
      features(refs[p], nbrs[p], grid->f_low, &feat[size_t(p) * 4]);
    }
    for (int j = 0; j < 4; ++j) {
      double mu = 0, var = 0;
      for (int p = 0; p < npair; ++p) mu += feat[size_t(p) * 4 + j];
      mu /= npair;
      for (int p = 0; p < npair; ++p) var += (feat[size_t(p) * 4 + j] - mu) * (feat[size_t(p) * 4 + j] - mu);
      s->feat_mean[j] = mu;
      s->feat_std[j] = std::sqrt(var / npair) > 0 ? std::sqrt(var / npair) : 1.0;
    }
    std::vector<float> xs(feat.size());
    for (int p = 0; p < npair; ++p)
      for (int j = 0; j < 4; ++j) xs[size_t(p) * 4 + j] = float((feat[size_t(p) * 4 + j] - s->feat_mean[j]) / s->feat_std[j]);
    s->X = dev_alloc<float>(xs.size(), "surrogate: device allocation failed");
    copy_sync(ctx, s->X, xs.data(), sizeof(float) * xs.size(), hipMemcpyHostToDevice);

    // exact analytic kernels on the window: H [npair][L]
    double2* H = dev_alloc<double2>(size_t(npair) * L, "surrogate: device allocation failed");
    window_kernels(ctx, grid, refs, nbrs, npair, L, H);
    // randomized range finder: Y = A Om with A = H^T [L][npair] (the spectrum decays fast
    // enough that no power iteration is needed; one would cube the condition number)
    const int r2 = nomega;
    double2* Om = dev_alloc<double2>(size_t(npair) * r2, "surrogate: device allocation failed");
    {
      std::vector<double2> oh(size_t(npair) * r2);
      std::vector<double> od(size_t(npair) * r2);
      copy_sync(ctx, od.data(), omega, sizeof(double) * od.size(), hipMemcpyDeviceToHost);
      for (size_t i = 0; i < od.size(); ++i) oh[i] = make_double2(od[i], 0.0);
      copy_sync(ctx, Om, oh.data(), sizeof(double2) * oh.size(), hipMemcpyHostToDevice);
    }
    double2* Y = dev_alloc<double2>(size_t(L) * r2, "surrogate: device allocation failed");
    zgemm(ctx, H, L, 1, 0, Om, r2, 0, 0, Y, r2, L, r2, npair);       // Y = H^T Om
    // orthonormal basis of range(Y) by Cholesky-QR done twice, each pass through the
    // eigen-decomposition of the Gram matrix: Q1 = Y V diag(lam^-1/2) keeps the
    // directions with lam > 1e-14 lam_max (condition of Y below 1e7), and the second
    // pass restores orthogonality to rounding level
    auto chol_qr = [&](const double2* Yin, int ncol, bool cut, int* kept) {
      double2* G = dev_alloc<double2>(size_t(ncol) * ncol, "surrogate: device allocation failed");
      zgemm(ctx, Yin, ncol, 1, 1, Yin, ncol, 0, 0, G, ncol, ncol, ncol, L);   // G = Y^H Y
      std::vector<double> lam;
      std::vector<cd> Vg;
      herm_eig(to_host(ctx, G, size_t(ncol) * ncol), ncol, lam, Vg);
      (void)hipFree(G);
      int k = 0;
      while (k < ncol && lam[k] > 0 && (!cut || lam[k] > lam[0] * 1e-14)) ++k;
      RF_CHECK(k >= 1, "rf_surrogate_create: training kernels are all zero");
      std::vector<cd> S(size_t(ncol) * k);
      for (int i = 0; i < ncol; ++i)
        for (int c = 0; c < k; ++c) S[size_t(i) * k + c] = Vg[size_t(i) * ncol + c] / std::sqrt(lam[c]);
      double2* Sd = to_dev(ctx, S);
      double2* Qo = dev_alloc<double2>(size_t(L) * k, "surrogate: device allocation failed");
      zgemm(ctx, Yin, ncol, 0, 0, Sd, k, 0, 0, Qo, k, L, k, ncol);
      RF_HIP(hipStreamSynchronize(ctx->stream));
      (void)hipFree(Sd);
      *kept = k;
      return Qo;
    };
    int kr = 0, kr2 = 0;
    double2* Q1 = chol_qr(Y, r2, true, &kr);
    double2* Q = chol_qr(Q1, kr, false, &kr2);
    (void)hipFree(Q1);
    RF_CHECK(kr2 == kr, "rf_surrogate_create: basis lost rank in re-orthogonalisation");
    double2* Bm = dev_alloc<double2>(size_t(kr) * npair, "surrogate: device allocation failed");
    zgemm(ctx, Q, kr, 1, 1, H, L, 1, 0, Bm, npair, kr, npair, L);    // B = Q^H H^T
    double2* M2 = dev_alloc<double2>(size_t(kr) * kr, "surrogate: device allocation failed");
    zgemm(ctx, Bm, npair, 0, 0, Bm, npair, 1, 1, M2, kr, kr, kr, npair);   // B B^H
    std::vector<double> mu;
    std::vector<cd> W;
    herm_eig(to_host(ctx, M2, size_t(kr) * kr), kr, mu, W);
    // U = Q W[:, :rank] (zero columns beyond the numerical rank)
    std::vector<cd> Wr(size_t(kr) * rank, cd(0, 0));
    for (int i = 0; i < kr; ++i)
      for (int c = 0; c < std::min(rank, kr); ++c) Wr[size_t(i) * rank + c] = W[size_t(i) * kr + c];
    double2* Wd = to_dev(ctx, Wr);
    s->U = dev_alloc<double2>(size_t(L) * rank, "surrogate: device allocation failed");
    zgemm(ctx, Q, kr, 0, 0, Wd, rank, 0, 0, s->U, rank, L, rank, kr);
    s->kr = kr;
    s->svals.clear();
    for (int c = 0; c < kr; ++c) s->svals.push_back(std::sqrt(std::max(0.0, mu[c])));
    // coefficients c_p = U^H h_p  ->  C [npair][rank] = (W^H B)^T
    double2* Cf = dev_alloc<double2>(size_t(npair) * rank, "surrogate: device allocation failed");
    // c_p[j] = sum_i conj(W[i][j]) B[i][p]
    zgemm(ctx, Bm, npair, 1, 0, Wd, rank, 0, 1, Cf, rank, npair, rank, kr);
    std::vector<cd> ch = to_host(ctx, Cf, size_t(npair) * rank);
    double mx = 0;
    for (const cd& v : ch) mx = std::max(mx, std::abs(v));
    s->out_scale = mx > 0 ? mx : 1.0;
    s->T = dev_alloc<float>(size_t(npair) * mlpdef::kOut, "surrogate: device allocation failed");
    hipLaunchKernelGGL(k_to_targets, dim3(unsigned(npair)), dim3(64), 0, ctx->stream, Cf, npair, rank,
                       1.0 / s->out_scale, s->T);
    RF_HIP(hipGetLastError());
    RF_HIP(hipStreamSynchronize(ctx->stream));
    for (void* p : {(void*)H, (void*)Om, (void*)Y, (void*)Q, (void*)Bm, (void*)M2, (void*)Wd, (void*)Cf})
      (void)hipFree(p);
    s->theta = dev_alloc<float>(mlpdef::kParams, "surrogate: device allocation failed");
    s->grad = dev_alloc<float>(mlpdef::kParams, "surrogate: device allocation failed");
    s->m1 = dev_alloc<float>(mlpdef::kParams, "surrogate: device allocation failed");
    s->m2 = dev_alloc<float>(mlpdef::kParams, "surrogate: device allocation failed");
    s->counter = dev_alloc<int32_t>(2, "surrogate: device allocation failed");
    s->lpart = dev_alloc<float>(kMseBlocks, "surrogate: device allocation failed");
    *out = s;
  });
  if (st != RF_OK && s) free_surrogate(s);
  return st;
}

rf_status rf_surrogate_info(const rf_surrogate* s, int32_t* window, int32_t* rank, int32_t* numerical_rank,
                            double* svals, double* out_scale, int64_t* steps_trained) {
  if (!s) return RF_E_INVAL;
  if (window) *window = s->window;
  if (rank) *rank = s->rank;
  if (numerical_rank) *numerical_rank = s->kr;
  if (svals)
    for (int i = 0; i < s->kr; ++i) svals[i] = s->svals[i];
  if (out_scale) *out_scale = s->out_scale;
  if (steps_trained) *steps_trained = s->steps_total;
  return RF_OK;
}

rf_status rf_surrogate_set_params(rf_ctx* ctx, rf_surrogate* s, const float* theta) {
  if (!ctx || !s || !theta) return RF_E_INVAL;
  return guarded(ctx, [&] {
    RF_HIP(hipMemcpyAsync(s->theta, theta, sizeof(float) * mlpdef::kParams, hipMemcpyDeviceToDevice, ctx->stream));
    fill_u32(ctx, reinterpret_cast<uint32_t*>(s->m1), 0u, mlpdef::kParams);   // +0.0f
    fill_u32(ctx, reinterpret_cast<uint32_t*>(s->m2), 0u, mlpdef::kParams);
    RF_HIP(hipStreamSynchronize(ctx->stream));
    fill_u32(ctx, reinterpret_cast<uint32_t*>(s->counter), 0u, 2);
    RF_HIP(hipStreamSynchronize(ctx->stream));
    s->steps_total = 0;
  });
}

rf_status rf_surrogate_get_params(rf_ctx* ctx, const rf_surrogate* s, float* theta) {
  if (!ctx || !s || !theta) return RF_E_INVAL;
  return guarded(ctx, [&] {
    RF_HIP(hipMemcpyAsync(theta, s->theta, sizeof(float) * mlpdef::kParams, hipMemcpyDeviceToDevice, ctx->stream));
    RF_HIP(hipStreamSynchronize(ctx->stream));
  });
}

rf_status rf_surrogate_dataset(rf_ctx* ctx, const rf_surrogate* s, float* x, float* t) {
  if (!ctx || !s || (!x && !t)) return RF_E_INVAL;
  return guarded(ctx, [&] {
    if (x)
      RF_HIP(hipMemcpyAsync(x, s->X, sizeof(float) * size_t(s->npair) * mlpdef::kIn, hipMemcpyDeviceToDevice,
                            ctx->stream));
    if (t)
      RF_HIP(hipMemcpyAsync(t, s->T, sizeof(float) * size_t(s->npair) * mlpdef::kOut, hipMemcpyDeviceToDevice,
                            ctx->stream));
    RF_HIP(hipStreamSynchronize(ctx->stream));
  });
}

rf_status rf_surrogate_grad(rf_ctx* ctx, rf_surrogate* s, const float* x, const float* t, int32_t rows,
                            float* loss_host, float* grad_out) {
  if (!ctx || !s) return RF_E_INVAL;
  return guarded(ctx, [&] {
    RF_CHECK(x && t && grad_out && rows >= 1, "rf_surrogate_grad: bad arguments");
    ensure_batch(s, rows);
    mlp_forward(ctx, s->theta, x, rows, s->pre, s->act, s->out);
    const int64_t n = int64_t(rows) * mlpdef::kOut;
    float* dout = s->out;     // gradient written in place of the outputs
    hipLaunchKernelGGL(k_mse, dim3(kMseBlocks), dim3(256), 0, ctx->stream, s->out, t, dout, s->lpart, n);
    float* lh = dev_alloc<float>(1, "surrogate: device allocation failed");
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, ctx->stream, s->lpart, kMseBlocks, n, lh,
                       (const int32_t*)nullptr);
    mlp_backward(ctx, s->theta, x, rows, s->pre, s->act, dout, s->d0, s->d1, grad_out);
    float l = 0;
    RF_HIP(hipMemcpyAsync(&l, lh, sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    RF_HIP(hipStreamSynchronize(ctx->stream));
    (void)hipFree(lh);
    if (loss_host) *loss_host = l;
  });
}

rf_status rf_surrogate_train(rf_ctx* ctx, rf_surrogate* s, const int32_t* order, int32_t steps, int32_t batch,
                             float lr, float* loss_host) {
  if (!ctx || !s) return RF_E_INVAL;
  return guarded(ctx, [&] {
    RF_CHECK(order && steps >= 1 && batch >= 1, "rf_surrogate_train: bad arguments");
    RF_CHECK(ctx->stream != nullptr, "rf_surrogate_train: needs a non-null stream (graph capture)");
    ensure_batch(s, batch);
    if (s->hist_cap < steps) {
      if (s->loss_hist) (void)hipFree(s->loss_hist);
      s->loss_hist = dev_alloc<float>(size_t(steps), "surrogate: device allocation failed");
      s->hist_cap = steps;
      if (s->exec) {
        (void)hipGraphExecDestroy(s->exec);
        s->exec = nullptr;
      }
    }
    fill_u32(ctx, reinterpret_cast<uint32_t*>(s->counter), 0u, 1);
    if (s->exec && (s->order != order || s->lr != lr || s->graph_steps != steps || s->graph_batch != batch)) {
      (void)hipGraphExecDestroy(s->exec);
      s->exec = nullptr;
    }
    const int64_t n = int64_t(batch) * mlpdef::kOut;
    if (!s->exec) {
      hipGraph_t graph = nullptr;
      RF_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
      try {
        hipLaunchKernelGGL(k_gather, dim3(unsigned(batch)), dim3(128), 0, ctx->stream, s->X, s->T, order, s->counter,
                           batch, s->xb, s->tb);
        mlp_forward(ctx, s->theta, s->xb, batch, s->pre, s->act, s->out);
        hipLaunchKernelGGL(k_mse, dim3(kMseBlocks), dim3(256), 0, ctx->stream, s->out, s->tb, s->out, s->lpart, n);
        hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, ctx->stream, s->lpart, kMseBlocks, n, s->loss_hist,
                           (const int32_t*)s->counter);
        mlp_backward(ctx, s->theta, s->xb, batch, s->pre, s->act, s->out, s->d0, s->d1, s->grad);
        hipLaunchKernelGGL(k_adam, dim3(gblocks(mlpdef::kParams, 1024)), dim3(256), 0, ctx->stream, s->theta,
                           s->grad, s->m1, s->m2, s->counter, int64_t(mlpdef::kParams), lr, int64_t(steps));
        hipLaunchKernelGGL(k_count, dim3(1), dim3(64), 0, ctx->stream, s->counter);
        RF_HIP(hipGetLastError());
      } catch (...) {
        hipGraph_t g2 = nullptr;
        (void)hipStreamEndCapture(ctx->stream, &g2);
        if (g2) (void)hipGraphDestroy(g2);
        throw;
      }
      RF_HIP(hipStreamEndCapture(ctx->stream, &graph));
      hipError_t e = hipGraphInstantiate(&s->exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) throw Error{RF_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
      s->order = order;
      s->lr = lr;
      s->graph_steps = steps;
      s->graph_batch = batch;
    }
    for (int i = 0; i < steps; ++i) RF_HIP(hipGraphLaunch(s->exec, ctx->stream));
    s->steps_total += steps;
    if (loss_host)
      RF_HIP(hipMemcpyAsync(loss_host, s->loss_hist, sizeof(float) * steps, hipMemcpyDeviceToHost, ctx->stream));
    RF_HIP(hipStreamSynchronize(ctx->stream));
  });
}

rf_status rf_surrogate_predict(rf_ctx* ctx, rf_surrogate* s, rf_tmpl ref, const rf_tmpl* nbr, int32_t nk,
                               void* coeffs) {
  if (!ctx || !s) return RF_E_INVAL;
  return guarded(ctx, [&] {
    RF_CHECK(nbr && coeffs && nk >= 1, "rf_surrogate_predict: bad arguments");
    predict_into(ctx, s, ref, nbr, nk, static_cast<double2*>(coeffs));
    RF_HIP(hipStreamSynchronize(ctx->stream));
  });
}

rf_status rf_surrogate_project(rf_ctx* ctx, rf_surrogate* s, rf_tmpl ref, const rf_tmpl* nbr, int32_t nk,
                               void* coeffs) {
  if (!ctx || !s) return RF_E_INVAL;
  double2* H = nullptr;
  rf_status st = guarded(ctx, [&] {
    RF_CHECK(nbr && coeffs && nk >= 1, "rf_surrogate_project: bad arguments");
    const int L = s->window;
    std::vector<rf_tmpl> refs(size_t(nk), ref);
    H = dev_alloc<double2>(size_t(nk) * L, "surrogate: device allocation failed");
    window_kernels(ctx, &s->grid, refs.data(), nbr, nk, L, H);
    // c[k][j] = sum_q conj(U[q][j]) H[k][q]
    zgemm(ctx, H, L, 0, 0, s->U, s->rank, 0, 1, static_cast<double2*>(coeffs), s->rank, nk, s->rank, L);
    RF_HIP(hipStreamSynchronize(ctx->stream));
  });
  if (H) (void)hipFree(H);
  return st;
}

rf_status rf_surrogate_encode(rf_ctx* ctx, rf_surrogate* s, rf_tmpl ref, const rf_tmpl* nbr, int32_t nk,
                              int32_t bits, int32_t use_network, void* codes, float* scales) {
  if (!ctx || !s) return RF_E_INVAL;
  double2* H = nullptr;
  double2* c = nullptr;
  rf_status st = guarded(ctx, [&] {
    RF_CHECK(nbr && codes && scales && nk >= 1, "rf_surrogate_encode: bad arguments");
    RF_CHECK(bits == 8 || bits == 16, "rf_surrogate_encode: bits must be 8 or 16");
    const int L = s->window;
    std::vector<rf_tmpl> refs(size_t(nk), ref);
    H = dev_alloc<double2>(size_t(nk) * L, "surrogate: device allocation failed");
    c = dev_alloc<double2>(size_t(nk) * s->rank * 2, "surrogate: device allocation failed");
    double2* p = use_network ? c + size_t(nk) * s->rank : nullptr;
    window_kernels(ctx, &s->grid, refs.data(), nbr, nk, L, H);
    zgemm(ctx, H, L, 0, 0, s->U, s->rank, 0, 1, c, s->rank, nk, s->rank, L);   // exact U^H h
    if (p) predict_into(ctx, s, ref, nbr, nk, p);
    if (bits == 8)
      hipLaunchKernelGGL(k_encode<int8_t>, dim3(unsigned(nk)), dim3(128), 0, ctx->stream, c, p, s->rank, 127,
                         static_cast<int8_t*>(codes), scales);
    else
      hipLaunchKernelGGL(k_encode<int16_t>, dim3(unsigned(nk)), dim3(128), 0, ctx->stream, c, p, s->rank, 32767,
                         static_cast<int16_t*>(codes), scales);
    RF_HIP(hipGetLastError());
    RF_HIP(hipStreamSynchronize(ctx->stream));
  });
  if (H) (void)hipFree(H);
  if (c) (void)hipFree(c);
  return st;
}

rf_status rf_surrogate_decode(rf_ctx* ctx, rf_surrogate* s, rf_tmpl ref, const rf_tmpl* nbr, int32_t nk,
                              int32_t bits, int32_t use_network, const void* codes, const float* scales,
                              void* coeffs) {
  if (!ctx || !s) return RF_E_INVAL;
  double2* p = nullptr;
  rf_status st = guarded(ctx, [&] {
    RF_CHECK(nbr && codes && scales && coeffs && nk >= 1, "rf_surrogate_decode: bad arguments");
    RF_CHECK(bits == 8 || bits == 16, "rf_surrogate_decode: bits must be 8 or 16");
    if (use_network) {
      p = dev_alloc<double2>(size_t(nk) * s->rank, "surrogate: device allocation failed");
      predict_into(ctx, s, ref, nbr, nk, p);
    }
    if (bits == 8)
      hipLaunchKernelGGL(k_decode<int8_t>, dim3(unsigned(nk)), dim3(64), 0, ctx->stream,
                         static_cast<const int8_t*>(codes), scales, p, s->rank, static_cast<double2*>(coeffs));
    else
      hipLaunchKernelGGL(k_decode<int16_t>, dim3(unsigned(nk)), dim3(64), 0, ctx->stream,
                         static_cast<const int16_t*>(codes), scales, p, s->rank, static_cast<double2*>(coeffs));
    RF_HIP(hipGetLastError());
    RF_HIP(hipStreamSynchronize(ctx->stream));
  });
  if (p) (void)hipFree(p);
  return st;
}

rf_status rf_surrogate_kernels(rf_ctx* ctx, rf_surrogate* s, const rf_grid* grid, const double* psd, rf_tmpl ref,
                               const rf_tmpl* nbr, int32_t nk, const void* coeffs, double thr, rf_thr_unit unit,
                               const rf_grid* check_grid, const void* check_xf, const double* check_psd,
                               double tol, rf_kernels** out, int32_t* fallback, float* check_err) {
  if (!ctx || !s) return RF_E_INVAL;
  rf_kernels* K = nullptr;
  rf_kernels* KE = nullptr;
  double2* coef = nullptr;
  double2* Hk = nullptr;
  rf_status st = guarded(ctx, [&] {
    validate_grid(grid);
    RF_CHECK(psd && nbr && out && nk >= 1, "rf_surrogate_kernels: bad arguments");
    RF_CHECK(grid->fs == s->grid.fs && grid->f_low == s->grid.f_low && grid->f_high == s->grid.f_high &&
                 grid->df_high == s->grid.df_high && grid->df_low_max == s->grid.df_low_max,
             "rf_surrogate_kernels: grid differs from the training grid");
    RF_CHECK(grid->n >= s->window, "rf_surrogate_kernels: segment shorter than the kernel window");
    RF_CHECK(std::isfinite(thr) && thr > 0, "rf_surrogate_kernels: threshold must be positive");
    *out = nullptr;
    const int L = s->window;
    // coefficients (predicted by the network unless given) and kernels on the window
    const double2* cf = static_cast<const double2*>(coeffs);
    if (!cf) {
      coef = dev_alloc<double2>(size_t(nk) * s->rank, "surrogate: device allocation failed");
      predict_into(ctx, s, ref, nbr, nk, coef);
      cf = coef;
    }
    Hk = dev_alloc<double2>(size_t(nk) * L, "surrogate: device allocation failed");
    zgemm(ctx, cf, s->rank, 0, 0, s->U, s->rank, 1, 0, Hk, L, nk, L, s->rank);   // Hk = C U^T
    // truncation as for the exact kernels
    const double thr_tap = unit == RF_THR_PER_SECOND ? thr / grid->fs : thr;
    std::vector<int32_t> lo(nk), hi(nk);
    std::vector<uint32_t> mx(nk);
    int32_t* lo_d = dev_alloc<int32_t>(size_t(nk) * 3, "surrogate: device allocation failed");
    int32_t* hi_d = lo_d + nk;
    uint32_t* mx_d = reinterpret_cast<uint32_t*>(hi_d + nk);
    fill_u32(ctx, reinterpret_cast<uint32_t*>(lo_d), 0x7FFFFFFFu, nk);
    fill_u32(ctx, reinterpret_cast<uint32_t*>(hi_d), 0x80000000u, nk);
    fill_u32(ctx, mx_d, 0u, nk);
    support_scan(ctx, Hk, L, nk, thr_tap, lo_d, hi_d, mx_d);
    RF_HIP(hipMemcpyAsync(lo.data(), lo_d, sizeof(int32_t) * nk, hipMemcpyDeviceToHost, ctx->stream));
    RF_HIP(hipMemcpyAsync(hi.data(), hi_d, sizeof(int32_t) * nk, hipMemcpyDeviceToHost, ctx->stream));
    RF_HIP(hipMemcpyAsync(mx.data(), mx_d, sizeof(uint32_t) * nk, hipMemcpyDeviceToHost, ctx->stream));
    RF_HIP(hipStreamSynchronize(ctx->stream));
    (void)hipFree(lo_d);
    std::vector<double2> hh(size_t(nk) * L);
    copy_sync(ctx, hh.data(), Hk, sizeof(double2) * hh.size(), hipMemcpyDeviceToHost);
    // norms through the band moment of the segment grid
    double* moment = static_cast<double*>(ctx->ws[WS_SCALAR].ensure(64));
    band_moment(ctx, grid, psd, moment);
    double mom = 0;
    RF_HIP(hipMemcpyAsync(&mom, moment, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    RF_HIP(hipStreamSynchronize(ctx->stream));
    const double df = grid->fs / double(grid->n);
    const Tf2Coef cref = tf2_coef(ref);
    const double nref = cref.amp * std::sqrt(4.0 * df * mom);
    auto build = [&](const std::vector<int32_t>& lo_, const std::vector<int32_t>& hi_,
                     const std::vector<double>& ks, std::function<double(int, int64_t)> tap) {
      rf_kernels* KK = new rf_kernels();
      KK->device = ctx->device;
      KK->nk = nk;
      KK->n_build = grid->n;
      KK->fs = grid->fs;
      KK->m_lo.resize(nk);
      KK->len.resize(nk);
      KK->off.resize(nk);
      KK->kscale.resize(nk);
      KK->norm_ratio.resize(nk);
      KK->df_low.resize(nk);
      std::vector<double> taps;
      for (int k = 0; k < nk; ++k) {
        const Tf2Coef ck = tf2_coef(nbr[k]);
        KK->norm_ratio[k] = nref / (ck.amp * std::sqrt(4.0 * df * mom));
        const double d = std::fabs(tf2_dtdf(ck, grid->f_low) - tf2_dtdf(cref, grid->f_low));
        KK->df_low[k] = std::min(d > 0 ? 1.0 / std::sqrt(d) : grid->df_low_max, grid->df_low_max);
        KK->off[k] = int64_t(taps.size());
        if (lo_[k] == 0x7FFFFFFF) {
          KK->m_lo[k] = 0;
          KK->len[k] = 0;
        } else {
          KK->m_lo[k] = lo_[k];
          KK->len[k] = hi_[k] - lo_[k] + 1;
          for (int64_t m = lo_[k]; m <= hi_[k]; ++m) taps.push_back(tap(k, m));
        }
        KK->kscale[k] = ks[k];
      }
      finalize_kernel_set(ctx, KK, taps);
      return KK;
    };
    // FP16 scales as the exact build sets them: from the largest |tap| (as float)
    std::vector<double> ksd(nk);
    for (int k = 0; k < nk; ++k) {
      float f;
      std::memcpy(&f, &mx[k], 4);
      ksd[k] = 1.0;
      if (f > 0) {
        int ex = 0;
        std::frexp(double(f), &ex);
        ksd[k] = std::ldexp(1.0, 14 - ex);
      }
    }
    auto sur_tap = [&](int k, int64_t m) { return hh[size_t(k) * L + size_t(m & (L - 1))].x; };
    K = build(lo, hi, ksd, sur_tap);
    // a support that reaches the window edge was cut by the window: exact kernel
    std::vector<int32_t> fb(nk, 0);
    std::vector<float> err(nk, 0.f);
    for (int k = 0; k < nk; ++k)
      if (lo[k] != 0x7FFFFFFF && (lo[k] <= -L / 2 + 1 || hi[k] >= L / 2)) fb[k] = 1;
    if (check_grid && check_xf && check_psd) {
      validate_grid(check_grid);
      RF_CHECK(check_grid->fs == grid->fs && check_grid->f_low == grid->f_low && check_grid->f_high == grid->f_high,
               "rf_surrogate_kernels: check grid must share fs and band");
      const int64_t nc = check_grid->n;
      float2* zr = dev_alloc<float2>(size_t(nc), "surrogate: device allocation failed");
      float2* zs = dev_alloc<float2>(size_t(nk) * nc, "surrogate: device allocation failed");
      float2* zd = dev_alloc<float2>(size_t(nk) * nc, "surrogate: device allocation failed");
      float* e = dev_alloc<float>(nk, "surrogate: device allocation failed");
      rf_status s1 = mf_ref_snr(ctx, check_grid, check_xf, check_psd, &ref, 1, zr, nullptr);
      if (s1 == RF_OK) s1 = snr_reconstruct(ctx, K, zr, nc, RF_PREC_SPLIT_FP16, zs, nullptr);
      if (s1 == RF_OK) s1 = mf_ref_snr(ctx, check_grid, check_xf, check_psd, nbr, nk, zd, nullptr);
      if (s1 == RF_OK) {
        hipLaunchKernelGGL(k_rowmaxdiff, dim3(unsigned(nk)), dim3(256), 0, ctx->stream, zs, zd, nc, e);
        RF_HIP(hipGetLastError());
        RF_HIP(hipMemcpyAsync(err.data(), e, sizeof(float) * nk, hipMemcpyDeviceToHost, ctx->stream));
        RF_HIP(hipStreamSynchronize(ctx->stream));
      }
      for (void* p : {(void*)zr, (void*)zs, (void*)zd, (void*)e}) (void)hipFree(p);
      if (s1 != RF_OK) throw Error{s1, ctx->last_error};
      for (int k = 0; k < nk; ++k)
        if (!(err[k] <= tol)) fb[k] = 1;
    }
    {
      std::vector<rf_tmpl> fnb;
      std::vector<int> fidx;
      for (int k = 0; k < nk; ++k)
        if (fb[k]) {
          fnb.push_back(nbr[k]);
          fidx.push_back(k);
        }
      if (!fnb.empty()) {
        // exact FP64 kernels for the fallback set, merged with the surrogate ones
        rf_status s2 = ratio_kernel_build(ctx, grid, psd, ref, fnb.data(), int32_t(fnb.size()), thr, unit, 0, &KE);
        if (s2 != RF_OK) throw Error{s2, ctx->last_error};
        std::vector<std::vector<double>> etaps(fnb.size());
        for (size_t i = 0; i < fnb.size(); ++i) {
          etaps[i].resize(size_t(KE->len[i]));
          if (KE->len[i] > 0)
            copy_sync(ctx, etaps[i].data(), KE->taps64 + KE->off[i], sizeof(double) * KE->len[i],
                             hipMemcpyDeviceToHost);
        }
        std::vector<int32_t> lo2 = lo, hi2 = hi;
        std::vector<double> ks2 = ksd;
        std::vector<int> which(nk, -1);
        for (size_t i = 0; i < fidx.size(); ++i) {
          const int k = fidx[i];
          which[k] = int(i);
          if (KE->len[i] == 0) {
            lo2[k] = 0x7FFFFFFF;
          } else {
            lo2[k] = int32_t(KE->m_lo[i]);
            hi2[k] = int32_t(KE->m_lo[i] + KE->len[i] - 1);
          }
          ks2[k] = KE->kscale[i];
        }
        auto merged_tap = [&](int k, int64_t m) {
          if (which[k] >= 0) return etaps[which[k]][size_t(m - lo2[k])];
          return sur_tap(k, m);
        };
        rf_kernels* K2 = build(lo2, hi2, ks2, merged_tap);
        free_kernel_set(K);
        K = K2;
        free_kernel_set(KE);
        KE = nullptr;
      }
    }
    if (fallback)
      for (int k = 0; k < nk; ++k) fallback[k] = fb[k];
    if (check_err)
      for (int k = 0; k < nk; ++k) check_err[k] = err[k];
    *out = K;
  });
  if (coef) (void)hipFree(coef);
  if (Hk) (void)hipFree(Hk);
  if (KE) free_kernel_set(KE);
  if (st != RF_OK && K) {
    free_kernel_set(K);
    if (out) *out = nullptr;
  }
  return st;
}

rf_status rf_surrogate_free(rf_surrogate* s) {
  if (!s) return RF_E_INVAL;
  (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  free_surrogate(s);
  return RF_OK;
}

}  // extern "C"
