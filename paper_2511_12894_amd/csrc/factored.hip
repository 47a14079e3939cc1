// Factored reconstruction: the correlation of sec. II.B eq. `convolution`,
// z_k[m] = (N_ref/N_k) sum_s z_ref[(m + s) mod n] w_k[s], with every kernel of a
// set replaced by its projection on the set's leading J-dimensional subspace.
//
// With W the K x L matrix of a set's kernels on their union support [M0, M0+L)
// and W W^T = V diag(lambda) V^T, the basis b_j = sum_k V[k][j] w_k (j < J)
// gives the projected kernels w~_k = sum_{j<J} V[k][j] b_j (the best rank-J
// approximation of W, Eckart-Young).  Then
//     z~_k[m] = sum_j C[j][k] y_j[m],  C[j][k] = (N_ref/N_k) V[k][j],
//     y_j[m]  = sum_s z_ref[(m + s) mod n] b_j[s],
// and y_j follows from one forward FFT of z_ref and J inverse FFTs:
//     FFT(y_j)[f] = FFT(z_ref)[f] conj(FFT(b_j)[f]) = FFT(z_ref)[f] IDFT(b_j)[f]
// (b_j real; IDFT = the unnormalised exp(+) sum of the FFT module).  A
// matched-filter series is band-limited (its spectrum vanishes off the
// positive band bins), so the products run over the band bins only.  Per
// output sample this is 4 J flops of mixing plus J/K of a direct matched
// filter's transforms, instead of 4 L flops of the dense correlation.
//
// The per-kernel relative residual ||w_k - w~_k|| / ||w_k|| =
// sqrt(sum_{j>=J} lambda_j V[k][j]^2 / G[k][k]) sets J.  Not in the paper.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "recon.h"
#include "symeig.h"

struct rf_factored {
  int device = 0;
  int64_t n = 0;
  int32_t nk = 0, J = 0, JP = 0, KP = 0;
  int64_t M0 = 0, L = 0, b0 = 0, nb = 0;
  float2* Ub = nullptr;      // [J][nb]: IDFT(b_j) on the band bins
  float* C = nullptr;        // [JP][KP]: (N_ref/N_k) V[k][j], zero padded
  float2* Q = nullptr;       // [n]: transform of conj(z_ref)
  float2* Qin = nullptr;     // [n]
  float2* Y = nullptr;       // [JP][n]: basis correlations y_j (rows from J on zero)
  // split-FP16 mixing: the coefficients as hi/lo FP16 B operand fragments
  // [JP/16][8 tiles][2 planes][64 lanes][8 basis indices] after the scale cscale
  _Float16* Cp = nullptr;
  // large sets (more than 256 kernels or 128 basis vectors): the same hi/lo
  // coefficients as [JP/16][KPL kernels][2 planes][16 basis indices], KPL a
  // multiple of 128, for the tiled mixing
  _Float16* CpL = nullptr;
  int32_t KPL = 0;
  bool large = false;
  uint32_t* zmax = nullptr;  // max(|re|, |im|) of the series being reconstructed (float bits)
  float l1max = 0.f;         // largest L1 norm of a basis vector
  float cscale = 1.f;        // power-of-two scale of the packed coefficients
  std::vector<double> lambda, resid;
};

namespace rf {
namespace {

inline unsigned nblocks(int64_t n, int64_t cap = 4096) {
  const int64_t b = (n + 255) / 256;
  return unsigned(std::max<int64_t>(1, std::min<int64_t>(b, cap)));
}

// dense kernel matrix W[k][s] = w_k[M0 + s] (zero outside its support)
__global__ void k_dense(const double* __restrict__ taps, const int64_t* __restrict__ off,
                        const int64_t* __restrict__ mlo, const int32_t* __restrict__ len, int64_t M0,
                        int64_t L, double* __restrict__ W) {
  const int k = blockIdx.y;
  const int64_t a = mlo[k] - M0, cnt = len[k];
  for (int64_t s = int64_t(blockIdx.x) * 256 + threadIdx.x; s < L; s += int64_t(gridDim.x) * 256)
    W[int64_t(k) * L + s] = (s >= a && s < a + cnt) ? taps[off[k] + (s - a)] : 0.0;
}

// C[M][N] = sum_k opA(i, k) opB(k, j); opA(i, k) = A[i lda + k] or A[k lda + i]
// (ta), opB(k, j) = B[k ldb + j] or B[j ldb + k] (tb).  FP64, 32 x 32 tiles.
__global__ __launch_bounds__(256) void k_dgemm(const double* __restrict__ A, int64_t lda, int ta,
                                               const double* __restrict__ B, int64_t ldb, int tb,
                                               double* __restrict__ C, int64_t ldc, int64_t M, int64_t N,
                                               int64_t K) {
  __shared__ double as[16][33];
  __shared__ double bs[16][33];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t i0 = int64_t(blockIdx.y) * 32, j0 = int64_t(blockIdx.x) * 32;
  double acc[2][2] = {{0, 0}, {0, 0}};
  for (int64_t k0 = 0; k0 < K; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 32; e += 256) {
      const int kk = e / 32, r = e % 32;
      const int64_t i = i0 + r, j = j0 + r, k = k0 + kk;
      as[kk][r] = (i < M && k < K) ? (ta ? A[k * lda + i] : A[i * lda + k]) : 0.0;
      bs[kk][r] = (j < N && k < K) ? (tb ? B[j * ldb + k] : B[k * ldb + j]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk)
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = fma(as[kk][ty * 2 + x], bs[kk][tx * 2 + y], acc[x][y]);
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

void dgemm(rf_ctx* ctx, const double* A, int64_t lda, int ta, const double* B, int64_t ldb, int tb, double* C,
           int64_t ldc, int64_t M, int64_t N, int64_t K) {
  RF_CHECK((M + 31) / 32 <= 65535, "factored: GEMM too tall");
  const dim3 grid{unsigned((N + 31) / 32), unsigned((M + 31) / 32)};
  hipLaunchKernelGGL(k_dgemm, grid, dim3(256), 0, ctx->stream, A, lda, ta, B, ldb, tb, C, ldc, M, N, K);
  RF_HIP(hipGetLastError());
}

// basis rows placed at their signed taps in length-n complex buffers (zeroed before)
__global__ void k_place(const double* __restrict__ Bm, int64_t L, int64_t M0, int64_t n,
                        double2* __restrict__ out) {
  const int j = blockIdx.y;
  for (int64_t s = int64_t(blockIdx.x) * 256 + threadIdx.x; s < L; s += int64_t(gridDim.x) * 256)
    out[int64_t(j) * n + ((M0 + s) & (n - 1))] = make_double2(Bm[int64_t(j) * L + s], 0.0);
}

__global__ void k_band_gather(const double2* __restrict__ in, int64_t n, int64_t b0, int64_t nb,
                              float2* __restrict__ out) {
  const int j = blockIdx.y;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < nb; i += int64_t(gridDim.x) * 256) {
    const double2 v = in[int64_t(j) * n + b0 + i];
    out[int64_t(j) * nb + i] = make_float2(float(v.x), float(v.y));
  }
}

// Mixing: z~_k[m] = sum_j C[j][k] y_j[m] on v_mfma_f32_32x32x2_f32 with rows =
// 32 kernels, columns = 32 output times, real and imaginary parts in separate
// accumulators, so that a lane holds one time of 16 kernels and every store of a
// row of accumulators writes two whole 256-byte runs of series.  A workgroup of
// 8 waves (4 above JP = 96) holds C in LDS as [j][sweep][lane][tile] so that one
// lane's operands of the tiles of a sweep are one 8- or 16-byte read.  Each wave
// owns 32 consecutive times per time block, keeps their y fragments for all j in
// registers and sweeps the kernel tiles 2 (or 4) at a time: per pair of basis
// indices, 4 (8) independent MFMAs.  Read-out: running peak keys of every
// (kernel, time lane) pair as LDS atomics (two time lanes a slot from JP = 112
// on, for room), one global atomic per kernel and workgroup at the end;
// crossings are recorded with the raw (re, im) and finished by a pass over the
// trigger list.  Persistent over time blocks.
constexpr int kMixTimesMax = 256;                // n must be a multiple of this
constexpr int kMixTiles = 8;                     // kernel tiles of the small-set mixings (up to 256 kernels)
constexpr int kFactMaxKernels = 1024;             // kernels per set
constexpr int kFactMaxBasis = 512;                // basis vectors per set
// two waves per SIMD (one hides the other's loads) sweeping 2 tiles at a time
// while the fragments fit in 256 registers, else one wave sweeping 4
template <int JP>
constexpr int mix_waves() { return JP <= 96 ? 8 : 4; }
template <int JP>
constexpr int mix_group() { return JP <= 96 ? 2 : 4; }
// (kernel, time lane) peak slots: 32 time lanes each while LDS allows
template <int JP>
constexpr int mix_slots() { return JP <= 96 ? 32 : 16; }

template <int JP, bool STORE, bool FUSED>
__global__ __launch_bounds__(64 * mix_waves<JP>(), 1) void k_mix(const float2* __restrict__ Y, int64_t n,
                                                                const float* __restrict__ Cg, int nk,
                                                                float2* __restrict__ zout, PeakOut po) {
  constexpr int kMixWaves = mix_waves<JP>();
  constexpr int kMixGroup = mix_group<JP>();
  constexpr int kMixTimes = 32 * kMixWaves;
  constexpr int KP = 32 * kMixTiles;
  constexpr int S = mix_slots<JP>();
  extern __shared__ __attribute__((aligned(16))) float smem[];
  constexpr int NG = kMixTiles / kMixGroup;                  // sweeps per time block
  float* Cs = smem;                                          // [JP][NG][32 lanes][kMixGroup]
  unsigned long long* keys = reinterpret_cast<unsigned long long*>(Cs + JP * KP);  // [KP][S]
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  for (int e = threadIdx.x; e < JP * KP; e += 64 * kMixWaves) {
    const int j = e / KP, k = e % KP, tile = k >> 5;
    Cs[((j * NG + tile / kMixGroup) * 32 + (k & 31)) * kMixGroup + tile % kMixGroup] = Cg[e];
  }
  if (FUSED)
    for (int e = threadIdx.x; e < KP * S; e += 64 * kMixWaves) keys[e] = 0ull;
  __syncthreads();
  const int64_t nblk = n / kMixTimes;
  const int kr = lane >> 5;                      // k index of this lane's operand half
  const int ngroups = (nk + 32 * kMixGroup - 1) / (32 * kMixGroup);
  const int slot = (lane & 31) / (32 / S);
  // store offset of this lane from a tile's row of kernel 32 tile + acc_row(i, 0) at time t0
  const uint32_t loff = uint32_t(4 * kr) * uint32_t(n) + uint32_t(lane & 31);
  // B operand: lane holds y_{2s + kr}[t0 + lane % 32] (rows J..JP-1 of Y are zero)
  float yre[JP / 2], yim[JP / 2];
  const float2* Ylane = Y + int64_t(kr) * n + 32 * wave + (lane & 31);
  auto loadB = [&](int64_t tb) {
    const float2* p = Ylane + tb * kMixTimes;
#pragma unroll
    for (int s = 0; s < JP / 2; ++s) {
      const float2 v = p[int64_t(2 * s) * n];
      yre[s] = v.x;
      yim[s] = v.y;
    }
  };
  // A operands of sweep g's tiles for basis pair s: C[2s + kr][(G g + t) 32 + lane % 32],
  // consecutive lanes reading consecutive words
  typedef float floatG __attribute__((ext_vector_type(kMixGroup)));
  const floatG* cb = reinterpret_cast<const floatG*>(Cs) + kr * NG * 32 + (lane & 31);
  for (int64_t tbk = blockIdx.x; tbk < nblk; tbk += gridDim.x) {
    const int64_t t0 = tbk * kMixTimes + 32 * wave;
    const int64_t m = t0 + (lane & 31);            // this lane's output time
    loadB(tbk);
    for (int g = 0; g < ngroups; ++g) {
      floatx16 cre[kMixGroup], cim[kMixGroup];
#pragma unroll
      for (int t = 0; t < kMixGroup; ++t) {
        cre[t] = floatx16{};
        cim[t] = floatx16{};
      }
      floatG bcur = cb[g * 32], bnext = bcur;
#pragma unroll
      for (int s = 0; s < JP / 2; ++s) {
        if (s + 1 < JP / 2) bnext = cb[((s + 1) * 2 * NG + g) * 32];
#pragma unroll
        for (int t = 0; t < kMixGroup; ++t) {
          cre[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(bcur[t], yre[s], cre[t], 0, 0, 0);
          cim[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(bcur[t], yim[s], cim[t], 0, 0, 0);
        }
        bcur = bnext;
      }
#pragma unroll
      for (int t = 0; t < kMixGroup; ++t) {
        // register i holds kernel kb + acc_row(i, 0) (kb carries the 4 (lane / 32) part)
        const int kb = (kMixGroup * g + t) * 32 + 4 * kr;
        if (STORE) {
          float2* zt = zout + int64_t((kMixGroup * g + t) * 32) * n + t0;     // wave-uniform
#pragma unroll
          for (int i = 0; i < 16; ++i)
            if (kb + acc_row(i, 0) < nk) (zt + int64_t(acc_row(i, 0)) * n)[loff] = make_float2(cre[t][i], cim[t][i]);
        }
        if (FUSED) {
          uint32_t cross = 0;
          const uint32_t ikey = 0xFFFFFFFFu - uint32_t(m);
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int k = kb + acc_row(i, 0);
            if (k < nk) {
              const float a2 = abs2_rn(cre[t][i], cim[t][i]);
              atomicMax(&keys[k * S + slot], (unsigned long long)((uint64_t(__float_as_uint(a2)) << 32) | ikey));
              if (a2 > po.thr2) cross |= 1u << i;
            }
          }
          // crossings (rare) in a rolled loop: one copy of the record code
          if (cross) {
#pragma unroll 1
            for (int i = 0; i < 16; ++i)
              if ((cross >> i) & 1u) {
                const unsigned long long sl = atomicAdd(po.count, 1ull);
                if (int64_t(sl) < po.cap) {
                  rf_trigger tr;            // (re, im) for now; finished by k_trig_finish
                  tr.tmpl = po.tmpl0 + kb + acc_row(i, 0);
                  tr.seg = po.seg;
                  tr.idx = int32_t(m);
                  tr.absz = cre[t][i];
                  tr.argz = cim[t][i];
                  po.trig[sl] = tr;
                }
              }
          }
        }
      }
    }
  }
  if (FUSED) {
    __syncthreads();
    for (int k = threadIdx.x; k < nk; k += 64 * kMixWaves) {
      unsigned long long b = 0ull;
      for (int s2 = 0; s2 < S; ++s2) b = max(b, keys[k * S + s2]);
      if (b) atomicMax(reinterpret_cast<unsigned long long*>(po.packed + int64_t(po.seg) * po.nk + po.tmpl0 + k), b);
    }
  }
}

// trigger records written with (re, im): |z| and arg z as every read-out writes them
__global__ void k_trig_finish(rf_trigger* __restrict__ trig, const unsigned long long* __restrict__ count,
                              int64_t cap) {
  const int64_t nt = int64_t(*count) < cap ? int64_t(*count) : cap;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < nt; i += int64_t(gridDim.x) * 256) {
    rf_trigger t = trig[i];
    const float re = t.absz, im = t.argz;
    t.absz = sqrtf(abs2_rn(re, im));
    t.argz = atan2f(im, re);
    trig[i] = t;
  }
}

typedef _Float16 half8 __attribute__((ext_vector_type(8)));

// Power-of-two scale that puts the FP16 parts of the basis correlations in
// range: |y_j[m]| <= max|z_ref| ||b_j||_1 (Hoelder), max|z_ref| <= sqrt(2)
// max(|re|, |im|); the bound times the scale stays below 2^14 (four times
// under the FP16 limit, room for the transforms' rounding).  Values far below
// the bound keep their relative precision: FP16 is floating point, and the
// subnormal floor sits about 2^-38 below the bound.
__device__ inline float y_scale(const uint32_t* zmax, float l1max) {
  const float bound = 1.41421357f * __uint_as_float(*zmax) * l1max;
  if (!(bound > 0.f) || !(bound < 3.0e38f)) return 1.f;
  int e = 0;
  frexpf(bound, &e);                 // bound in [2^(e-1), 2^e)
  return ldexpf(1.f, 14 - e);
}

// conj(z) as the forward-transform input, and max(|re|, |im|) of z (one
// atomic per workgroup into zmax, which starts at zero)
__global__ __launch_bounds__(256) void k_conj_max(const float2* __restrict__ z, int64_t n,
                                                  float2* __restrict__ out, uint32_t* zmax) {
  __shared__ float wmax[4];
  float m = 0.f;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const float2 v = z[i];
    out[i] = make_float2(v.x, -v.y);
    m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicMax(zmax, __float_as_uint(fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]))));
}

// L1 norm of each basis vector (row of Bm [J][L]), one workgroup per row
__global__ __launch_bounds__(256) void k_row_l1(const double* __restrict__ Bm, int64_t L, double* __restrict__ out) {
  __shared__ double part[256];
  const double* row = Bm + int64_t(blockIdx.x) * L;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < L; i += 256) s += fabs(row[i]);
  part[threadIdx.x] = s;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = part[0];
}

// Split-FP16 mixing on v_mfma_f32_32x32x16_f16, transposed against the FP32
// mixing: rows = 32 kernels, columns = 32 output times, K = 16 basis indices,
// so that a lane holds one time of 16 kernels and every store of a row of
// accumulators writes two whole 256-byte runs of series.  y ~ y_hi + y_lo (split
// in registers from the FP32 correlations after the scale s_y) and
// C ~ C_hi + C_lo (packed at build time, scale s_c); three products per term
// (hi hi, hi lo, lo hi) with FP32 accumulation, output times 1 / (s_y s_c)
// (exact: powers of two).  8 waves (2 per SIMD; 4 waves, one per SIMD, from
// 128 basis vectors on), the packed coefficients in LDS as
// [ks][tile][plane][lane] 16-byte fragments; each wave holds its 32 times'
// fragments for all basis indices and sweeps the kernel tiles two at a time.
// Read-out: the running peak key of every (kernel, time lane) pair is an LDS
// atomic max (two time lanes per slot from 112 basis vectors on, for room),
// reduced to one global atomic per kernel and workgroup at the end; crossings
// as in the FP32 mixing.
// two waves per SIMD while the fragments fit in 256 registers, else one
template <int JP>
constexpr int mix16_waves() { return JP <= 112 ? 8 : 4; }
template <int JP>
constexpr int mix16_slots() { return JP <= 96 ? 32 : 16; }

template <int JP, bool STORE, bool FUSED>
__global__ __launch_bounds__(64 * mix16_waves<JP>(), 1) void k_mix16(const float2* __restrict__ Y, int64_t n,
                                                                     const half8* __restrict__ Cp, int nk,
                                                                     const uint32_t* __restrict__ zmax,
                                                                     float l1max, float cscale,
                                                                     float2* __restrict__ zout, PeakOut po) {
  constexpr int KS = JP / 16;
  constexpr int W = mix16_waves<JP>();
  constexpr int G = 2;
  constexpr int S = mix16_slots<JP>();
  constexpr int KP = 32 * kMixTiles;
  extern __shared__ __attribute__((aligned(16))) float smem[];
  half8* Cs = reinterpret_cast<half8*>(smem);                                                      // [KS][8][2][64]
  unsigned long long* keys = reinterpret_cast<unsigned long long*>(Cs + KS * kMixTiles * 2 * 64);  // [KP][S]
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int ntiles = (nk + 31) >> 5;
  // store offset of this lane from a tile's row of kernel 32 tile + acc_row(i, 0) at time t0
  // (below 2^29 bytes for n up to 2^24)
  const uint32_t loff = uint32_t(4 * (lane >> 5)) * uint32_t(n) + uint32_t(lane & 31);
  for (int e = threadIdx.x; e < KS * kMixTiles * 2 * 64; e += 64 * W) Cs[e] = Cp[e];
  if (FUSED)
    for (int e = threadIdx.x; e < KP * S; e += 64 * W) keys[e] = 0ull;
  __syncthreads();
  const float sy = y_scale(zmax, l1max);
  const float inv = 1.f / (sy * cscale);
  const int64_t nblk = n / (32 * W);
  const int slot = (lane & 31) / (32 / S);
  // B operand: lane holds y_{16 ks + 8 (lane / 32) + q}[t0 + lane % 32], q < 8
  const float2* Ylane = Y + int64_t(8 * (lane >> 5)) * n + 32 * wave + (lane & 31);
  for (int64_t tbk = blockIdx.x; tbk < nblk; tbk += gridDim.x) {
    const int64_t t0 = tbk * (32 * W) + 32 * wave;
    const int64_t m = t0 + (lane & 31);         // this lane's output time
    half8 y[4][KS];                             // re hi, re lo, im hi, im lo
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      float2 v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = Ylane[tbk * (32 * W) + int64_t(16 * ks + q) * n];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float re = v[q].x * sy, im = v[q].y * sy;
        const _Float16 rh = _Float16(re), ih = _Float16(im);
        y[0][ks][q] = rh;
        y[1][ks][q] = _Float16(re - float(rh));
        y[2][ks][q] = ih;
        y[3][ks][q] = _Float16(im - float(ih));
      }
    }
    for (int g = 0; G * g < ntiles; ++g) {
      floatx16 cre[G], cim[G];
#pragma unroll
      for (int t = 0; t < G; ++t) {
        cre[t] = floatx16{};
        cim[t] = floatx16{};
      }
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int t = 0; t < G; ++t) {
          const half8 ch = Cs[((ks * kMixTiles + G * g + t) * 2 + 0) * 64 + lane];
          const half8 cl = Cs[((ks * kMixTiles + G * g + t) * 2 + 1) * 64 + lane];
          cre[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ch, y[0][ks], cre[t], 0, 0, 0);
          cim[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ch, y[2][ks], cim[t], 0, 0, 0);
          cre[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(cl, y[0][ks], cre[t], 0, 0, 0);
          cim[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(cl, y[2][ks], cim[t], 0, 0, 0);
          cre[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ch, y[1][ks], cre[t], 0, 0, 0);
          cim[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ch, y[3][ks], cim[t], 0, 0, 0);
        }
#pragma unroll
      for (int t = 0; t < G; ++t) {
        // register i holds kernel kb + acc_row(i, 0) (kb carries the 4 (lane / 32) part)
        const int kb = (G * g + t) * 32 + 4 * (lane >> 5);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          cre[t][i] *= inv;
          cim[t][i] *= inv;
        }
        if (STORE) {
          float2* zt = zout + int64_t((G * g + t) * 32) * n + t0;      // wave-uniform
#pragma unroll
          for (int i = 0; i < 16; ++i)
            if (kb + acc_row(i, 0) < nk) (zt + int64_t(acc_row(i, 0)) * n)[loff] = make_float2(cre[t][i], cim[t][i]);
        }
        if (FUSED) {
          uint32_t cross = 0;
          const uint32_t ikey = 0xFFFFFFFFu - uint32_t(m);
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int k = kb + acc_row(i, 0);
            if (k < nk) {
              const float a2 = abs2_rn(cre[t][i], cim[t][i]);
              atomicMax(&keys[k * S + slot], (unsigned long long)((uint64_t(__float_as_uint(a2)) << 32) | ikey));
              if (a2 > po.thr2) cross |= 1u << i;
            }
          }
          if (cross) {
#pragma unroll 1
            for (int i = 0; i < 16; ++i)
              if ((cross >> i) & 1u) {
                const unsigned long long sl = atomicAdd(po.count, 1ull);
                if (int64_t(sl) < po.cap) {
                  rf_trigger tr;            // (re, im) for now; finished by k_trig_finish
                  tr.tmpl = po.tmpl0 + kb + acc_row(i, 0);
                  tr.seg = po.seg;
                  tr.idx = int32_t(m);
                  tr.absz = cre[t][i];
                  tr.argz = cim[t][i];
                  po.trig[sl] = tr;
                }
              }
          }
        }
      }
    }
  }
  if (FUSED) {
    __syncthreads();
    for (int k = threadIdx.x; k < nk; k += 64 * W) {
      unsigned long long b = 0ull;
      for (int s2 = 0; s2 < S; ++s2) b = max(b, keys[k * S + s2]);
      if (b) atomicMax(reinterpret_cast<unsigned long long*>(po.packed + int64_t(po.seg) * po.nk + po.tmpl0 + k), b);
    }
  }
}

// Split-FP16 mixing of large sets (more than 256 kernels or 128 basis
// vectors), tiled as a matrix product: a workgroup owns 128 kernels and sweeps
// its share of the time axis 128 times at a time; per 16 basis indices it
// stages the coefficients (128 kernels x 16, hi and lo FP16 parts) and the
// basis correlations (16 x 128 times, real and imaginary, split into hi and lo
// after the scale s_y) in LDS, double-buffered, and each of its four waves
// takes a 64-kernel x 64-time block as 2 x 2 products of 32 x 32 on
// v_mfma_f32_32x32x16_f16 (rows kernels, columns times, three products per
// term, real and imaginary parts apart).  The read-out keeps each kernel's
// running peak key as LDS atomics over the workgroup's times, flushed to one
// global atomic per kernel at the end; crossings as in the other mixings.
constexpr int kLgTimes = 128;                     // times per tile (n must be a multiple)
constexpr int kLgKern = 128;                      // kernels per workgroup
constexpr int kLgCStride = 40;                    // halves per kernel row of a C stage (2 x 16 + pad)
constexpr int kLgYStride = 24;                    // halves per time row of a Y plane (16 + pad)
constexpr int kLgSlots = 8;                       // peak-key slots per kernel
constexpr int kLgCStage = kLgKern * kLgCStride;   // halves
constexpr int kLgYStage = 4 * kLgTimes * kLgYStride;

template <bool STORE, bool FUSED>
__global__ __launch_bounds__(256, 1) void k_mix16L(const float2* __restrict__ Y, int64_t n, int KS,
                                                   const _Float16* __restrict__ CpL, int KPL, int nk,
                                                   int tiles_per_block, const uint32_t* __restrict__ zmax,
                                                   float l1max, float cscale, float2* __restrict__ zout,
                                                   PeakOut po) {
  __shared__ __attribute__((aligned(16))) _Float16 cst[2][kLgCStage];
  __shared__ __attribute__((aligned(16))) _Float16 yst[2][kLgYStage];
  __shared__ unsigned long long keys[FUSED ? kLgKern * kLgSlots : 1];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int kh = wave & 1, th = wave >> 1;            // this wave: kernels 64 kh.., times 64 th..
  const int ktile = blockIdx.x;                        // kernels 128 ktile ..
  const int64_t ntt = n / kLgTimes;
  const int64_t tt0 = int64_t(blockIdx.y) * tiles_per_block;
  const int64_t tt1 = tt0 + tiles_per_block < ntt ? tt0 + tiles_per_block : ntt;
  if (FUSED)
    for (int e = threadIdx.x; e < kLgKern * kLgSlots; e += 256) keys[e] = 0ull;
  const float sy = y_scale(zmax, l1max);
  const float inv = 1.f / (sy * cscale);
  // staging roles: C rows (thread t: kernel t / 2, plane t % 2, 16 halves = 32 bytes);
  // Y (thread t: time t % 128, basis indices 8 (t / 128) .. + 7)
  const _Float16* csrc = CpL + (int64_t(ktile) * kLgKern + (threadIdx.x >> 1)) * 32 + (threadIdx.x & 1) * 16;
  const int yt = threadIdx.x & (kLgTimes - 1), yg = threadIdx.x >> 7;
  uint4 creg[2];
  float2 yreg[8];
  auto load = [&](int64_t tt, int ks) {
    const uint4* cp = reinterpret_cast<const uint4*>(csrc + int64_t(ks) * KPL * 32);
    creg[0] = cp[0];
    creg[1] = cp[1];
    const float2* yp = Y + int64_t(16 * ks + 8 * yg) * n + tt * kLgTimes + yt;
#pragma unroll
    for (int q = 0; q < 8; ++q) yreg[q] = yp[int64_t(q) * n];
  };
  auto put = [&](int b) {
    uint4* cd = reinterpret_cast<uint4*>(&cst[b][(threadIdx.x >> 1) * kLgCStride + (threadIdx.x & 1) * 16]);
    cd[0] = creg[0];
    cd[1] = creg[1];
    half8 p[4];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const float re = yreg[q].x * sy, im = yreg[q].y * sy;
      const _Float16 rh = _Float16(re), ih = _Float16(im);
      p[0][q] = rh;
      p[1][q] = _Float16(re - float(rh));
      p[2][q] = ih;
      p[3][q] = _Float16(im - float(ih));
    }
#pragma unroll
    for (int pl = 0; pl < 4; ++pl)
      *reinterpret_cast<half8*>(&yst[b][(pl * kLgTimes + yt) * kLgYStride + 8 * yg]) = p[pl];
  };
  const int kr = lane & 31, kq = 8 * (lane >> 5);
  for (int64_t tt = tt0; tt < tt1; ++tt) {
    floatx16 acc[2][2][2];                            // [kernel tile][time tile][re, im]
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        acc[a][b][0] = floatx16{};
        acc[a][b][1] = floatx16{};
      }
    load(tt, 0);
    __syncthreads();                                  // the previous tile's readers are done
    put(0);
    __syncthreads();
    for (int ks = 0; ks < KS; ++ks) {
      const int buf = ks & 1;
      if (ks + 1 < KS) load(tt, ks + 1);
      half8 ch[2], cl[2], yv[2][4];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const _Float16* row = &cst[buf][(64 * kh + 32 * a + kr) * kLgCStride + kq];
        ch[a] = *reinterpret_cast<const half8*>(row);
        cl[a] = *reinterpret_cast<const half8*>(row + 16);
      }
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int pl = 0; pl < 4; ++pl)
          yv[b][pl] = *reinterpret_cast<const half8*>(
              &yst[buf][(pl * kLgTimes + 64 * th + 32 * b + kr) * kLgYStride + kq]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          acc[a][b][0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ch[a], yv[b][0], acc[a][b][0], 0, 0, 0);
          acc[a][b][1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ch[a], yv[b][2], acc[a][b][1], 0, 0, 0);
          acc[a][b][0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(cl[a], yv[b][0], acc[a][b][0], 0, 0, 0);
          acc[a][b][1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(cl[a], yv[b][2], acc[a][b][1], 0, 0, 0);
          acc[a][b][0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ch[a], yv[b][1], acc[a][b][0], 0, 0, 0);
          acc[a][b][1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ch[a], yv[b][3], acc[a][b][1], 0, 0, 0);
        }
      if (ks + 1 < KS) {
        put(buf ^ 1);
        __syncthreads();
      }
    }
    // epilogue: register i of lane l holds kernel 32 tile + acc_row(i, l), time 32 tile + l % 32
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int64_t m = tt * kLgTimes + 64 * th + 32 * b + kr;
        const int kb = ktile * kLgKern + 64 * kh + 32 * a;       // + acc_row(i, lane)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          acc[a][b][0][i] *= inv;
          acc[a][b][1][i] *= inv;
        }
        if (STORE) {
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int k = kb + acc_row(i, lane);
            if (k < nk) zout[int64_t(k) * n + m] = make_float2(acc[a][b][0][i], acc[a][b][1][i]);
          }
        }
        if (FUSED) {
          uint32_t cross = 0;
          const unsigned long long ikey = 0xFFFFFFFFu - uint32_t(m);
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int kl = 64 * kh + 32 * a + acc_row(i, lane);
            if (kb - 64 * kh - 32 * a + kl < nk) {
              const float a2 = abs2_rn(acc[a][b][0][i], acc[a][b][1][i]);
              atomicMax(&keys[kl * kLgSlots + (kr & (kLgSlots - 1))],
                        (unsigned long long)(uint64_t(__float_as_uint(a2)) << 32) | ikey);
              if (a2 > po.thr2) cross |= 1u << i;
            }
          }
          if (cross) {
#pragma unroll 1
            for (int i = 0; i < 16; ++i)
              if ((cross >> i) & 1u) {
                const unsigned long long sl = atomicAdd(po.count, 1ull);
                if (int64_t(sl) < po.cap) {
                  rf_trigger tr;            // (re, im) for now; finished by k_trig_finish
                  tr.tmpl = po.tmpl0 + kb + acc_row(i, lane);
                  tr.seg = po.seg;
                  tr.idx = int32_t(m);
                  tr.absz = acc[a][b][0][i];
                  tr.argz = acc[a][b][1][i];
                  po.trig[sl] = tr;
                }
              }
          }
        }
      }
  }
  if (FUSED) {
    __syncthreads();
    for (int kl = threadIdx.x; kl < kLgKern; kl += 256) {
      const int k = ktile * kLgKern + kl;
      if (k >= nk) continue;
      unsigned long long b = 0ull;
      for (int s2 = 0; s2 < kLgSlots; ++s2) b = max(b, keys[kl * kLgSlots + s2]);
      if (b) atomicMax(reinterpret_cast<unsigned long long*>(po.packed + int64_t(po.seg) * po.nk + po.tmpl0 + k), b);
    }
  }
}

void mix16L_launch(rf_ctx* ctx, const rf_factored* F, float2* zout, const PeakOut& po, bool fused) {
  int dev = 0, cus = 0;
  RF_HIP(hipGetDevice(&dev));
  RF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int ktiles = F->KPL / kLgKern;
  const int64_t ntt = F->n / kLgTimes;
  // about two workgroups per CU over all kernel tiles, each over a contiguous run of time tiles
  const int64_t ny = std::max<int64_t>(1, std::min<int64_t>(ntt, (2 * int64_t(cus) + ktiles - 1) / ktiles));
  const int per = int((ntt + ny - 1) / ny);
  const dim3 grid(unsigned(ktiles), unsigned((ntt + per - 1) / per));
  const int KS = F->JP / 16;
  const _Float16* Cp = F->CpL;
  if (zout && fused)
    hipLaunchKernelGGL((k_mix16L<true, true>), grid, dim3(256), 0, ctx->stream, F->Y, F->n, KS, Cp, F->KPL, F->nk,
                       per, F->zmax, F->l1max, F->cscale, zout, po);
  else if (zout)
    hipLaunchKernelGGL((k_mix16L<true, false>), grid, dim3(256), 0, ctx->stream, F->Y, F->n, KS, Cp, F->KPL, F->nk,
                       per, F->zmax, F->l1max, F->cscale, zout, po);
  else
    hipLaunchKernelGGL((k_mix16L<false, true>), grid, dim3(256), 0, ctx->stream, F->Y, F->n, KS, Cp, F->KPL, F->nk,
                       per, F->zmax, F->l1max, F->cscale, zout, po);
  RF_HIP(hipGetLastError());
}

template <int JP>
void mix16_launch_jp(rf_ctx* ctx, const rf_factored* F, float2* zout, const PeakOut& po, bool fused) {
  constexpr int KS = JP / 16;
  constexpr int W = mix16_waves<JP>();
  const size_t lds = sizeof(half8) * size_t(KS) * kMixTiles * 2 * 64 +
                     (fused ? sizeof(unsigned long long) * 32 * kMixTiles * mix16_slots<JP>() : 0);
  int dev = 0, cus = 0;
  RF_HIP(hipGetDevice(&dev));
  RF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t nblk = F->n / (32 * W);
  const unsigned grid = unsigned(std::max<int64_t>(1, std::min<int64_t>(nblk, cus)));
  const half8* Cp = reinterpret_cast<const half8*>(F->Cp);
#define RF_MIX16(S, FU)                                                                                  \
  do {                                                                                                   \
    auto kfn = k_mix16<JP, S, FU>;                                                                       \
    RF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kfn),                                       \
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));                   \
    hipLaunchKernelGGL(kfn, dim3(grid), dim3(64 * W), lds, ctx->stream, F->Y, F->n, Cp, F->nk, F->zmax,  \
                       F->l1max, F->cscale, zout, po);                                                   \
  } while (0)
  if (zout && fused) RF_MIX16(true, true);
  else if (zout) RF_MIX16(true, false);
  else RF_MIX16(false, true);
#undef RF_MIX16
  RF_HIP(hipGetLastError());
}

void mix16_launch(rf_ctx* ctx, const rf_factored* F, float2* zout, const PeakOut& po, bool fused) {
  switch (F->JP) {
    case 16: mix16_launch_jp<16>(ctx, F, zout, po, fused); break;
    case 32: mix16_launch_jp<32>(ctx, F, zout, po, fused); break;
    case 48: mix16_launch_jp<48>(ctx, F, zout, po, fused); break;
    case 64: mix16_launch_jp<64>(ctx, F, zout, po, fused); break;
    case 80: mix16_launch_jp<80>(ctx, F, zout, po, fused); break;
    case 96: mix16_launch_jp<96>(ctx, F, zout, po, fused); break;
    case 112: mix16_launch_jp<112>(ctx, F, zout, po, fused); break;
    case 128: mix16_launch_jp<128>(ctx, F, zout, po, fused); break;
    default: throw Error{RF_E_INVAL, "factored: basis size out of range"};
  }
}

template <int JP>
void mix_launch_jp(rf_ctx* ctx, const rf_factored* F, float2* zout, const PeakOut& po, bool fused) {
  constexpr int KP = 32 * kMixTiles;
  constexpr int kMixWaves = mix_waves<JP>();
  constexpr int kMixTimes = 32 * kMixWaves;
  const size_t lds = sizeof(float) * size_t(JP) * KP + (fused ? sizeof(unsigned long long) * KP * mix_slots<JP>() : 0);
  int dev = 0, cus = 0;
  RF_HIP(hipGetDevice(&dev));
  RF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t nblk = F->n / kMixTimes;
  const unsigned grid = unsigned(std::max<int64_t>(1, std::min<int64_t>(nblk, cus)));
#define RF_MIX(S, FU)                                                                                    \
  do {                                                                                                   \
    auto kfn = k_mix<JP, S, FU>;                                                                         \
    RF_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kfn),                                       \
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));                   \
    hipLaunchKernelGGL(kfn, dim3(grid), dim3(64 * kMixWaves), lds, ctx->stream, F->Y, F->n, F->C, F->nk, \
                       zout, po);                                                                        \
  } while (0)
  if (zout && fused) RF_MIX(true, true);
  else if (zout) RF_MIX(true, false);
  else RF_MIX(false, true);
#undef RF_MIX
  RF_HIP(hipGetLastError());
}

void mix_launch(rf_ctx* ctx, const rf_factored* F, float2* zout, const PeakOut& po, bool fused) {
  switch (F->JP) {
    case 16: mix_launch_jp<16>(ctx, F, zout, po, fused); break;
    case 32: mix_launch_jp<32>(ctx, F, zout, po, fused); break;
    case 48: mix_launch_jp<48>(ctx, F, zout, po, fused); break;
    case 64: mix_launch_jp<64>(ctx, F, zout, po, fused); break;
    case 80: mix_launch_jp<80>(ctx, F, zout, po, fused); break;
    case 96: mix_launch_jp<96>(ctx, F, zout, po, fused); break;
    case 112: mix_launch_jp<112>(ctx, F, zout, po, fused); break;
    case 128: mix_launch_jp<128>(ctx, F, zout, po, fused); break;
    default: throw Error{RF_E_INVAL, "factored: basis size out of range"};
  }
}

void free_factored(rf_factored* F) {
  if (!F) return;
  for (void* p : {(void*)F->Ub, (void*)F->C, (void*)F->Q, (void*)F->Qin, (void*)F->Y, (void*)F->Cp,
                  (void*)F->CpL, (void*)F->zmax})
    if (p) (void)hipFree(p);
  delete F;
}

}  // namespace

void trig_finish(rf_ctx* ctx, rf_trigger* trig, const unsigned long long* count, int64_t cap) {
  if (cap <= 0) return;
  hipLaunchKernelGGL(k_trig_finish, dim3(nblocks(cap, 1024)), dim3(256), 0, ctx->stream, trig, count, cap);
  RF_HIP(hipGetLastError());
}


FactoredView factored_view(const rf_factored* F) { return FactoredView{F->device, F->n, F->nk, F->large}; }

void factored_enqueue(rf_ctx* ctx, const rf_factored* F, const void* z_ref, int64_t n, rf_prec prec, void* z_out,
                      const PeakOut* po) {
  fill_u32(ctx, F->zmax, 0u, 1);
  // 512 workgroups at most: one atomic each on the one maximum (4096 took 50 us at 2^20)
  hipLaunchKernelGGL(k_conj_max, dim3(nblocks(n, 512)), dim3(256), 0, ctx->stream,
                     static_cast<const float2*>(z_ref), n, F->Qin, F->zmax);
  RF_HIP(hipGetLastError());
  fft_inverse_f32(ctx, F->Qin, F->Q, n, 1);
  // basis correlations: the band products formed inside the first transform pass, in
  // batches of at most 2^28 / n transforms (bounded transform scratch)
  const int per = int(std::max<int64_t>(1, std::min<int64_t>(F->J, (int64_t(1) << 28) / n)));
  for (int j0 = 0; j0 < F->J; j0 += per)
    fft_inverse_band_f32(ctx, F->Q, F->Ub + int64_t(j0) * F->nb, F->b0, F->nb, float(1.0 / double(n)),
                         F->Y + int64_t(j0) * n, n, std::min(per, F->J - j0));
  const PeakOut p = po ? *po : PeakOut{};
  if (F->large)
    mix16L_launch(ctx, F, static_cast<float2*>(z_out), p, po != nullptr);
  else if (prec == RF_PREC_SPLIT_FP16)
    mix16_launch(ctx, F, static_cast<float2*>(z_out), p, po != nullptr);
  else
    mix_launch(ctx, F, static_cast<float2*>(z_out), p, po != nullptr);
}

}  // namespace rf

using namespace rf;

extern "C" {

rf_status rf_factored_build(rf_ctx* ctx, const rf_kernels* K, const rf_grid* grid, double tol, int32_t jmax,
                            rf_factored** out) {
  if (!ctx) return RF_E_INVAL;
  rf_factored* F = nullptr;
  double* W = nullptr;
  rf_status st = guarded(ctx, [&] {
    validate_grid(grid);
    RF_CHECK(K && out, "rf_factored_build: null pointer");
    *out = nullptr;
    RF_CHECK(K->nk >= 1 && K->nk <= kFactMaxKernels, "rf_factored_build: 1 to 1024 kernels per set");
    RF_CHECK(jmax >= 1 && jmax <= kFactMaxBasis, "rf_factored_build: jmax must be in [1, 512]");
    RF_CHECK(std::isfinite(tol), "rf_factored_build: bad tolerance");
    const int nk = K->nk;
    const int64_t n = grid->n;
    RF_CHECK(n % kMixTimesMax == 0, "rf_factored_build: n must be a multiple of 256");
    RF_CHECK(n >= K->n_build, "rf_factored_build: grid shorter than the kernels' build length");
    int64_t M0 = INT64_MAX, M1 = INT64_MIN;
    for (int k = 0; k < nk; ++k)
      if (K->len[k] > 0) {
        M0 = std::min(M0, K->m_lo[k]);
        M1 = std::max(M1, K->m_lo[k] + K->len[k]);
      }
    RF_CHECK(M0 != INT64_MAX, "rf_factored_build: every kernel is empty");
    const int64_t L = M1 - M0;
    RF_CHECK(L <= n, "rf_factored_build: union support longer than the segment");
    F = new rf_factored();
    F->device = ctx->device;
    F->n = n;
    F->nk = nk;
    F->M0 = M0;
    F->L = L;
    int64_t jlo, jhi;
    band_limits(grid, &jlo, &jhi);
    RF_CHECK(jlo >= 0 && jhi >= jlo && jhi <= n / 2, "rf_factored_build: empty band");
    F->b0 = jlo;
    F->nb = jhi - jlo + 1;
    // dense kernel matrix and its Gram matrix (FP64)
    W = dev_alloc<double>(size_t(nk) * L, "factored: device allocation failed");
    {
      int64_t* meta = dev_alloc<int64_t>(size_t(nk) * 2, "factored: device allocation failed");
      int32_t* lend = dev_alloc<int32_t>(size_t(nk), "factored: device allocation failed");
      std::vector<int64_t> h(size_t(nk) * 2);
      for (int k = 0; k < nk; ++k) {
        h[k] = K->off[k];
        h[nk + k] = K->m_lo[k];
      }
      copy_sync(ctx, meta, h.data(), sizeof(int64_t) * h.size(), hipMemcpyHostToDevice);
      copy_sync(ctx, lend, K->len.data(), sizeof(int32_t) * nk, hipMemcpyHostToDevice);
      hipLaunchKernelGGL(k_dense, dim3(nblocks(L, 1024), unsigned(nk)), dim3(256), 0, ctx->stream, K->taps64, meta,
                         meta + nk, lend, M0, L, W);
      RF_HIP(hipGetLastError());
      RF_HIP(hipStreamSynchronize(ctx->stream));
      (void)hipFree(meta);
      (void)hipFree(lend);
    }
    double* G = dev_alloc<double>(size_t(nk) * nk, "factored: device allocation failed");
    dgemm(ctx, W, L, 0, W, L, 1, G, nk, nk, nk, L);             // G = W W^T
    std::vector<double> gh(size_t(nk) * nk);
    copy_sync(ctx, gh.data(), G, sizeof(double) * gh.size(), hipMemcpyDeviceToHost);
    (void)hipFree(G);
    std::vector<double> lam, V;
    sym_eig(gh, nk, lam, V);
    // smallest J whose largest per-kernel relative residual is within tol
    const int jcap = std::min<int>(jmax, nk);
    std::vector<double> tail(nk, 0.0), res(nk, 0.0);
    int J = jcap;
    for (int j = nk - 1; j >= 0; --j) {
      double worst = 0.0;
      for (int k = 0; k < nk; ++k) {
        // residual with basis size j + 1 is the tail from j + 1 on
        const double g = gh[size_t(k) * nk + k];
        worst = std::max(worst, g > 0 ? std::sqrt(std::max(0.0, tail[k]) / g) : 0.0);
      }
      if (j + 1 <= jcap && worst <= tol) J = j + 1;
      for (int k = 0; k < nk; ++k) tail[k] += std::max(0.0, lam[j]) * V[size_t(k) * nk + j] * V[size_t(k) * nk + j];
    }
    for (int k = 0; k < nk; ++k) {
      double t = 0.0;
      for (int j = J; j < nk; ++j) t += std::max(0.0, lam[j]) * V[size_t(k) * nk + j] * V[size_t(k) * nk + j];
      const double g = gh[size_t(k) * nk + k];
      res[k] = g > 0 ? std::sqrt(t / g) : 0.0;
    }
    F->J = J;
    F->JP = ((J + 15) / 16) * 16;
    F->large = nk > 32 * kMixTiles || F->JP > 128;
    F->KPL = ((nk + kLgKern - 1) / kLgKern) * kLgKern;
    F->KP = F->large ? F->KPL : 32 * kMixTiles;
    F->lambda = lam;
    F->resid = res;
    // basis b_j = sum_k V[k][j] w_k: B [J][L] = V_J^T W
    std::vector<double> vj(size_t(nk) * J);
    for (int k = 0; k < nk; ++k)
      for (int j = 0; j < J; ++j) vj[size_t(k) * J + j] = V[size_t(k) * nk + j];
    double* Vd = dev_alloc<double>(vj.size(), "factored: device allocation failed");
    copy_sync(ctx, Vd, vj.data(), sizeof(double) * vj.size(), hipMemcpyHostToDevice);
    double* Bm = dev_alloc<double>(size_t(J) * L, "factored: device allocation failed");
    dgemm(ctx, Vd, J, 1, W, L, 0, Bm, L, J, L, nk);
    (void)hipFree(W);
    W = nullptr;
    (void)hipFree(Vd);
    // basis spectra on the band bins, FP64 transforms in batches
    F->Ub = dev_alloc<float2>(size_t(J) * F->nb, "factored: device allocation failed");
    {
      const int per = int(std::max<int64_t>(1, std::min<int64_t>(J, (int64_t(1) << 25) / n)));
      double2* buf = static_cast<double2*>(ctx->ws[WS_BUILD].ensure(sizeof(double2) * size_t(n) * per));
      double2* tr = static_cast<double2*>(ctx->ws[WS_Y].ensure(sizeof(double2) * size_t(n) * per));
      for (int j0 = 0; j0 < J; j0 += per) {
        const int cnt = std::min(per, J - j0);
        fill_u64(ctx, reinterpret_cast<uint64_t*>(buf), 0ull, int64_t(2) * n * cnt);
        hipLaunchKernelGGL(k_place, dim3(nblocks(L, 1024), unsigned(cnt)), dim3(256), 0, ctx->stream,
                           Bm + int64_t(j0) * L, L, M0, n, buf);
        RF_HIP(hipGetLastError());
        fft_inverse_f64(ctx, buf, tr, n, cnt);
        hipLaunchKernelGGL(k_band_gather, dim3(nblocks(F->nb, 1024), unsigned(cnt)), dim3(256), 0, ctx->stream,
                           tr, n, F->b0, F->nb, F->Ub + int64_t(j0) * F->nb);
        RF_HIP(hipGetLastError());
      }
      RF_HIP(hipStreamSynchronize(ctx->stream));
    }
    // largest L1 norm of a basis vector (bounds the correlations for the FP16 split)
    {
      double* l1 = dev_alloc<double>(size_t(J), "factored: device allocation failed");
      hipLaunchKernelGGL(k_row_l1, dim3(unsigned(J)), dim3(256), 0, ctx->stream, Bm, L, l1);
      RF_HIP(hipGetLastError());
      std::vector<double> l1h(J);
      copy_sync(ctx, l1h.data(), l1, sizeof(double) * J, hipMemcpyDeviceToHost);
      (void)hipFree(l1);
      F->l1max = float(*std::max_element(l1h.begin(), l1h.end()) * (1.0 + 1e-6));
    }
    (void)hipFree(Bm);
    // mixing coefficients with the norm ratios folded in
    std::vector<float> ch(size_t(F->JP) * F->KP, 0.f);
    std::vector<double> cd(size_t(F->JP) * F->KP, 0.0);
    double cmax = 0.0;
    for (int j = 0; j < J; ++j)
      for (int k = 0; k < nk; ++k) {
        const double c = V[size_t(k) * nk + j] * K->norm_ratio[k];
        cd[size_t(j) * F->KP + k] = c;
        ch[size_t(j) * F->KP + k] = float(c);
        cmax = std::max(cmax, std::fabs(c));
      }
    if (!F->large) {
      F->C = dev_alloc<float>(ch.size(), "factored: device allocation failed");
      copy_sync(ctx, F->C, ch.data(), sizeof(float) * ch.size(), hipMemcpyHostToDevice);
    }
    // the same, split into FP16 hi + lo after a power-of-two scale (largest
    // scaled value in [2^13, 2^14)).  Small sets: in the operand layout of the
    // 32x32x16 product, lane l of k-step ks, tile t holds
    // C[16 ks + 8 (l / 32) + q][32 t + l % 32]; large sets: [ks][kernel][plane][16].
    int e2 = 0;
    std::frexp(cmax > 0 ? cmax : 1.0, &e2);
    const double cs = std::ldexp(1.0, 14 - e2);
    F->cscale = float(cs);
    if (F->large) {
      const int KS = F->JP / 16;
      std::vector<_Float16> cp(size_t(KS) * F->KPL * 32);
      for (int ks = 0; ks < KS; ++ks)
        for (int k = 0; k < F->KPL; ++k)
          for (int b = 0; b < 16; ++b) {
            const double c = cd[size_t(16 * ks + b) * F->KP + k] * cs;
            const _Float16 hi = _Float16(float(c));
            const _Float16 lo = _Float16(float(c - double(float(hi))));
            const size_t base = (size_t(ks) * F->KPL + k) * 32 + b;
            cp[base] = hi;
            cp[base + 16] = lo;
          }
      F->CpL = dev_alloc<_Float16>(cp.size(), "factored: device allocation failed");
      copy_sync(ctx, F->CpL, cp.data(), sizeof(_Float16) * cp.size(), hipMemcpyHostToDevice);
    } else {
      const int KS = F->JP / 16;
      std::vector<_Float16> cp(size_t(KS) * kMixTiles * 2 * 64 * 8);
      for (int ks = 0; ks < KS; ++ks)
        for (int t = 0; t < kMixTiles; ++t)
          for (int l = 0; l < 64; ++l)
            for (int q = 0; q < 8; ++q) {
              const double c = cd[size_t(16 * ks + 8 * (l / 32) + q) * F->KP + 32 * t + l % 32] * cs;
              const _Float16 hi = _Float16(float(c));
              const _Float16 lo = _Float16(float(c - double(float(hi))));
              const size_t base = ((size_t(ks) * kMixTiles + t) * 2) * 64 * 8 + size_t(l) * 8 + q;
              cp[base] = hi;
              cp[base + 64 * 8] = lo;
            }
      F->Cp = dev_alloc<_Float16>(cp.size(), "factored: device allocation failed");
      copy_sync(ctx, F->Cp, cp.data(), sizeof(_Float16) * cp.size(), hipMemcpyHostToDevice);
    }
    F->zmax = dev_alloc<uint32_t>(1, "factored: device allocation failed");
    // run buffers; rows J..JP-1 of Y stay zero (the mixing reads them as padding)
    F->Q = dev_alloc<float2>(size_t(n), "factored: device allocation failed");
    F->Qin = dev_alloc<float2>(size_t(n), "factored: device allocation failed");
    F->Y = dev_alloc<float2>(size_t(F->JP) * n, "factored: device allocation failed");
    fill_u64(ctx, reinterpret_cast<uint64_t*>(F->Y), 0ull, int64_t(F->JP) * n);
    RF_HIP(hipStreamSynchronize(ctx->stream));
    *out = F;
  });
  if (W) (void)hipFree(W);
  if (st != RF_OK && F) free_factored(F);
  return st;
}

rf_status rf_factored_info(const rf_factored* F, int32_t* J, int64_t* m0, int64_t* len, double* lambda,
                           double* resid) {
  if (!F) return RF_E_INVAL;
  if (J) *J = F->J;
  if (m0) *m0 = F->M0;
  if (len) *len = F->L;
  if (lambda)
    for (int k = 0; k < F->nk; ++k) lambda[k] = F->lambda[k];
  if (resid)
    for (int k = 0; k < F->nk; ++k) resid[k] = F->resid[k];
  return RF_OK;
}

rf_status snr_reconstruct_factored(rf_ctx* ctx, const rf_factored* F, const void* z_ref, int64_t n, rf_prec prec,
                                   void* z_out, const rf_peak_args* fused) {
  if (!ctx) return RF_E_INVAL;
  return guarded(ctx, [&] {
    RF_CHECK(F && z_ref, "snr_reconstruct_factored: null pointer");
    RF_CHECK(prec == RF_PREC_FP32 || prec == RF_PREC_SPLIT_FP16, "snr_reconstruct_factored: unknown precision");
    RF_CHECK(n == F->n, "snr_reconstruct_factored: series length differs from the build");
    if (F->large && prec != RF_PREC_SPLIT_FP16)
      throw Error{RF_E_UNSUPPORTED, "snr_reconstruct_factored: sets of more than 256 kernels or 128 basis "
                                    "vectors mix in split FP16 only"};
    RF_CHECK(z_out || fused, "snr_reconstruct_factored: need z_out or fused read-out");
    if (fused) {
      RF_CHECK(fused->peaks && fused->ntrig && fused->cap >= 0 && (fused->cap == 0 || fused->trig),
               "snr_reconstruct_factored: bad fused read-out arguments");
      RF_CHECK(std::isfinite(fused->thr) && fused->thr >= 0, "snr_reconstruct_factored: bad threshold");
    }
    PeakOut po{};
    uint64_t* packed = nullptr;
    if (fused) {
      packed = static_cast<uint64_t*>(ctx->ws[WS_PEAK].ensure(sizeof(uint64_t) * (F->nk + 1)));
      fill_u64(ctx, packed, 0ull, F->nk + 1);
      po.packed = packed;
      po.count = reinterpret_cast<unsigned long long*>(packed + F->nk);
      po.trig = fused->trig;
      po.cap = fused->cap;
      po.thr2 = fused->thr * fused->thr;
      po.seg = 0;
      po.nk = F->nk;
    }
    factored_enqueue(ctx, F, z_ref, n, prec, z_out, fused ? &po : nullptr);
    if (fused) trig_finish(ctx, fused->trig, po.count, fused->cap);
    if (fused) {
      peaks_finalize(ctx, packed, F->nk, fused->peaks);
      unsigned long long cnt = 0;
      RF_HIP(hipMemcpyAsync(&cnt, po.count, sizeof(cnt), hipMemcpyDeviceToHost, ctx->stream));
      RF_HIP(hipStreamSynchronize(ctx->stream));
      *fused->ntrig = int64_t(cnt);
      if (int64_t(cnt) > fused->cap) throw Error{RF_E_OVERFLOW, "snr_reconstruct_factored: trigger buffer overflow"};
    }
  });
}

rf_status rf_factored_free(rf_factored* F) {
  if (!F) return RF_E_INVAL;
  (void)hipSetDevice(F->device);
  (void)hipDeviceSynchronize();
  free_factored(F);
  return RF_OK;
}

}  // extern "C"
