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
  float2* S = nullptr;       // [J][n]: basis spectra (zero off the band)
  float2* Y = nullptr;       // [JP][n]: basis correlations y_j (rows from J on zero)
  std::vector<double> lambda, resid;
};

namespace rf {
namespace {

template <typename T>
T* falloc(size_t count) {
  void* p = nullptr;
  if (hipMalloc(&p, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess) {
    (void)hipGetLastError();
    throw Error{RF_E_NOMEM, "factored: device allocation failed"};
  }
  return static_cast<T*>(p);
}

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

__global__ void k_conj(const float2* __restrict__ z, int64_t n, float2* __restrict__ out) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const float2 v = z[i];
    out[i] = make_float2(v.x, -v.y);
  }
}

// S[j][b0 + i] = conj(Q[b0 + i]) Ub[j][i] / n  (FFT(z_ref) = conj(Q))
__global__ void k_band_products(const float2* __restrict__ Q, const float2* __restrict__ Ub, int64_t n,
                                int64_t b0, int64_t nb, int J, float inv_n, float2* __restrict__ S) {
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < nb; i += int64_t(gridDim.x) * 256) {
    const float2 q = Q[b0 + i];
    const float xr = q.x * inv_n, xi = -q.y * inv_n;
    for (int j = 0; j < J; ++j) {
      const float2 u = Ub[int64_t(j) * nb + i];
      S[int64_t(j) * n + b0 + i] = make_float2(xr * u.x - xi * u.y, xr * u.y + xi * u.x);
    }
  }
}

// Mixing: z~_k[m] = sum_j C[j][k] y_j[m] on v_mfma_f32_32x32x2_f32, rows = 32
// output times, columns = 32 kernels, real and imaginary parts in separate
// accumulators.  A workgroup of 8 waves (4 above JP = 96) holds C in LDS as
// [j][lane][tile] so that one lane's operands of the tiles of a sweep are one
// 8- or 16-byte read.  Each wave owns 32 consecutive times per time block, keeps
// their y fragments for all j in registers and sweeps the kernel tiles 2 (or
// 4) at a time: per pair of basis indices, 4 (8) independent MFMAs.  Crossings are recorded with
// the raw (re, im) and finished by a pass over the trigger list.  Persistent
// over time blocks; peaks kept per wave in LDS, one atomic per kernel and
// workgroup at the end.
constexpr int kMixTimesMax = 256;                // n must be a multiple of this
constexpr int kMixTiles = 8;                     // kernel tiles per set (up to 256 kernels)
// two waves per SIMD (one hides the other's loads) sweeping 2 tiles at a time
// while the fragments fit in 256 registers, else one wave sweeping 4
template <int JP>
constexpr int mix_waves() { return JP <= 96 ? 8 : 4; }
template <int JP>
constexpr int mix_group() { return JP <= 96 ? 2 : 4; }
template <int JP>
constexpr bool mix_prefetch() { return false; }

template <int JP, bool STORE, bool FUSED>
__global__ __launch_bounds__(64 * mix_waves<JP>(), 1) void k_mix(const float2* __restrict__ Y, int64_t n, int J,
                                                                const float* __restrict__ Cg, int nk,
                                                                float2* __restrict__ zout, PeakOut po) {
  constexpr int kMixWaves = mix_waves<JP>();
  constexpr int kMixGroup = mix_group<JP>();
  constexpr int kMixTimes = 32 * kMixWaves;
  constexpr int KP = 32 * kMixTiles;
  extern __shared__ __attribute__((aligned(16))) float smem[];
  constexpr int NG = kMixTiles / kMixGroup;                  // sweeps per time block
  float* Cs = smem;                                          // [JP][NG][32 lanes][kMixGroup]
  Best* best = reinterpret_cast<Best*>(Cs + JP * KP);        // [kMixWaves][KP]
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int e = threadIdx.x; e < JP * KP; e += 64 * kMixWaves) {
    const int j = e / KP, k = e % KP, tile = k >> 5;
    Cs[((j * NG + tile / kMixGroup) * 32 + (k & 31)) * kMixGroup + tile % kMixGroup] = Cg[e];
  }
  if (FUSED)
    for (int e = threadIdx.x; e < kMixWaves * KP; e += 64 * kMixWaves) best[e] = Best{-1.f, INT32_MAX};
  __syncthreads();
  const int64_t nblk = n / kMixTimes;
  const int kr = lane >> 5;                      // k index of this lane's operand half
  const int ngroups = (nk + 32 * kMixGroup - 1) / (32 * kMixGroup);
  // A operand: lane holds y_{2s + kr}[t0 + lane % 32] (rows J..JP-1 of Y are zero)
  float are[JP / 2], aim[JP / 2];
  const float2* Ylane = Y + int64_t(kr) * n + 32 * wave + (lane & 31);
  auto loadA = [&](int64_t tb, float (&r)[JP / 2], float (&im)[JP / 2]) {
    const float2* p = Ylane + tb * kMixTimes;
#pragma unroll
    for (int s = 0; s < JP / 2; ++s) {
      const float2 v = p[int64_t(2 * s) * n];
      r[s] = v.x;
      im[s] = v.y;
    }
  };
  // B operands of sweep g's tiles for basis pair s: C[2s + kr][(G g + t) 32 + lane % 32],
  // consecutive lanes reading consecutive words
  typedef float floatG __attribute__((ext_vector_type(kMixGroup)));
  const floatG* cb = reinterpret_cast<const floatG*>(Cs) + kr * NG * 32 + (lane & 31);
  if (int64_t(blockIdx.x) < nblk) loadA(blockIdx.x, are, aim);
  for (int64_t tbk = blockIdx.x; tbk < nblk; tbk += gridDim.x) {
    const int64_t t0 = tbk * kMixTimes + 32 * wave;
    float nre[JP / 2], nim[JP / 2];
    if (mix_prefetch<JP>() && tbk + gridDim.x < nblk) loadA(tbk + gridDim.x, nre, nim);
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
          cre[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(are[s], bcur[t], cre[t], 0, 0, 0);
          cim[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(aim[s], bcur[t], cim[t], 0, 0, 0);
        }
        bcur = bnext;
      }
#pragma unroll
      for (int t = 0; t < kMixGroup; ++t) {
        const int k = (kMixGroup * g + t) * 32 + (lane & 31);
        const bool live = k < nk;
        Best bt{-1.f, INT32_MAX};
        uint32_t cross = 0;
        if (STORE && live) {
          // rows i, i + 1 (i even) are consecutive times: one 16-byte store
          float4* zrow = reinterpret_cast<float4*>(zout + int64_t(k) * n + t0);
#pragma unroll
          for (int i = 0; i < 16; i += 2)
            zrow[acc_row(i, lane) >> 1] = make_float4(cre[t][i], cim[t][i], cre[t][i + 1], cim[t][i + 1]);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int64_t m = t0 + acc_row(i, lane);
          const float re = cre[t][i], im = cim[t][i];
          if (FUSED) {
            const float a2 = abs2_rn(re, im);
            bt = better(bt, Best{a2, int32_t(m)});
            if (live && a2 > po.thr2) cross |= 1u << i;
          }
        }
        // crossings (rare) in a rolled loop: one copy of the record code
        if (FUSED && cross) {
#pragma unroll 1
          for (int i = 0; i < 16; ++i)
            if ((cross >> i) & 1u) {
              const unsigned long long slot = atomicAdd(po.count, 1ull);
              if (int64_t(slot) < po.cap) {
                rf_trigger tr;              // (re, im) for now; finished by k_trig_finish
                tr.tmpl = k;
                tr.seg = po.seg;
                tr.idx = int32_t(t0 + acc_row(i, lane));
                tr.absz = cre[t][i];
                tr.argz = cim[t][i];
                po.trig[slot] = tr;
              }
            }
        }
        if (FUSED) {
          const Best o{__shfl_xor(bt.a2, 32), __shfl_xor(bt.idx, 32)};
          bt = better(bt, o);
          if (lane < 32 && live) {
            Best& b = best[wave * KP + k];
            b = better(b, bt);
          }
        }
      }
    }
    if (mix_prefetch<JP>()) {
#pragma unroll
      for (int s = 0; s < JP / 2; ++s) {
        are[s] = nre[s];
        aim[s] = nim[s];
      }
    } else if (tbk + gridDim.x < nblk) {
      loadA(tbk + gridDim.x, are, aim);
    }
  }
  if (FUSED) {
    __syncthreads();
    for (int k = threadIdx.x; k < nk; k += 64 * kMixWaves) {
      Best b = best[k];
      for (int w = 1; w < kMixWaves; ++w) b = better(b, best[w * KP + k]);
      if (b.a2 >= 0.f) {
        const uint64_t key = (uint64_t(__float_as_uint(b.a2)) << 32) | uint64_t(0xFFFFFFFFu - uint32_t(b.idx));
        atomicMax(reinterpret_cast<unsigned long long*>(po.packed + int64_t(po.seg) * po.nk + k),
                  (unsigned long long)key);
      }
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

template <int JP>
void mix_launch_jp(rf_ctx* ctx, const rf_factored* F, float2* zout, const PeakOut& po, bool fused) {
  constexpr int KP = 32 * kMixTiles;
  constexpr int kMixWaves = mix_waves<JP>();
  constexpr int kMixTimes = 32 * kMixWaves;
  const size_t lds = sizeof(float) * size_t(JP) * KP + (fused ? sizeof(Best) * kMixWaves * KP : 0);
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
    hipLaunchKernelGGL(kfn, dim3(grid), dim3(64 * kMixWaves), lds, ctx->stream, F->Y, F->n, F->J, F->C,  \
                       F->nk, zout, po);                                                                 \
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
  for (void* p : {(void*)F->Ub, (void*)F->C, (void*)F->Q, (void*)F->Qin, (void*)F->S, (void*)F->Y})
    if (p) (void)hipFree(p);
  delete F;
}

void fcopy(rf_ctx* ctx, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  RF_HIP(hipMemcpyAsync(dst, src, bytes, kind, ctx->stream));
  RF_HIP(hipStreamSynchronize(ctx->stream));
}

template <typename Fn>
rf_status fguard(rf_ctx* ctx, Fn&& f) {
  try {
    RF_HIP(hipSetDevice(ctx->device));
    f();
    return RF_OK;
  } catch (const Error& e) {
    ctx->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->last_error = "host allocation failed";
    return RF_E_NOMEM;
  } catch (const std::exception& e) {
    ctx->last_error = e.what();
    return RF_E_HIP;
  }
}

}  // namespace
}  // namespace rf

using namespace rf;

extern "C" {

rf_status rf_factored_build(rf_ctx* ctx, const rf_kernels* K, const rf_grid* grid, double tol, int32_t jmax,
                            rf_factored** out) {
  if (!ctx) return RF_E_INVAL;
  rf_factored* F = nullptr;
  double* W = nullptr;
  rf_status st = fguard(ctx, [&] {
    validate_grid(grid);
    RF_CHECK(K && out, "rf_factored_build: null pointer");
    *out = nullptr;
    RF_CHECK(K->nk >= 1 && K->nk <= 32 * kMixTiles, "rf_factored_build: 1 to 256 kernels per set");
    RF_CHECK(jmax >= 1 && jmax <= 128, "rf_factored_build: jmax must be in [1, 128]");
    RF_CHECK(std::isfinite(tol), "rf_factored_build: bad tolerance");
    const int nk = K->nk;
    const int64_t n = grid->n;
    RF_CHECK(n % kMixTimesMax == 0, "rf_factored_build: n must be a multiple of 256");
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
    W = falloc<double>(size_t(nk) * L);
    {
      int64_t* meta = falloc<int64_t>(size_t(nk) * 2);
      int32_t* lend = falloc<int32_t>(size_t(nk));
      std::vector<int64_t> h(size_t(nk) * 2);
      for (int k = 0; k < nk; ++k) {
        h[k] = K->off[k];
        h[nk + k] = K->m_lo[k];
      }
      fcopy(ctx, meta, h.data(), sizeof(int64_t) * h.size(), hipMemcpyHostToDevice);
      fcopy(ctx, lend, K->len.data(), sizeof(int32_t) * nk, hipMemcpyHostToDevice);
      hipLaunchKernelGGL(k_dense, dim3(nblocks(L, 1024), unsigned(nk)), dim3(256), 0, ctx->stream, K->taps64, meta,
                         meta + nk, lend, M0, L, W);
      RF_HIP(hipGetLastError());
      RF_HIP(hipStreamSynchronize(ctx->stream));
      (void)hipFree(meta);
      (void)hipFree(lend);
    }
    double* G = falloc<double>(size_t(nk) * nk);
    dgemm(ctx, W, L, 0, W, L, 1, G, nk, nk, nk, L);             // G = W W^T
    std::vector<double> gh(size_t(nk) * nk);
    fcopy(ctx, gh.data(), G, sizeof(double) * gh.size(), hipMemcpyDeviceToHost);
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
    F->KP = 32 * kMixTiles;
    F->lambda = lam;
    F->resid = res;
    // basis b_j = sum_k V[k][j] w_k: B [J][L] = V_J^T W
    std::vector<double> vj(size_t(nk) * J);
    for (int k = 0; k < nk; ++k)
      for (int j = 0; j < J; ++j) vj[size_t(k) * J + j] = V[size_t(k) * nk + j];
    double* Vd = falloc<double>(vj.size());
    fcopy(ctx, Vd, vj.data(), sizeof(double) * vj.size(), hipMemcpyHostToDevice);
    double* Bm = falloc<double>(size_t(J) * L);
    dgemm(ctx, Vd, J, 1, W, L, 0, Bm, L, J, L, nk);
    (void)hipFree(W);
    W = nullptr;
    (void)hipFree(Vd);
    // basis spectra on the band bins, FP64 transforms in batches
    F->Ub = falloc<float2>(size_t(J) * F->nb);
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
    (void)hipFree(Bm);
    // mixing coefficients with the norm ratios folded in
    std::vector<float> ch(size_t(F->JP) * F->KP, 0.f);
    for (int j = 0; j < J; ++j)
      for (int k = 0; k < nk; ++k) ch[size_t(j) * F->KP + k] = float(V[size_t(k) * nk + j] * K->norm_ratio[k]);
    F->C = falloc<float>(ch.size());
    fcopy(ctx, F->C, ch.data(), sizeof(float) * ch.size(), hipMemcpyHostToDevice);
    // run buffers; the band products never touch the off-band bins, zeroed once
    F->Q = falloc<float2>(size_t(n));
    F->Qin = falloc<float2>(size_t(n));
    F->S = falloc<float2>(size_t(J) * n);
    F->Y = falloc<float2>(size_t(F->JP) * n);     // rows J..JP-1 stay zero (mixing pads)
    fill_u64(ctx, reinterpret_cast<uint64_t*>(F->S), 0ull, int64_t(J) * n);
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

rf_status snr_reconstruct_factored(rf_ctx* ctx, const rf_factored* F, const void* z_ref, int64_t n, void* z_out,
                                   const rf_peak_args* fused) {
  if (!ctx) return RF_E_INVAL;
  return fguard(ctx, [&] {
    RF_CHECK(F && z_ref, "snr_reconstruct_factored: null pointer");
    RF_CHECK(n == F->n, "snr_reconstruct_factored: series length differs from the build");
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
    hipLaunchKernelGGL(k_conj, dim3(nblocks(n)), dim3(256), 0, ctx->stream, static_cast<const float2*>(z_ref), n,
                       F->Qin);
    RF_HIP(hipGetLastError());
    fft_inverse_f32(ctx, F->Qin, F->Q, n, 1);
    hipLaunchKernelGGL(k_band_products, dim3(nblocks(F->nb)), dim3(256), 0, ctx->stream, F->Q, F->Ub, n, F->b0,
                       F->nb, F->J, float(1.0 / double(n)), F->S);
    RF_HIP(hipGetLastError());
    fft_inverse_f32(ctx, F->S, F->Y, n, F->J);
    mix_launch(ctx, F, static_cast<float2*>(z_out), po, fused != nullptr);
    if (fused && fused->cap > 0) {
      hipLaunchKernelGGL(k_trig_finish, dim3(nblocks(fused->cap, 1024)), dim3(256), 0, ctx->stream, fused->trig,
                         po.count, fused->cap);
      RF_HIP(hipGetLastError());
    }
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
