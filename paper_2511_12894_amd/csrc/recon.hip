// Reconstruction of neighbour SNR series from the reference series
// (section II.B, equation convolution, on the circular segment):
//
//   z_k[m] = c_k sum_{s} z_ref[(m + s) mod n] w_k[s],   c_k = N_ref / N_k,
//
// cast as a matrix product per tile of up to 128 kernels that share one
// union support [m0, m0 + 16 ksteps): A[m][s] = z_ref[m + m0 + s] is a Hankel
// matrix of the reference series (rows: output times, real and imaginary
// parts as two operands), B[s][k] = w_k[s + m0] (zero outside kernel k's own
// support).  A workgroup owns 128 output times x 128 kernels; its four
// wavefronts each own 64 times x 64 kernels as 2 x 2 blocks of 32 x 32 MFMA
// tiles.  The Hankel operand is read from a sliding window of z_ref staged in
// LDS; B is pre-packed in fragment order so each MFMA operand is one
// coalesced 256 B / 1 KiB load.  Accumulation runs in chunks of 512 taps: the
// matrix-core accumulator restarts per chunk and is added into a second FP32
// total, which bounds the rounding growth over long kernels.
//
// Two arithmetic forms: FP32 operands on the FP32 matrix cores
// (v_mfma_f32_32x32x2_f32), and split FP16 (z = z_hi + z_lo, w = w_hi + w_lo
// after power-of-two scaling; hi*hi + hi*lo + lo*hi with
// v_mfma_f32_32x32x16_f16, FP32 accumulation).
//
// Optional fused read-out: instead of (or besides) storing the series, the
// epilogue folds every output into the per-kernel peak (|z|^2 compared in FP32,
// smallest index on ties) and appends threshold crossings.
#include "recon.h"

namespace rf {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

// Output element (row, col) held by lane `lane` in accumulator register i of a
// 32 x 32 MFMA tile: col = lane % 32, row = 8 (i / 4) + 4 (lane / 32) + i % 4.
__device__ inline int acc_row(int i, int lane) { return 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3); }

struct Best {
  float a2;
  int32_t idx;
};
__device__ inline Best better(Best a, Best b) {
  // larger |z|^2 wins; equal values: smaller index
  if (b.a2 > a.a2 || (b.a2 == a.a2 && b.idx < a.idx)) return b;
  return a;
}

__device__ inline float abs2_rn(float re, float im) {
  return __fadd_rn(__fmul_rn(re, re), __fmul_rn(im, im));
}

// Epilogue shared by both forms: scale, store and/or fold into the read-out.
// tot[tb][nb][part] holds the wave's 2 x 2 blocks of (re, im).
template <bool STORE, bool FUSED>
__device__ inline void epilogue(floatx16 (&tot)[2][2][2], const TileDev& T, int64_t n, int64_t n0,
                                int tw, int nw, int lane, const float* __restrict__ colscale,
                                const int32_t* __restrict__ slot_kernel, float extra_scale,
                                float2* __restrict__ zout, const PeakOut& po) {
#pragma unroll
  for (int nb = 0; nb < 2; ++nb) {
    const int slot = (2 * nw + nb) * 32 + (lane & 31);
    const bool live = slot < T.count;
    const int k = live ? slot_kernel[T.first + slot] : 0;
    const float cs = live ? colscale[T.first + slot] * extra_scale : 0.f;
    Best best{-1.f, INT32_MAX};
#pragma unroll
    for (int tb = 0; tb < 2; ++tb) {
      const int64_t base = n0 + 64 * tw + 32 * tb;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int64_t m = base + acc_row(i, lane);
        const float re = tot[tb][nb][0][i] * cs;
        const float im = tot[tb][nb][1][i] * cs;
        if (STORE && live) zout[int64_t(k) * n + m] = make_float2(re, im);
        if (FUSED) {
          const float a2 = abs2_rn(re, im);
          best = better(best, Best{a2, int32_t(m)});
          if (live && a2 > po.thr2) {
            const unsigned long long slot_t = atomicAdd(po.count, 1ull);
            if (int64_t(slot_t) < po.cap) {
              rf_trigger tr;
              tr.tmpl = k;
              tr.seg = po.seg;
              tr.idx = int32_t(m);
              tr.absz = sqrtf(a2);
              tr.argz = atan2f(im, re);
              po.trig[slot_t] = tr;
            }
          }
        }
      }
    }
    if (FUSED) {
      Best o{__shfl_xor(best.a2, 32), __shfl_xor(best.idx, 32)};
      best = better(best, o);
      if (live && lane < 32) {
        const uint64_t key = (uint64_t(__float_as_uint(best.a2)) << 32) |
                             uint64_t(0xFFFFFFFFu - uint32_t(best.idx));
        atomicMax(reinterpret_cast<unsigned long long*>(po.packed + int64_t(po.seg) * po.nk + k),
                  (unsigned long long)key);
      }
    }
  }
}

template <bool STORE, bool FUSED>
__global__ __launch_bounds__(256) void k_recon_f32(const float2* __restrict__ z, int64_t n,
                                                   const TileDev* __restrict__ tiles,
                                                   const float* __restrict__ b32,
                                                   const float* __restrict__ colscale,
                                                   const int32_t* __restrict__ slot_kernel,
                                                   float2* __restrict__ zout, PeakOut po) {
  __shared__ float zr[kChunk + kTimes];
  __shared__ float zi[kChunk + kTimes];
  const TileDev T = tiles[blockIdx.y];
  const int64_t n0 = int64_t(blockIdx.x) * kTimes;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tw = wave & 1, nw = wave >> 1;
  const int row = lane & 31, kh = lane >> 5;
  floatx16 tot[2][2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) tot[a][b][c] = floatx16{};
  const int64_t ntaps = T.ksteps * 16;
  const float* __restrict__ B = b32 + T.b32_off;
  const int64_t mask = n - 1;
  for (int64_t t0 = 0; t0 < ntaps; t0 += kChunk) {
    const int ch = int(ntaps - t0 < kChunk ? ntaps - t0 : kChunk);
    __syncthreads();
    for (int i = threadIdx.x; i < ch + kTimes; i += 256) {
      const float2 v = z[(n0 + T.m0 + t0 + i) & mask];
      zr[i] = v.x;
      zi[i] = v.y;
    }
    __syncthreads();
    floatx16 acc[2][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][b][c] = floatx16{};
    const float* __restrict__ Bc = B + (t0 / 2) * 256;
#pragma unroll 4
    for (int s = 0; s < ch / 2; ++s) {
      float bv[2];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) bv[nb] = Bc[(s * 4 + 2 * nw + nb) * 64 + lane];
#pragma unroll
      for (int tb = 0; tb < 2; ++tb) {
        const int idx = 64 * tw + 32 * tb + row + 2 * s + kh;
        const float ar = zr[idx], ai = zi[idx];
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
          acc[tb][nb][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bv[nb], acc[tb][nb][0], 0, 0, 0);
          acc[tb][nb][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, bv[nb], acc[tb][nb][1], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) tot[a][b][c] += acc[a][b][c];
  }
  epilogue<STORE, FUSED>(tot, T, n, n0, tw, nw, lane, colscale, slot_kernel, 1.f, zout, po);
}

// LDS window of the split reference series: 4 planes (re_hi, re_lo, im_hi,
// im_lo) x 4 copies shifted by 0..3 samples, so that the 8 consecutive
// samples an MFMA lane needs start on an 8-byte boundary in one of the copies.
constexpr int kWin = kChunk + kTimes + 16;

template <bool STORE, bool FUSED>
__global__ __launch_bounds__(256) void k_recon_f16(const __half* __restrict__ zs, int64_t n,
                                                   const TileDev* __restrict__ tiles,
                                                   const __half* __restrict__ b16,
                                                   const float* __restrict__ colscale,
                                                   const int32_t* __restrict__ slot_kernel,
                                                   const float* __restrict__ zinv,
                                                   float2* __restrict__ zout, PeakOut po) {
  __shared__ __attribute__((aligned(16))) _Float16 win[4][4][kWin];
  const TileDev T = tiles[blockIdx.y];
  const int64_t n0 = int64_t(blockIdx.x) * kTimes;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tw = wave & 1, nw = wave >> 1;
  const int row = lane & 31, kh = lane >> 5;
  const int sigma = row & 3;
  floatx16 tot[2][2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int c = 0; c < 2; ++c) tot[a][b][c] = floatx16{};
  const int64_t ntaps = T.ksteps * 16;
  const half8* __restrict__ B = reinterpret_cast<const half8*>(b16 + T.b16_off);
  const _Float16* __restrict__ zp = reinterpret_cast<const _Float16*>(zs);
  const int64_t mask = n - 1;
  for (int64_t t0 = 0; t0 < ntaps; t0 += kChunk) {
    const int ch = int(ntaps - t0 < kChunk ? ntaps - t0 : kChunk);
    __syncthreads();
    for (int i = threadIdx.x; i < ch + kTimes; i += 256) {
      const int64_t g = (n0 + T.m0 + t0 + i) & mask;
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) {
        const _Float16 v = zp[int64_t(pl) * n + g];
#pragma unroll
        for (int sg = 0; sg < 4; ++sg) {
          const int p = i - sg;
          if (p >= 0) win[pl][sg][p] = v;
        }
      }
    }
    __syncthreads();
    floatx16 acc[2][2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][b][c] = floatx16{};
    const half8* __restrict__ Bc = B + (t0 / 16) * 512;
#pragma unroll 2
    for (int s = 0; s < ch / 16; ++s) {
      half8 bh[2], bl[2];
#pragma unroll
      for (int nb = 0; nb < 2; ++nb) {
        const int blk = 2 * nw + nb;
        bh[nb] = Bc[((s * 4 + blk) * 2 + 0) * 64 + lane];
        bl[nb] = Bc[((s * 4 + blk) * 2 + 1) * 64 + lane];
      }
#pragma unroll
      for (int tb = 0; tb < 2; ++tb) {
        const int p = (row - sigma) + 64 * tw + 32 * tb + 8 * kh + 16 * s;
        half8 a[4];
#pragma unroll
        for (int pl = 0; pl < 4; ++pl) {
          const uint2* src = reinterpret_cast<const uint2*>(&win[pl][sigma][p]);
          uint2 lo = src[0], hi = src[1];
          uint4 u = make_uint4(lo.x, lo.y, hi.x, hi.y);
          __builtin_memcpy(&a[pl], &u, 16);
        }
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
#pragma unroll
          for (int part = 0; part < 2; ++part) {
            floatx16 c = acc[tb][nb][part];
            c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[2 * part + 0], bh[nb], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[2 * part + 0], bl[nb], c, 0, 0, 0);
            c = __builtin_amdgcn_mfma_f32_32x32x16_f16(a[2 * part + 1], bh[nb], c, 0, 0, 0);
            acc[tb][nb][part] = c;
          }
        }
      }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c) tot[a][b][c] += acc[a][b][c];
  }
  epilogue<STORE, FUSED>(tot, T, n, n0, tw, nw, lane, colscale, slot_kernel, *zinv, zout, po);
}

// max(|re|, |im|) over the series, as float bits (non-negative floats order as integers)
__global__ __launch_bounds__(256) void k_absmax(const float2* __restrict__ z, int64_t n,
                                                uint32_t* out) {
  float m = 0.f;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const float2 v = z[i];
    m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

// Split into 4 FP16 planes after scaling by s = 2^e, max * s in [2^13, 2^14).
__global__ __launch_bounds__(256) void k_split(const float2* __restrict__ z, int64_t n,
                                               const uint32_t* __restrict__ maxbits, __half* zs,
                                               float* inv_scale) {
  const float mx = __uint_as_float(*maxbits);
  int ex = 0;
  frexpf(mx, &ex);
  const float s = mx > 0.f ? ldexpf(1.f, 14 - ex) : 1.f;
  if (blockIdx.x == 0 && threadIdx.x == 0) *inv_scale = 1.f / s;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const float2 v = z[i];
    const float re = v.x * s, im = v.y * s;
    const __half rh = __float2half_rn(re), ih = __float2half_rn(im);
    zs[i] = rh;
    zs[n + i] = __float2half_rn(re - __half2float(rh));
    zs[2 * n + i] = ih;
    zs[3 * n + i] = __float2half_rn(im - __half2float(ih));
  }
}

__device__ inline double tap_of(const double* __restrict__ taps64, const int64_t* __restrict__ off,
                                const int64_t* __restrict__ mlo, const int32_t* __restrict__ len,
                                int k, int64_t tap) {
  const int64_t l = tap - mlo[k];
  return (l >= 0 && l < len[k]) ? taps64[off[k] + l] : 0.0;
}

__global__ void k_pack_b32(const double* __restrict__ taps64, const int64_t* __restrict__ off,
                           const int64_t* __restrict__ mlo, const int32_t* __restrict__ len,
                           const TileDev* __restrict__ tiles, const int32_t* __restrict__ slot_kernel,
                           float* b32) {
  const TileDev T = tiles[blockIdx.y];
  const int64_t total = T.ksteps * 8 * 4 * 64;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t s = e / 256;
    const int blk = int((e / 64) & 3), lane = int(e & 63);
    const int slot = blk * 32 + (lane & 31);
    double v = 0.0;
    if (slot < T.count) v = tap_of(taps64, off, mlo, len, slot_kernel[T.first + slot], T.m0 + 2 * s + (lane >> 5));
    b32[T.b32_off + e] = float(v);
  }
}

__global__ void k_pack_b16(const double* __restrict__ taps64, const int64_t* __restrict__ off,
                           const int64_t* __restrict__ mlo, const int32_t* __restrict__ len,
                           const double* __restrict__ kscale, const TileDev* __restrict__ tiles,
                           const int32_t* __restrict__ slot_kernel, __half* b16) {
  const TileDev T = tiles[blockIdx.y];
  const int64_t total = T.ksteps * 4 * 2 * 64 * 8;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t s = e / 4096;
    const int blk = int((e / 1024) & 3), part = int((e / 512) & 1), lane = int((e / 8) & 63),
              ee = int(e & 7);
    const int slot = blk * 32 + (lane & 31);
    float out = 0.f;
    if (slot < T.count) {
      const int k = slot_kernel[T.first + slot];
      const double v = tap_of(taps64, off, mlo, len, k, T.m0 + 16 * s + 8 * (lane >> 5) + ee) * kscale[k];
      const __half hi = __float2half_rn(float(v));
      out = part == 0 ? __half2float(hi) : float(v - double(__half2float(hi)));
    }
    b16[T.b16_off + e] = __float2half_rn(out);
  }
}

// Standalone read-out over nt series (blockIdx.y).
__global__ __launch_bounds__(256) void k_peaks(const float2* __restrict__ z, int64_t n, PeakOut po) {
  const float2* x = z + int64_t(blockIdx.y) * n;
  Best best{-1.f, INT32_MAX};
  for (int64_t m = int64_t(blockIdx.x) * 256 + threadIdx.x; m < n; m += int64_t(gridDim.x) * 256) {
    const float2 v = x[m];
    const float a2 = abs2_rn(v.x, v.y);
    best = better(best, Best{a2, int32_t(m)});
    if (a2 > po.thr2) {
      const unsigned long long slot_t = atomicAdd(po.count, 1ull);
      if (int64_t(slot_t) < po.cap) {
        rf_trigger tr;
        tr.tmpl = int32_t(blockIdx.y);
        tr.seg = po.seg;
        tr.idx = int32_t(m);
        tr.absz = sqrtf(a2);
        tr.argz = atan2f(v.y, v.x);
        po.trig[slot_t] = tr;
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    Best q{__shfl_xor(best.a2, o), __shfl_xor(best.idx, o)};
    best = better(best, q);
  }
  if ((threadIdx.x & 63) == 0 && best.idx != INT32_MAX) {
    const uint64_t key = (uint64_t(__float_as_uint(best.a2)) << 32) |
                         uint64_t(0xFFFFFFFFu - uint32_t(best.idx));
    atomicMax(reinterpret_cast<unsigned long long*>(po.packed + int64_t(po.seg) * po.nk + blockIdx.y),
              (unsigned long long)key);
  }
}

__global__ void k_peaks_finalize(const uint64_t* __restrict__ packed, int64_t count, rf_peak* out) {
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < count;
       t += int64_t(gridDim.x) * blockDim.x) {
    const uint64_t p = packed[t];
    rf_peak pk;
    pk.max_absz = sqrtf(__uint_as_float(uint32_t(p >> 32)));
    pk.argmax = int32_t(0xFFFFFFFFu - uint32_t(p & 0xFFFFFFFFu));
    out[t] = pk;
  }
}

inline unsigned nblk(int64_t n, unsigned cap) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  return unsigned(b > cap ? cap : b);
}

}  // namespace

void recon_launch(rf_ctx* ctx, rf_prec prec, const void* zsrc, int64_t n, const TileDev* tiles,
                  int ntiles, const rf_kernels* K, const float* zinv, float2* zout, const PeakOut& po,
                  bool fused) {
  dim3 grid(unsigned(n / kTimes), unsigned(ntiles));
  const bool store = zout != nullptr;
#define RF_RECON(S, F)                                                                          \
  if (prec == RF_PREC_FP32)                                                                     \
    hipLaunchKernelGGL((k_recon_f32<S, F>), grid, dim3(256), 0, ctx->stream,                    \
                       static_cast<const float2*>(zsrc), n, tiles, K->b32, K->colscale32,       \
                       K->slot_kernel, zout, po);                                               \
  else                                                                                          \
    hipLaunchKernelGGL((k_recon_f16<S, F>), grid, dim3(256), 0, ctx->stream,                    \
                       static_cast<const __half*>(zsrc), n, tiles, K->b16, K->colscale16,       \
                       K->slot_kernel, zinv, zout, po);
  if (store && fused) {
    RF_RECON(true, true)
  } else if (store) {
    RF_RECON(true, false)
  } else {
    RF_RECON(false, true)
  }
#undef RF_RECON
  RF_HIP(hipGetLastError());
}

void split_launch(rf_ctx* ctx, const float2* z, int64_t n, uint32_t* maxbits, __half* zs,
                  float* inv_scale) {
  fill_u32(ctx, maxbits, 0u, 1);
  hipLaunchKernelGGL(k_absmax, dim3(nblk(n, 2048)), dim3(256), 0, ctx->stream, z, n, maxbits);
  RF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_split, dim3(nblk(n, 4096)), dim3(256), 0, ctx->stream, z, n, maxbits, zs,
                     inv_scale);
  RF_HIP(hipGetLastError());
}

void pack_launch(rf_ctx* ctx, const rf_kernels* K, const int64_t* off_dev, const int64_t* mlo_dev,
                 const int32_t* len_dev, const double* kscale_dev, const TileDev* tiles_dev,
                 int ntiles, int64_t max_ksteps) {
  dim3 g32(nblk(max_ksteps * 2048, 4096), unsigned(ntiles));
  hipLaunchKernelGGL(k_pack_b32, g32, dim3(256), 0, ctx->stream, K->taps64, off_dev, mlo_dev,
                     len_dev, tiles_dev, K->slot_kernel, K->b32);
  RF_HIP(hipGetLastError());
  dim3 g16(nblk(max_ksteps * 4096, 4096), unsigned(ntiles));
  hipLaunchKernelGGL(k_pack_b16, g16, dim3(256), 0, ctx->stream, K->taps64, off_dev, mlo_dev,
                     len_dev, kscale_dev, tiles_dev, K->slot_kernel, K->b16);
  RF_HIP(hipGetLastError());
}

void peaks_launch(rf_ctx* ctx, const float2* z, int nt, int64_t n, const PeakOut& po) {
  dim3 grid(nblk(n, 1024), unsigned(nt));
  hipLaunchKernelGGL(k_peaks, grid, dim3(256), 0, ctx->stream, z, n, po);
  RF_HIP(hipGetLastError());
}

void peaks_finalize(rf_ctx* ctx, const uint64_t* packed, int64_t count, rf_peak* out) {
  hipLaunchKernelGGL(k_peaks_finalize, dim3(nblk(count, 256)), dim3(256), 0, ctx->stream, packed,
                     count, out);
  RF_HIP(hipGetLastError());
}

}  // namespace rf
