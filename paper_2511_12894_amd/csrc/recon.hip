// Reconstruction of neighbour SNR series from the reference series
// (section II.B, equation convolution, on the circular segment):
//
//   z_k[m] = c_k sum_{s} z_ref[(m + s) mod n] w_k[s],   c_k = N_ref / N_k,
//
// cast as a matrix product per tile of up to 32 kernels that share one union
// support [m0, m0 + 16 ksteps): A[m][s] = z_ref[m + m0 + s] is a Hankel matrix
// of the reference series (rows: output times; real and imaginary parts are
// two operands), B[s][k] = w_k[s + m0] (zero outside kernel k's own support).
// Kernels are sorted by first tap before tiling, so a 32-kernel tile's union
// support is close to each kernel's own, and one tile's B operand (about 2 MB)
// stays resident in an XCD's L2 while consecutive workgroups -- spread over
// all XCDs -- sweep the time axis of the same tile.
//
// A workgroup owns 256 output times x 32 kernels; each of its four wavefronts
// owns 64 times as two 32 x 32 MFMA tiles (real and imaginary part each).  A
// set's last tile of at most 16 kernels is paired: its columns 16..31 hold the
// same kernels with their taps 32 later, B[s][16 + k] = w_k[s + m0 - 32], which
// gives the outputs 32 times later from the same rows of A, so one 32 x 32 tile
// per part covers a wave's 64 times and the tile costs half the products.  The
// Hankel operand comes from a sliding window of z_ref staged in LDS (double
// buffered: the next chunk's window is loaded into registers and stored to
// the idle buffer while the current chunk computes); B is pre-packed in
// fragment order, so each operand is one coalesced load.  Software
// pipelining: register rings keep the loads of later steps in flight while
// step s runs on the matrix cores, and the loads are issued one behind each
// matrix instruction rather than in a block.  The matrix-core accumulators
// are folded into an FP64 running total at fixed intervals, bounding the
// rounding growth over long kernels.
//
// Two arithmetic forms: FP32 operands on the FP32 matrix cores
// (v_mfma_f32_32x32x2_f32), and split FP16 (z = z_hi + z_lo, w = w_hi + w_lo
// after power-of-two scaling; hi*hi + hi*lo + lo*hi with
// v_mfma_f32_32x32x16_f16, FP32 accumulation).  In the split form the second
// time block's Hankel fragment at step s is the first block's fragment at step
// s + 2, so one LDS fragment load per plane and step serves both blocks.  The
// split form takes the two correction products only in the 512-tap blocks of
// a tile where some kernel has a tap of at least half an FP16 unit after its
// scale (the kernels are a narrow peak with a long low tail; elsewhere hi*hi
// alone is within 1e-6), in a second pass over those blocks; its FP32 partial
// sums are folded into FP64 every 8 steps only in the 1024-tap blocks that
// hold a kernel's largest taps, and every 32 steps elsewhere.
//
// Optional fused read-out: instead of (or besides) storing the series, the
// epilogue folds every output into the per-kernel peak (|z|^2 compared in FP32,
// smallest index on ties) and appends threshold crossings.
#include <algorithm>

#include <type_traits>

#include "recon.h"

namespace rf {
namespace {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));

// Epilogue shared by both forms: scale, store and/or fold into the read-out.
// tot[tb][ri] holds the wave's time blocks (NTB = 2: times t_base + 32 tb of
// column slot; NTB = 1, a paired tile: times t_base + 32 (column / 16) of slot
// column % 16), real and imaginary part.
template <bool STORE, bool FUSED, int NTB>
__device__ __attribute__((always_inline)) inline void epilogue(floatx16 (&tot)[2][2], const TileDev& T,
                                                               int64_t n, int64_t t_base, int lane,
                                                               const float* __restrict__ colscale,
                                                               const int32_t* __restrict__ slot_kernel,
                                                               float extra_scale, float2* __restrict__ zout,
                                                               const PeakOut& po) {
  const int col = lane & 31;
  const int slot = NTB == 1 ? (col & (kPairKernels - 1)) : col;
  const int64_t t_col = t_base + (NTB == 1 ? (col / kPairKernels) * kPairShift : 0);
  const bool live = slot < T.count;
  const int k = live ? slot_kernel[T.first + slot] : 0;
  const float cs = live ? colscale[T.first + slot] * extra_scale : 0.f;
  Best best{-1.f, INT32_MAX};
#pragma unroll
  for (int tb = 0; tb < NTB; ++tb) {
    const int64_t base = t_col + 32 * tb;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int64_t m = base + acc_row(i, lane);
      const float re = tot[tb][0][i] * cs;
      const float im = tot[tb][1][i] * cs;
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
    if (NTB == 1) {   // the slot's other column (lane ^ 16) holds its later times
      Best o2{__shfl_xor(best.a2, kPairKernels), __shfl_xor(best.idx, kPairKernels)};
      best = better(best, o2);
    }
    if (live && lane < (NTB == 1 ? kPairKernels : 32)) {
      const uint64_t key = (uint64_t(__float_as_uint(best.a2)) << 32) |
                           uint64_t(0xFFFFFFFFu - uint32_t(best.idx));
      atomicMax(reinterpret_cast<unsigned long long*>(po.packed + int64_t(po.seg) * po.nk + k),
                (unsigned long long)key);
    }
  }
}

// Window of a chunk: samples z[(n0 + m0 + t0 + i) mod n], i < ch + kTimes + 32
// (32 extra so that the prefetch of three steps ahead stays inside the buffer).
// Steps between folds of the matrix-core accumulator into the FP64 total: FP32
// form 16 two-tap steps (32 taps), split form 8 sixteen-tap steps (128 taps)
// where the kernels' large taps are.  At |z| ~ 20 the FP32 roundings of longer
// partial sums reached 1.1e-5 (split) and 1.4e-5 (FP32) on some outputs.
constexpr int kFoldF16 = 8;
// Steps the split form's first pass loads its B fragments ahead.
constexpr int kAheadB1 = 12;
static_assert(kFoldF16 == 8, "pass 1 folds after every 8-step half of its 16-step groups");
static_assert(kAheadB1 < 16 && kAheadB1 <= kOperandPadSteps, "B ring period and operand padding");
constexpr int kFoldF32 = 16;
// Split form: the hi*hi sums are folded every kFoldF16 steps only in the
// 1024-tap blocks that hold a scaled tap of at least kFoldTap (1/64..1/32 of
// the kernel's largest, which is scaled into [2^13, 2^14)).  Elsewhere the
// partial sums stay far below |z|, and so do their FP32 roundings: folding
// only there left the largest error of every output unchanged (5.7e-6 at 64 s).
constexpr double kFoldTap = 256.0;

constexpr int kWin = kChunk + kTimes + 32;
constexpr int kWinMax = kChunkMax + kTimes + 64;   // F fragments are read up to 4 steps past a chunk
constexpr int kStage = (kWin + 255) / 256;
static_assert(kWin % 2 == 0, "window pairs");

__device__ inline void zero(floatx16 (&a)[2][2]) {
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) a[x][y] = floatx16{};
}

// FP64 running total of a wave's outputs: tot[tb][ri][i] (128 registers).
struct Tot64 {
  double v[2][2][16];
};
__device__ inline void zero64(Tot64& t) {
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 16; ++i) t.v[x][y][i] = 0.0;
}
template <int NTB>
__device__ inline void fold64(Tot64& t, floatx16 (&a)[2][2]) {
#pragma unroll
  for (int x = 0; x < NTB; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
#pragma unroll
      for (int i = 0; i < 16; ++i) t.v[x][y][i] += double(a[x][y][i]);
      a[x][y] = floatx16{};
    }
}
template <int NTB>
__device__ inline void to_f32(const Tot64& t, floatx16 (&o)[2][2]) {
#pragma unroll
  for (int x = 0; x < NTB; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 16; ++i) o[x][y][i] = float(t.v[x][y][i]);
}

// FP32 form, one workgroup: output times [n0, n0 + kTimes) of tile T; NTB time
// blocks a wave (1 for a paired tile).
template <bool STORE, bool FUSED, int NTB>
__device__ __attribute__((always_inline)) inline void recon_f32_block(float (*zr)[kWin], float (*zi)[kWin],
                                                                      const float2* __restrict__ z, int64_t n,
                                                                      const TileDev& T, const float* b32,
                                                                      const float* __restrict__ colscale,
                                                                      const int32_t* __restrict__ slot_kernel,
                                                                      float2* __restrict__ zout,
                                                                      const PeakOut& po) {
  const int64_t n0 = int64_t(blockIdx.x) * kTimes;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = lane & 31, kh = lane >> 5;
  floatx16 acc[2][2];
  Tot64 tot;
  zero64(tot);
  const int64_t ntaps = T.ksteps * 16;
  const int nch = int((ntaps + kChunk - 1) / kChunk);
  const int64_t last2 = T.ksteps * 8 - 1;           // last 2-tap step of the tile
  const float* B = b32 + T.b32_off + lane;
  const int64_t mask = n - 1;
  const int64_t gbase = n0 + T.m0;
  float2 stage[kStage];
  auto gather = [&](int64_t t0) {
#pragma unroll
    for (int r = 0; r < kStage; ++r) {
      const int i = threadIdx.x + 256 * r;
      if (i < kWin) stage[r] = z[(gbase + t0 + i) & mask];
    }
  };
  auto put = [&](int buf) {
#pragma unroll
    for (int r = 0; r < kStage; ++r) {
      const int i = threadIdx.x + 256 * r;
      if (i < kWin) {
        zr[buf][i] = stage[r].x;
        zi[buf][i] = stage[r].y;
      }
    }
  };
  if (nch > 0) {
    gather(0);
    put(0);
  }
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int64_t t0 = int64_t(c) * kChunk;
    const int ch = int(ntaps - t0 < kChunk ? ntaps - t0 : kChunk);
    const int buf = c & 1;
    const bool more = c + 1 < nch;
    if (more) gather(t0 + kChunk);
    zero(acc);
    const float* wr = &zr[buf][64 * wave + row + kh];
    const float* wi = &zi[buf][64 * wave + row + kh];
    const int64_t s0 = t0 / 2;
    const int nst = ch / 2;                 // multiple of 64 (tiles span 128-tap multiples)
    float bq[4], aq[4][2][2];
    auto load = [&](int st, float& bb, float (&aa)[2][2]) {
      const int64_t g = s0 + st < last2 ? s0 + st : last2;
      bb = B[g * 64];
#pragma unroll
      for (int tb = 0; tb < NTB; ++tb) {
        aa[tb][0] = wr[32 * tb + 2 * st];
        aa[tb][1] = wi[32 * tb + 2 * st];
      }
    };
    auto mma = [&](float bb, const float (&aa)[2][2]) {
#pragma unroll
      for (int tb = 0; tb < NTB; ++tb)
#pragma unroll
        for (int ri = 0; ri < 2; ++ri)
          acc[tb][ri] = __builtin_amdgcn_mfma_f32_32x32x2f32(aa[tb][ri], bb, acc[tb][ri], 0, 0, 0);
    };
    // the loads of a later step issue one behind each matrix instruction
    auto interleave = [] {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
      __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // global read
      for (int i = 0; i < 2 * NTB - 1; ++i) {
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS read
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
      }
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      __builtin_amdgcn_sched_barrier(0);
    };
    load(0, bq[0], aq[0]);
    load(1, bq[1], aq[1]);
    load(2, bq[2], aq[2]);
    // FP32 products enter the accumulator two at a time: it is folded into the
    // FP64 total every kFoldF32 steps, so only FP32 roundings of partial sums
    // over 32 taps reach the result, whatever the kernel length
    for (int s64 = 0; s64 < nst; s64 += kFoldF32) {
      for (int s = s64; s < s64 + kFoldF32; s += 4) {
        load(s + 3, bq[3], aq[3]);
        mma(bq[0], aq[0]);
        interleave();
        load(s + 4, bq[0], aq[0]);
        mma(bq[1], aq[1]);
        interleave();
        load(s + 5, bq[1], aq[1]);
        mma(bq[2], aq[2]);
        interleave();
        load(s + 6, bq[2], aq[2]);
        mma(bq[3], aq[3]);
        interleave();
      }
      fold64<NTB>(tot, acc);
    }
    if (more) put(buf ^ 1);
    __syncthreads();
  }
  floatx16 totf[2][2];
  to_f32<NTB>(tot, totf);
  epilogue<STORE, FUSED, NTB>(totf, T, n, n0 + 64 * wave, lane, colscale, slot_kernel, 1.f, zout, po);
}

template <bool STORE, bool FUSED>
__global__ __launch_bounds__(256, 2) void k_recon_f32(const float2* __restrict__ z, int64_t n,
                                                      const TileDev* __restrict__ tiles,
                                                      const float* b32,
                                                      const float* __restrict__ colscale,
                                                      const int32_t* __restrict__ slot_kernel,
                                                      float2* __restrict__ zout, PeakOut po) {
  __shared__ float zr[2][kWin];
  __shared__ float zi[2][kWin];
  const TileDev T = tiles[blockIdx.y];
  if (T.pair)
    recon_f32_block<STORE, FUSED, 1>(zr, zi, z, n, T, b32, colscale, slot_kernel, zout, po);
  else
    recon_f32_block<STORE, FUSED, 2>(zr, zi, z, n, T, b32, colscale, slot_kernel, zout, po);
}

// LDS window of the split reference series: 4 planes (re_hi, re_lo, im_hi,
// im_lo), each holding 4 copies shifted by 0..3 samples, so that the 8
// consecutive samples an MFMA lane needs start on an 8-byte boundary in one of
// the copies.  The copies are interleaved in 8-byte groups, (copy sg, position
// p) at half index (p & ~3) * 4 + sg * 4 + (p & 3): the 64 lanes of a fragment
// load then touch consecutive 8-byte groups (no bank conflicts).
__device__ inline int win_index(int sg, int p) { return (p & ~3) * 4 + sg * 4 + (p & 3); }

// 8 consecutive samples of one copy: two 8-byte groups 16 halves apart.
__device__ inline half8 lds_frag(const _Float16* p) {
  const uint2* src = reinterpret_cast<const uint2*>(p);
  const uint2 lo = src[0], hi = src[4];
  const uint4 u = make_uint4(lo.x, lo.y, hi.x, hi.y);
  half8 h;
  __builtin_memcpy(&h, &u, 16);
  return h;
}


// One work item of the split form: output times [n0, n0 + kTimes) of tile T,
// window chunks of `chunk` taps (256, 512 or 1024; a multiple of 64).
template <bool STORE, bool FUSED, int NTB>
__device__ __attribute__((always_inline)) inline void recon_f16_item(
    _Float16 (*win)[4][4 * kWinMax], const __half* __restrict__ zs, int64_t n, const TileDev& T, int64_t n0,
    int chunk, const __half* b16, const uint32_t* __restrict__ gflag, const float* __restrict__ colscale,
    const int32_t* __restrict__ slot_kernel, float zinv, float2* __restrict__ zout, const PeakOut& po) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row = lane & 31, kh = lane >> 5;
  const int sigma = row & 3;
  // hi*hi products accumulate in `acc`, folded into the FP64 total every
  // kFoldF16 steps where the kernels' large taps are (at most 8 FP32 roundings
  // at the size of |z| per fold; granule bit 2); the two correction products, 2^-11 smaller,
  // accumulate in `cor` over the whole item, folded once at its end.
  floatx16 acc[2][2], cor[2][2];
  Tot64 tot;
#pragma unroll
  for (int x = 0; x < NTB; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 16; ++i) tot.v[x][y][i] = 0.0;
  zero(acc);
  zero(cor);
  auto fold64 = [&](floatx16 (&a)[2][2]) {
#pragma unroll
    for (int x = 0; x < NTB; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
#pragma unroll
        for (int i = 0; i < 16; ++i) tot.v[x][y][i] += double(a[x][y][i]);
        a[x][y] = floatx16{};
      }
  };
  const int64_t ntaps = T.ksteps * 16;
  const half8* B = reinterpret_cast<const half8*>(b16 + T.b16_off) + lane;
  const uint2* __restrict__ zq = reinterpret_cast<const uint2*>(zs);   // 4 halves per element
  const int64_t mask = n - 1;
  const int64_t gbase = n0 + T.m0;        // a multiple of 4 (tiles start on 4-tap boundaries)
  // Window refill in 4-position blocks: block k of every copy sg holds samples
  // 4k + sg .. 4k + sg + 3, 16 contiguous halves (32 bytes) in the interleaved
  // layout, so block k needs samples 4k .. 4k + 6, two aligned 4-sample loads
  // per plane.  Thread t handles block t and, for chunks above 736 taps, block
  // t + 256, both through the same staging registers (two rounds per chunk).
  // The window of a chunk of cs taps holds cs + kTimes + 32 samples.
  int nblk = 0;
  uint2 stage[4][2];
  auto load_blk = [&](int64_t t0, int k, uint2 (&v)[4][2]) {
    const int64_t g = ((gbase + t0 + 4 * k) & mask) >> 2;
    const int64_t g2 = ((gbase + t0 + 4 * k + 4) & mask) >> 2;
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) {
      v[pl][0] = zq[int64_t(pl) * (n >> 2) + g];
      v[pl][1] = zq[int64_t(pl) * (n >> 2) + g2];
    }
  };
  auto store_blk = [&](int buf, int k, const uint2 (&v)[4][2]) {
#pragma unroll
    for (int pl = 0; pl < 4; ++pl) {
      // halves 0..7 of the block's samples as four 32-bit words
      const uint32_t w0 = v[pl][0].x, w1 = v[pl][0].y, w2 = v[pl][1].x, w3 = v[pl][1].y;
      const uint32_t o0 = __builtin_amdgcn_alignbit(w1, w0, 16);   // halves 1, 2
      const uint32_t o1 = __builtin_amdgcn_alignbit(w2, w1, 16);   // halves 3, 4
      const uint32_t o2 = __builtin_amdgcn_alignbit(w3, w2, 16);   // halves 5, 6
      // copy 0: halves 0-3, copy 1: 1-4, copy 2: 2-5, copy 3: 3-6
      uint4* dst = reinterpret_cast<uint4*>(&win[buf][pl][16 * k]);
      dst[0] = make_uint4(w0, w1, o0, o1);
      dst[1] = make_uint4(w1, w2, o1, o2);
    }
  };
  auto gather = [&](int64_t t0, int k) {
    if (k < nblk) load_blk(t0, k, stage);
  };
  auto put = [&](int buf, int k) {
    if (k < nblk) store_blk(buf, k, stage);
  };
  // fragment F(j): 8 samples at position p0 + 16 j of copy `sigma` (p0 is a
  // multiple of 4; in the interleaved layout 4 positions are 16 halves)
  const int p0 = (row - sigma) + 64 * wave + 8 * kh;
  // Granule flag bits of taps [a, b) of the tile (a a multiple of 256).
  auto flagbits = [&](int64_t a, int64_t e) {
    const int64_t b = e < ntaps ? e : ntaps;
    uint32_t need = 0;
    for (int64_t g = a / 256; g < (b + 255) / 256; ++g) need |= gflag[T.gflag_off + g];
    return __builtin_amdgcn_readfirstlane(int(need));
  };
  // Pass-2 chunk c (kCorrChunk taps) takes the correction products if one of
  // its granules has bit 1 (a scaled tap of at least 1/2).  Pass-1 chunk c
  // (`chunk` taps) takes the short folds if a granule of the 1024-tap blocks
  // (from the tile's first tap) that it lies in has bit 2: the same steps get
  // them whatever the chunk size (256, 512 or 1024), so every chunk size gives
  // the same sums.
  auto flagged = [&](int c) {
    return (flagbits(int64_t(c) * kCorrChunk, int64_t(c + 1) * kCorrChunk) & 1) != 0;
  };
  auto foldflag = [&](int c) {
    return (flagbits((int64_t(c) * chunk / 1024) * 1024, (int64_t(c + 1) * chunk + 1023) / 1024 * 1024) & 2) != 0;
  };
  // B ring, run on across consecutive chunks.  Pass 1 needs only the hi
  // fragment: step s in slot s % 16, loaded kAheadB1 steps ahead, which also
  // covers the window refill loads that the in-order load counter puts ahead
  // of the later B loads.  Pass 2: hi and lo fragments of step s in slots
  // s % 8 and 8 + s % 8, loaded six steps (of twice the matrix work) ahead.
  half8 br[16];
  // Two passes over the item's window chunks.  Pass 1 (CORR false): the
  // hi*hi product of every chunk of `chunk` taps into `acc`, folded into the
  // FP64 total every kFoldF16 steps of the chunks with bit 2 and at the pass's
  // end; it reads the hi planes and the hi operand only.  Pass 2 (CORR true):
  // the two correction products of the flagged chunks of kCorrChunk taps into
  // `cor`.  Each pass restarts the window and the rings; only the FP64 total
  // carries over from pass 1.
  auto pass = [&](auto corr_tag) {
    constexpr bool CORR = decltype(corr_tag)::value;
    const int cs = CORR ? kCorrChunk : chunk;
    const int nch = int((ntaps + cs - 1) / cs);
    nblk = (cs + kTimes + 32) / 4;
    auto next_chunk = [&](int c) {
      ++c;
      if constexpr (CORR)
        while (c < nch && !flagged(c)) ++c;
      return c;
    };
    auto loadB = [&](int64_t st, half8& h, half8& l) {   // st < ksteps + kAheadB1: inside the padding
      if (CORR) l = B[st * 128 + 64];
      h = B[st * 128];
    };
    int c = next_chunk(-1);
    if (c >= nch) return;
    gather(int64_t(c) * cs, threadIdx.x);
    put(0, threadIdx.x);
    gather(int64_t(c) * cs, threadIdx.x + 256);
    put(0, threadIdx.x + 256);
    __syncthreads();
    int buf = 0;
    int prev = -2;                          // chunk the B ring last ran through
    while (c < nch) {
      const int64_t t0 = int64_t(c) * cs;
      const int ch = int(ntaps - t0 < cs ? ntaps - t0 : cs);
      const int cn = next_chunk(c);
      const bool more = cn < nch;
      const int64_t tn = int64_t(cn) * cs;
      if (more) gather(tn, threadIdx.x);
      const int64_t s0 = t0 / 16;
      if (prev != c - 1) {
        if constexpr (CORR) {
#pragma unroll
          for (int j = 0; j < 6; ++j) loadB(s0 + j, br[j], br[8 + j]);
        } else {
          // in slot order: the load counter's waits in the step loop then
          // hold the same slack on entry as from one group to the next
#pragma unroll
          for (int j = 0; j < kAheadB1; ++j) {
            loadB(s0 + j, br[j], br[j]);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
      const _Float16* wb[4];
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) wb[pl] = &win[buf][pl][win_index(sigma, p0)];
      const int nst = ch / 16;              // multiple of 8 (tiles span 128-tap multiples)
      half8 f[8][4];                        // F ring [slot][plane], slot = step % 8
      auto loadF = [&](int j, half8 (&ff)[4]) {
#pragma unroll
        for (int pl = 0; pl < 4; ++pl)
          if (CORR || pl % 2 == 0) ff[pl] = lds_frag(wb[pl] + 64 * j);
      };
      // step s: time block 0 uses F(s), time block 1 uses F(s + 2) (a paired
      // tile has one block: its later times come from its shifted columns);
      // pass 1 the hi*hi product, pass 2 the hi*lo and lo*hi products,
      // consecutive MFMAs feeding independent accumulators
      auto mma = [&](const half8 (&f0)[4], const half8 (&f1)[4], const half8& h, const half8& l) {
#pragma unroll
        for (int part = CORR ? 1 : 0; part < (CORR ? 3 : 1); ++part)
#pragma unroll
          for (int tb = 0; tb < NTB; ++tb)
#pragma unroll
            for (int ri = 0; ri < 2; ++ri) {
              const half8 av = (tb == 0 ? f0 : f1)[2 * ri + (part == 2 ? 1 : 0)];
              const half8 bv = part == 1 ? l : h;
              if (part == 0)
                acc[tb][ri] = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, bv, acc[tb][ri], 0, 0, 0);
              else
                cor[tb][ri] = __builtin_amdgcn_mfma_f32_32x32x16_f16(av, bv, cor[tb][ri], 0, 0, 0);
            }
      };
#pragma unroll
      for (int j = 0; j < 4; ++j) loadF(j, f[j]);
      // F runs four steps ahead (slots step % 8); the LDS counter holds at most
      // 15 fragment reads in flight, so more would only wait by count.  q is a
      // multiple of 8 and, in pass 1, q % 16 == base; `pre` false: no B
      // prefetch (pass 1's last group of a tile, which no chunk follows).
      auto steps = [&](int q, auto count, auto base, auto pre) {
        constexpr int B0 = decltype(base)::value;
#pragma unroll
        for (int h = 0; h < decltype(count)::value; ++h) {
          loadF(q + h + 4, f[(h + 4) & 7]);
          if constexpr (CORR) {
            loadB(s0 + q + h + 6, br[(h + 6) & 7], br[8 + ((h + 6) & 7)]);
            mma(f[h & 7], f[(h + 2) & 7], br[h & 7], br[8 + (h & 7)]);
          } else {
            if constexpr (decltype(pre)::value)
              loadB(s0 + q + h + kAheadB1, br[(B0 + h + kAheadB1) & 15], br[(B0 + h + kAheadB1) & 15]);
            mma(f[h & 7], f[(h + 2) & 7], br[(B0 + h) & 15], br[(B0 + h) & 15]);
          }
          // the step's loads issued one behind each of its first MFMAs, so that
          // every load issues while a matrix instruction runs
          if constexpr (NTB == 1) {
            for (int i = 0; i < (CORR ? 4 : 2); ++i) {
              __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
              __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS read
            }
            __builtin_amdgcn_sched_group_barrier(0x020, CORR ? 2 : 1, 0);   // global read
          } else if constexpr (CORR) {
            for (int i = 0; i < 4; ++i) {
              __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
              __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS read
            }
            for (int i = 0; i < 2; ++i) {
              __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
              __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);   // global read
            }
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
          } else {
            for (int i = 0; i < 2; ++i) {
              __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
              __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // LDS read
            }
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      };
      // The next visited chunk's window goes to the idle buffer in two rounds:
      // block t (loaded at this chunk's start) after the first 32 steps, block
      // t + 256 (loaded then) at the chunk's end.
      // pass 1 folds acc every kFoldF16 steps only in chunks whose 1024-tap
      // blocks hold a tap of at least kFoldTap (scaled): elsewhere every tap is
      // below 1/32 of its kernel's largest and the FP32 partial sums stay small
      const bool fold_here = !CORR && foldflag(c);
      bool round1 = false;
      int q = 0;
      // pass 1: groups of 16 steps (the B ring's period), folded after each 8
      constexpr int P = CORR ? 32 : 16;
      for (; q + P <= nst; q += P) {
        if constexpr (CORR) {
          steps(q, std::integral_constant<int, 32>{}, std::integral_constant<int, 0>{}, std::true_type{});
        } else {
          steps(q, std::integral_constant<int, 8>{}, std::integral_constant<int, 0>{}, std::true_type{});
          if (fold_here) fold64(acc);
          steps(q + 8, std::integral_constant<int, 8>{}, std::integral_constant<int, 8>{}, std::true_type{});
          if (fold_here) fold64(acc);
        }
        if (more && !round1 && q + P >= 32) {
          put(buf ^ 1, threadIdx.x);
          gather(tn, threadIdx.x + 256);
          round1 = true;
        }
      }
      // the rest in groups of 8: in pass 2 up to three; in pass 1 at most one,
      // with q % 16 == 0, only in a tile's last chunk (chunks span multiples
      // of 16 steps), so it needs no B prefetch
      if constexpr (CORR) {
        for (; q < nst; q += 8)
          steps(q, std::integral_constant<int, 8>{}, std::integral_constant<int, 0>{}, std::true_type{});
      } else if (q < nst) {
        steps(q, std::integral_constant<int, 8>{}, std::integral_constant<int, 0>{}, std::false_type{});
        if (fold_here) fold64(acc);
      }
      if (more) put(buf ^ 1, threadIdx.x + (round1 ? 256 : 0));
      __syncthreads();
      prev = c;
      c = cn;
      buf ^= 1;
    }
  };
  pass(std::false_type{});
  fold64(acc);
  pass(std::true_type{});
  fold64(cor);
  floatx16 totf[2][2];
#pragma unroll
  for (int x = 0; x < NTB; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 16; ++i) totf[x][y][i] = float(tot.v[x][y][i]);
  epilogue<STORE, FUSED, NTB>(totf, T, n, n0 + 64 * wave, lane, colscale, slot_kernel, zinv, zout, po);
}

// A work item on either tile kind (the branch is uniform over the workgroup).
template <bool STORE, bool FUSED>
__device__ __attribute__((always_inline)) inline void recon_f16_any(
    _Float16 (*win)[4][4 * kWinMax], const __half* __restrict__ zs, int64_t n, const TileDev& T, int64_t n0,
    int chunk, const __half* b16, const uint32_t* __restrict__ gflag, const float* __restrict__ colscale,
    const int32_t* __restrict__ slot_kernel, float zinv, float2* __restrict__ zout, const PeakOut& po) {
  if (T.pair)
    recon_f16_item<STORE, FUSED, 1>(win, zs, n, T, n0, chunk, b16, gflag, colscale, slot_kernel, zinv, zout, po);
  else
    recon_f16_item<STORE, FUSED, 2>(win, zs, n, T, n0, chunk, b16, gflag, colscale, slot_kernel, zinv, zout, po);
}

template <bool STORE, bool FUSED>
__global__ __launch_bounds__(256, 1) void k_recon_f16(const __half* __restrict__ zs, int64_t n,
                                                      const TileDev* __restrict__ tiles,
                                                      const __half* b16,
                                                      const uint32_t* __restrict__ gflag,
                                                      const float* __restrict__ colscale,
                                                      const int32_t* __restrict__ slot_kernel,
                                                      const float* __restrict__ zinv,
                                                      float2* __restrict__ zout, PeakOut po, int chunk) {
  __shared__ __attribute__((aligned(16))) _Float16 win[2][4][4 * kWinMax];
  recon_f16_any<STORE, FUSED>(win, zs, n, tiles[blockIdx.y], int64_t(blockIdx.x) * kTimes, chunk, b16,
                              gflag, colscale, slot_kernel, *zinv, zout, po);
}

// Persistent form over a work list: every workgroup takes items
// (segment, tile, time block, chunk) from a queue in the order given (longest
// tiles first) until the list is exhausted; every wave reaches the exit.
__global__ __launch_bounds__(256, 1) void k_recon_f16_queue(const __half* __restrict__ zs_all, int64_t n,
                                                            int32_t nref,
                                                            const BatchTile* __restrict__ tiles,
                                                            const WorkItem* __restrict__ items,
                                                            QueueSpec qs, uint32_t* counter,
                                                            const __half* b16,
                                                            const uint32_t* __restrict__ gflag,
                                                            const float* __restrict__ colscale,
                                                            const int32_t* __restrict__ slot_kernel,
                                                            const float* __restrict__ zinv_all,
                                                            PeakOut po) {
  __shared__ __attribute__((aligned(16))) _Float16 win[2][4][4 * kWinMax];
  __shared__ int32_t s_item;
  // the home queue first (workgroups are dispatched to the XCDs in turn, so with
  // one queue per XCD a workgroup's home queue is its XCD's), then the others'
  // remaining items; every counter only grows, so each loop ends
  const int home = qs.nq > 1 ? int(blockIdx.x % unsigned(qs.nq)) : 0;
  for (int d = 0; d < qs.nq; ++d) {
    const int qi = (home + d) % qs.nq;
    const int32_t lo = qs.off[qi], cnt = qs.off[qi + 1] - qs.off[qi];
    for (;;) {
      if (threadIdx.x == 0) s_item = int32_t(atomicAdd(counter + qi, 1u));
      __syncthreads();
      const int32_t it = s_item;
      __syncthreads();
      if (it >= cnt) break;
      const WorkItem w = items[lo + it];
      const BatchTile bt = tiles[w.tile];
      const int64_t sr = int64_t(w.seg) * nref + bt.ref;
      PeakOut p = po;
      p.seg = w.seg;
      for (int b = 0; b < w.nblk; ++b)
        recon_f16_any<false, true>(win, zs_all + sr * 4 * n, n, bt.t, int64_t(w.tblock + b) * kTimes, w.chunk,
                                   b16, gflag, colscale, slot_kernel, zinv_all[sr], nullptr, p);
    }
  }
}

// max(|re|, |im|) over the series, as float bits (non-negative floats order as
// integers); one atomic per workgroup
__global__ __launch_bounds__(256) void k_absmax(const float2* __restrict__ z, int64_t n,
                                                uint32_t* out) {
  __shared__ float wmax[4];
  z += int64_t(blockIdx.y) * n;
  out += blockIdx.y;
  float m = 0.f;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256) {
    const float2 v = z[i];
    m = fmaxf(m, fmaxf(fabsf(v.x), fabsf(v.y)));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    atomicMax(out, __float_as_uint(fmaxf(fmaxf(wmax[0], wmax[1]), fmaxf(wmax[2], wmax[3]))));
}

// Split into 4 FP16 planes after scaling by s = 2^e, max * s in [2^13, 2^14).
__global__ __launch_bounds__(256) void k_split(const float2* __restrict__ z, int64_t n,
                                               const uint32_t* __restrict__ maxbits, __half* zs,
                                               float* inv_scale) {
  z += int64_t(blockIdx.y) * n;
  maxbits += blockIdx.y;
  zs += int64_t(blockIdx.y) * 4 * n;
  inv_scale += blockIdx.y;
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

// Kernel slot and tap shift of operand column c of tile T: column c holds slot c,
// or in a paired tile slot c mod 16, its taps kPairShift later in columns 16..31.
__device__ inline int col_slot(const TileDev& T, int c) { return T.pair ? (c & (kPairKernels - 1)) : c; }
__device__ inline int col_shift(const TileDev& T, int c) { return T.pair && c >= kPairKernels ? kPairShift : 0; }

// FP32 operand of a tile: per 2-tap step g, lane l holds column l%32 at tap
// m0 + 2 g + l/32 (w_{slot}[tap - shift]).
__global__ void k_pack_b32(const double* __restrict__ taps64, const int64_t* __restrict__ off,
                           const int64_t* __restrict__ mlo, const int32_t* __restrict__ len,
                           const TileDev* __restrict__ tiles, const int32_t* __restrict__ slot_kernel,
                           float* b32) {
  const TileDev T = tiles[blockIdx.y];
  const int64_t total = T.ksteps * kB32PerStep;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t g = e / 64;
    const int lane = int(e & 63);
    const int slot = col_slot(T, lane & 31);
    double v = 0.0;
    if (slot < T.count)
      v = tap_of(taps64, off, mlo, len, slot_kernel[T.first + slot],
                 T.m0 + 2 * g + (lane >> 5) - col_shift(T, lane & 31));
    b32[T.b32_off + e] = float(v);
  }
}

// FP16 operand of a tile: per 16-tap step s, the hi fragment then the lo
// fragment; lane l holds 8 halves of column l%32 at taps m0 + 16 s + 8 (l/32) +
// 0..7 (w_{slot}[tap - shift], scaled by the kernel's power-of-two s_k).  Also marks the tile's 256-tap
// granules (gflag, zeroed before): bit 1 where a scaled tap reaches 1/2 (the
// correction products), bit 2 where one reaches kFoldTap (the short folds).
__global__ void k_pack_b16(const double* __restrict__ taps64, const int64_t* __restrict__ off,
                           const int64_t* __restrict__ mlo, const int32_t* __restrict__ len,
                           const double* __restrict__ kscale, const TileDev* __restrict__ tiles,
                           const int32_t* __restrict__ slot_kernel, __half* b16, uint32_t* gflag) {
  const TileDev T = tiles[blockIdx.y];
  const int64_t total = T.ksteps * kB16PerStep;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t s = e / 1024;
    const int part = int((e / 512) & 1), lane = int((e / 8) & 63), ee = int(e & 7);
    const int slot = col_slot(T, lane & 31);
    float out = 0.f;
    if (slot < T.count) {
      const int k = slot_kernel[T.first + slot];
      const double v =
          tap_of(taps64, off, mlo, len, k, T.m0 + 16 * s + 8 * (lane >> 5) + ee - col_shift(T, lane & 31)) * kscale[k];
      // a tap of at least half an FP16 unit (scaled) needs the correction products
      if (part == 0 && fabs(v) >= 0.5) atomicOr(&gflag[T.gflag_off + s / 16], fabs(v) >= kFoldTap ? 3u : 1u);
      const __half hi = __float2half_rn(float(v));
      out = part == 0 ? __half2float(hi) : float(v - double(__half2float(hi)));
    }
    b16[T.b16_off + e] = __float2half_rn(out);
  }
}

// Standalone read-out over nt series (blockIdx.y).  VEC: series 16-byte aligned,
// read two samples per 16-byte load, four loads in flight per thread.
template <bool VEC>
__global__ __launch_bounds__(256) void k_peaks(const float2* __restrict__ z, int64_t n, PeakOut po) {
  const float2* x = z + int64_t(blockIdx.y) * n;
  Best best{-1.f, INT32_MAX};
  const int64_t stride = int64_t(gridDim.x) * 256;
  if constexpr (VEC) {
    const float4* x4 = reinterpret_cast<const float4*>(x);
    const int64_t n2 = n / 2;
    for (int64_t m2 = int64_t(blockIdx.x) * 256 + threadIdx.x; m2 < n2; m2 += 4 * stride) {
      float4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (m2 + u * stride < n2) v[u] = x4[m2 + u * stride];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (m2 + u * stride < n2) {
          const int64_t m = 2 * (m2 + u * stride);
          peak_visit(best, v[u].x, v[u].y, m, po);
          peak_visit(best, v[u].z, v[u].w, m + 1, po);
        }
    }
  } else {
    for (int64_t m = int64_t(blockIdx.x) * 256 + threadIdx.x; m < n; m += stride) {
      const float2 v = x[m];
      peak_visit(best, v.x, v.y, m, po);
    }
  }
  peak_commit(best, po);
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
                       static_cast<const __half*>(zsrc), n, tiles, K->b16, K->gflag,            \
                       K->colscale16, K->slot_kernel, zinv, zout, po, int(kChunkMax));
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
                  float* inv_scale, int nseries) {
  fill_u32(ctx, maxbits, 0u, nseries);
  const unsigned per = nblk(n, unsigned(std::max(64, 2048 / nseries)));
  hipLaunchKernelGGL(k_absmax, dim3(std::min(per, 512u), unsigned(nseries)), dim3(256), 0, ctx->stream, z, n,
                     maxbits);
  RF_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_split, dim3(per, unsigned(nseries)), dim3(256), 0, ctx->stream, z, n, maxbits,
                     zs, inv_scale);
  RF_HIP(hipGetLastError());
}

int queue_blocks(int device) {
  int per_cu = 0, ncu = 0;
  RF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_recon_f16_queue, 256, 0));
  RF_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device));
  return std::max(1, per_cu) * std::max(1, ncu);
}

void queue_launch(rf_ctx* ctx, int nblocks, const __half* zs_all, int64_t n, int nref,
                  const BatchTile* tiles, const WorkItem* items, const QueueSpec& qs, uint32_t* counter,
                  const __half* b16, const uint32_t* gflag, const float* colscale,
                  const int32_t* slot_kernel, const float* zinv_all, const PeakOut& po) {
  RF_CHECK(qs.nq >= 1 && qs.nq <= kMaxQueues && qs.off[0] == 0, "queue: bad queue layout");
  for (int i = 0; i < qs.nq; ++i) RF_CHECK(qs.off[i + 1] >= qs.off[i], "queue: bad queue layout");
  fill_u32(ctx, counter, 0u, qs.nq);
  hipLaunchKernelGGL(k_recon_f16_queue, dim3(unsigned(nblocks)), dim3(256), 0, ctx->stream, zs_all, n,
                     nref, tiles, items, qs, counter, b16, gflag, colscale, slot_kernel, zinv_all, po);
  RF_HIP(hipGetLastError());
}

void pack_launch(rf_ctx* ctx, const rf_kernels* K, const int64_t* off_dev, const int64_t* mlo_dev,
                 const int32_t* len_dev, const double* kscale_dev, const TileDev* tiles_dev,
                 int ntiles, int64_t max_ksteps) {
  dim3 g32(nblk(max_ksteps * kB32PerStep, 4096), unsigned(ntiles));
  hipLaunchKernelGGL(k_pack_b32, g32, dim3(256), 0, ctx->stream, K->taps64, off_dev, mlo_dev,
                     len_dev, tiles_dev, K->slot_kernel, K->b32);
  RF_HIP(hipGetLastError());
  dim3 g16(nblk(max_ksteps * kB16PerStep, 4096), unsigned(ntiles));
  hipLaunchKernelGGL(k_pack_b16, g16, dim3(256), 0, ctx->stream, K->taps64, off_dev, mlo_dev,
                     len_dev, kscale_dev, tiles_dev, K->slot_kernel, K->b16, K->gflag);
  RF_HIP(hipGetLastError());
}

void peaks_launch(rf_ctx* ctx, const float2* z, int nt, int64_t n, const PeakOut& po) {
  // about 4096 blocks in total, at least 16 and at most 1024 per series
  int64_t per = 4096 / nt;
  per = per < 16 ? 16 : (per > 1024 ? 1024 : per);
  const int64_t cap = (n + 255) / 256;
  if (per > cap) per = cap;
  const dim3 grid{unsigned(per), unsigned(nt), 1u};
  if (reinterpret_cast<uintptr_t>(z) % 16 == 0 && n % 2 == 0)
    hipLaunchKernelGGL(k_peaks<true>, grid, dim3(256), 0, ctx->stream, z, n, po);
  else
    hipLaunchKernelGGL(k_peaks<false>, grid, dim3(256), 0, ctx->stream, z, n, po);
  RF_HIP(hipGetLastError());
}

void peaks_finalize(rf_ctx* ctx, const uint64_t* packed, int64_t count, rf_peak* out) {
  hipLaunchKernelGGL(k_peaks_finalize, dim3(nblk(count, 256)), dim3(256), 0, ctx->stream, packed,
                     count, out);
  RF_HIP(hipGetLastError());
}

}  // namespace rf
