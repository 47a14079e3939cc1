// Internal interface of the reconstruction and read-out kernels.
#pragma once

#include "rf_internal.h"

namespace rf {

constexpr int kTileKernels = 32;   // kernels per tile (one 32-wide MFMA block)
constexpr int kPairKernels = 16;   // kernels of a paired tile (each in two columns)
constexpr int kPairShift = 32;     // taps (and output times) between a paired tile's two columns
constexpr int kTimes = 256;        // output times per workgroup (4 waves x 64)
constexpr int kChunk = 512;        // taps per LDS window chunk / accumulation chunk
constexpr int kChunkMax = 1024;    // largest chunk a split-FP16 work item may use
// Split form: the correction products run in their own pass over window
// chunks of this fixed size, taken where the chunk holds a scaled tap of at
// least 1/2.  Fixed, so that the steps with corrections (and the sums) do not
// depend on the chunk size of the first pass; 512 rather than 1024 leaves 20 %
// fewer steps with corrections on realistic kernels.
constexpr int kCorrChunk = 512;
constexpr int kStepAlign = 8;      // tiles span a multiple of 8 16-tap steps
constexpr int kB32PerStep = 512;   // FP32 operand floats per 16-tap step of a tile
constexpr int kB16PerStep = 1024;  // FP16 operand halves per 16-tap step (hi + lo)
constexpr int kOperandPadSteps = 16; // zero steps after the last tile: operand prefetch past a
                                    // tile's end stays inside the buffer


typedef float floatx16 __attribute__((ext_vector_type(16)));

// Output element (row, col) held by lane `lane` in accumulator register i of a
// 32 x 32 MFMA tile: col = lane % 32, row = 8 (i / 4) + 4 (lane / 32) + i % 4.
__device__ inline int acc_row(int i, int lane) { return 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3); }

// Running peak of a series: larger |z|^2 wins, equal values the smaller index.
struct Best {
  float a2;
  int32_t idx;
};
__device__ inline Best better(Best a, Best b) {
  if (b.a2 > a.a2 || (b.a2 == a.a2 && b.idx < a.idx)) return b;
  return a;
}

// |z|^2 with both products and the sum rounded separately (no fused multiply-add),
// the rounding every read-out and every check of it uses
__device__ inline float abs2_rn(float re, float im) {
  return __fadd_rn(__fmul_rn(re, re), __fmul_rn(im, im));
}

// Read-out target of a launch.  packed[seg * nk + k] holds the running peak
// key (|z|^2 float bits << 32 | ~index); triggers append at *count.
struct PeakOut {
  uint64_t* packed;
  rf_trigger* trig;
  unsigned long long* count;
  int64_t cap;
  float thr2;
  int32_t seg;
  int32_t nk;
  int32_t tmpl0;   // added to blockIdx.y for the template of a peak or trigger
};

// Threshold crossing of one sample (series tmpl0 + blockIdx.y of the launch).
__device__ inline void crossing(float a2, float re, float im, int64_t m, const PeakOut& po) {
  if (a2 > po.thr2) {
    const unsigned long long slot_t = atomicAdd(po.count, 1ull);
    if (int64_t(slot_t) < po.cap) {
      rf_trigger tr;
      tr.tmpl = po.tmpl0 + int32_t(blockIdx.y);
      tr.seg = po.seg;
      tr.idx = int32_t(m);
      tr.absz = sqrtf(a2);
      tr.argz = atan2f(im, re);
      po.trig[slot_t] = tr;
    }
  }
}

// The same, the record holding the raw (re, im) in (absz, argz) for trig_finish
// to complete after the launch (the read-out code stays small).
__device__ inline void crossing_raw(float a2, float re, float im, int64_t m, const PeakOut& po) {
  if (a2 > po.thr2) {
    const unsigned long long slot_t = atomicAdd(po.count, 1ull);
    if (int64_t(slot_t) < po.cap) {
      rf_trigger tr;
      tr.tmpl = po.tmpl0 + int32_t(blockIdx.y);
      tr.seg = po.seg;
      tr.idx = int32_t(m);
      tr.absz = re;
      tr.argz = im;
      po.trig[slot_t] = tr;
    }
  }
}

// One sample of a read-out: running peak and threshold crossing.
__device__ inline void peak_visit(Best& best, float re, float im, int64_t m, const PeakOut& po) {
  const float a2 = abs2_rn(re, im);
  best = better(best, Best{a2, int32_t(m)});
  crossing(a2, re, im, m, po);
}

// The same for samples one thread visits in rising index order: a strictly
// larger |z|^2 replaces the running peak, so among equal values the first
// (smallest) index stays, as better() keeps it.
__device__ inline void peak_visit_rising(Best& best, float re, float im, int32_t m, const PeakOut& po) {
  const float a2 = abs2_rn(re, im);
  if (a2 > best.a2) {
    best.a2 = a2;
    best.idx = m;
  }
  crossing(a2, re, im, m, po);
}
// ... with raw trigger records (trig_finish completes them)
__device__ inline void peak_visit_rising_raw(Best& best, float re, float im, int32_t m, const PeakOut& po) {
  const float a2 = abs2_rn(re, im);
  if (a2 > best.a2) {
    best.a2 = a2;
    best.idx = m;
  }
  crossing_raw(a2, re, im, m, po);
}

// A workgroup's running peaks (every thread's) merged into packed[seg * nk +
// tmpl0 + blockIdx.y] (workgroups of at most 1024 threads).
__device__ inline void peak_commit(Best best, const PeakOut& po) {
  for (int o = 32; o > 0; o >>= 1) {
    Best q{__shfl_xor(best.a2, o), __shfl_xor(best.idx, o)};
    best = better(best, q);
  }
  __shared__ float sa[16];
  __shared__ int32_t si[16];
  const int wv = int(threadIdx.x >> 6), nw = int((blockDim.x + 63) >> 6);
  if ((threadIdx.x & 63) == 0) {
    sa[wv] = best.a2;
    si[wv] = best.idx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < nw; ++i) best = better(best, Best{sa[i], si[i]});
    if (best.idx != INT32_MAX) {
      const uint64_t key = (uint64_t(__float_as_uint(best.a2)) << 32) |
                           uint64_t(0xFFFFFFFFu - uint32_t(best.idx));
      unsigned long long* dst =
          reinterpret_cast<unsigned long long*>(po.packed + int64_t(po.seg) * po.nk + po.tmpl0 + blockIdx.y);
      // keys only grow: a value read at or above this key (even a stale one) makes
      // the atomic a no-op, so most workgroups of a long series skip it
      if (__hip_atomic_load(dst, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < key)
        atomicMax(dst, (unsigned long long)key);
    }
  }
}

// Batched form: a tile of some reference's kernel set (slot arrays global
// over the batch) and one unit of work of the persistent launch.
struct BatchTile {
  TileDev t;
  int32_t ref;
  int32_t pad;
};
// Work item: segment, tile, first time block, window chunk (taps) and the
// number of consecutive 256-time blocks it covers.
struct WorkItem {
  int32_t seg, tile, tblock, chunk, nblk, pad;
};
// Queues of the persistent launch: nq (1, or one per XCD) contiguous sublists of
// the item array, queue i holding items [off[i], off[i + 1]).
constexpr int kMaxQueues = 8;
struct QueueSpec {
  int32_t nq;
  int32_t off[kMaxQueues + 1];
};

void recon_launch(rf_ctx* ctx, rf_prec prec, const void* zsrc, int64_t n, const TileDev* tiles,
                  int ntiles, const rf_kernels* K, const float* zinv, float2* zout, const PeakOut& po,
                  bool fused);
void split_launch(rf_ctx* ctx, const float2* z, int64_t n, uint32_t* maxbits, __half* zs,
                  float* inv_scale, int nseries = 1);
int queue_blocks(int device);
void queue_launch(rf_ctx* ctx, int nblocks, const __half* zs_all, int64_t n, int nref,
                  const BatchTile* tiles, const WorkItem* items, const QueueSpec& qs, uint32_t* counter,
                  const __half* b16, const uint32_t* gflag, const float* colscale,
                  const int32_t* slot_kernel, const float* zinv_all, const PeakOut& po);
void pack_launch(rf_ctx* ctx, const rf_kernels* K, const int64_t* off_dev, const int64_t* mlo_dev,
                 const int32_t* len_dev, const double* kscale_dev, const TileDev* tiles_dev,
                 int ntiles, int64_t max_ksteps);
void peaks_launch(rf_ctx* ctx, const float2* z, int nt, int64_t n, const PeakOut& po);
void peaks_finalize(rf_ctx* ctx, const uint64_t* packed, int64_t count, rf_peak* out);
// Trigger records written with the raw (re, im) in (absz, argz): replace them by
// |z| and arg z as every read-out writes them (the first min(*count, cap)).
void trig_finish(rf_ctx* ctx, rf_trigger* trig, const unsigned long long* count, int64_t cap);
// Matched filter of `batch` templates (a multiple of nt, coefficients coef[b % nt])
// against the conditioned data q, as fft_inverse_tmpl_f32, with the last
// transform pass reading the series out into po instead of storing them; its
// trigger records hold the raw (re, im) until trig_finish.
void fft_inverse_tmpl_peaks_f32(rf_ctx* ctx, const rf_grid* g, const float2* q, const Tf2Coef* coef, int nt,
                                const double* moment, int batch, const PeakOut& po);

// A factored set's reconstruction of one series z_ref (n samples), enqueued on the
// context's stream: the basis correlations and the mixing into z_out and/or the
// read-out po (packed peaks at po->seg * po->nk + po->tmpl0 + k, trigger records
// raw until trig_finish).  Arguments checked by the caller.
struct FactoredView {
  int device;
  int64_t n;
  int32_t nk;
  bool large;
};
FactoredView factored_view(const rf_factored* F);
void factored_enqueue(rf_ctx* ctx, const rf_factored* F, const void* z_ref, int64_t n, rf_prec prec, void* z_out,
                      const PeakOut* po);

}  // namespace rf
