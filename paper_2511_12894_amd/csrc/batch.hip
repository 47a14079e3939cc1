// Batched reconstruction: several data segments x several reference groups,
// each group with its own (uneven) set of truncated kernels.  Per call, one
// device sequence -- reference matched filters of every (segment, reference),
// split of every reference series, one persistent split-FP16 reconstruction
// launch over all (segment, tile, time block) work items with the fused
// peak/threshold read-out, peak finalisation -- captured once in a hipGraph
// and replayed.  The graph reads and writes only buffers the batch owns (the
// caller's data are copied in before a replay, the read-out copied out after
// it), so a replay does not depend on the caller's pointers.  Work items are
// ordered longest tile first so the queues end on short items.  An autotuner
// chooses, per tile-length bucket (bounds at the tertiles of the batch's own
// tile lengths), the window chunk and the number of 256-time blocks per work
// item, and whether the items sit in one queue or in one queue per XCD (tiles
// dealt to the queues in turn, so a tile's operands stay in one XCD's L2), by
// timing the candidates on sampled work items on the device.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>

#include "recon.h"

struct rf_batch {
  int device = 0;
  rf_grid grid{};
  int32_t nseg = 0, nref = 0;
  int64_t n = 0;
  int32_t ktotal = 0;                  // kernels over all groups
  std::vector<int32_t> kbase;          // first global kernel index of each group
  const double* psd = nullptr;         // caller's device PSD (borrowed)
  // device tables
  rf::Tf2Coef* coef = nullptr;         // [nref]
  double* moment = nullptr;
  rf::BatchTile* tiles = nullptr;
  rf::WorkItem* items = nullptr;
  __half* b16 = nullptr;
  float* colscale = nullptr;
  int32_t* slot_kernel = nullptr;
  // host copies
  std::vector<rf::BatchTile> htiles;
  std::vector<rf::WorkItem> hitems;
  int64_t max_ksteps = 0;
  // per-call buffers
  float2* q = nullptr;                 // [nseg][band bins]: conditioned data
  float2* zref = nullptr;              // [nseg][nref][n]
  float2* fa = nullptr;                // FFT scratch owned by the batch
  float2* fb = nullptr;
  __half* zs = nullptr;                // [nseg][nref][4][n]
  uint32_t* gflag = nullptr;           // granule flags of every set's tiles
  uint32_t* maxbits = nullptr;         // [nseg * nref]
  float* zinv = nullptr;               // [nseg * nref]
  uint64_t* packed = nullptr;          // [nseg * ktotal] + trigger count
  uint32_t* counter = nullptr;
  int nblocks = 0;
  size_t items_cap = 0;                // work items the item buffer holds (one block each)
  // tuning: window chunk (taps) and 256-time blocks per work item for each tile-length
  // bucket, one queue or one per XCD, bucket bounds (16-tap steps)
  int chunk_for_bucket[3] = {512, 512, 512};
  int blocks_for_bucket[3] = {1, 1, 1};
  int xcd_queues = 0;
  int64_t bucket_hi[2] = {64, 512};
  int64_t bucket_hi_tertiles[2] = {64, 512};   // the bounds set at creation
  std::vector<int32_t> order;          // tiles with work, longest first
  rf::QueueSpec qs{};
  // buffers the captured graph reads and writes (never the caller's)
  double2* xf_own = nullptr;           // [nseg][n/2+1]: copy of the caller's data
  rf_peak* peaks_own = nullptr;        // [nseg][ktotal]
  rf_trigger* trig_own = nullptr;      // [trig_cap]
  int64_t trig_cap = 0;
  // captured graphs (reference series; reconstruction and read-out) and the
  // read-out settings they were captured with
  hipGraphExec_t exec = nullptr;
  hipGraphExec_t exec_ref = nullptr;
  int64_t g_cap = -1;
  float g_thr = -1.f;
  int64_t captures = 0, replays = 0;
  // events around the reconstruction graph of each run (on the context's stream)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  float last_recon_ms = 0.f;
};

namespace rf {
namespace {

int bucket_of(const rf_batch* b, int64_t ksteps) {
  return ksteps <= b->bucket_hi[0] ? 0 : (ksteps <= b->bucket_hi[1] ? 1 : 2);
}

void drop_graphs(rf_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->exec_ref) (void)hipGraphExecDestroy(b->exec_ref);
  b->exec = nullptr;
  b->exec_ref = nullptr;
}

void free_batch(rf_batch* b) {
  if (!b) return;
  drop_graphs(b);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  for (void* p : {(void*)b->coef, (void*)b->moment, (void*)b->tiles, (void*)b->items, (void*)b->b16,
                  (void*)b->colscale, (void*)b->slot_kernel, (void*)b->q, (void*)b->zref, (void*)b->zs,
                  (void*)b->maxbits, (void*)b->zinv, (void*)b->packed, (void*)b->counter, (void*)b->gflag,
                  (void*)b->fa, (void*)b->fb, (void*)b->xf_own, (void*)b->peaks_own, (void*)b->trig_own})
    if (p) (void)hipFree(p);
  delete b;
}

// Work items of `tiles` (positions p in a longest-first list) over segments
// [0, nseg) and time blocks [0, ntb), each tile's items in queue p % nq.
void build_items(const rf_batch* b, const std::vector<int32_t>& tiles, int nq, int32_t nseg, int32_t ntb,
                 std::vector<WorkItem>& items, QueueSpec& qs) {
  std::vector<std::vector<WorkItem>> lists(static_cast<size_t>(nq));
  for (size_t p = 0; p < tiles.size(); ++p) {
    const int32_t t = tiles[p];
    const int bk = bucket_of(b, b->htiles[t].t.ksteps);
    const int32_t nb = b->blocks_for_bucket[bk], c = b->chunk_for_bucket[bk];
    auto& L = lists[p % size_t(nq)];
    for (int32_t sg = 0; sg < nseg; ++sg)
      for (int32_t q = 0; q < ntb; q += nb) L.push_back(WorkItem{sg, t, q, c, std::min(nb, ntb - q), 0});
  }
  items.clear();
  qs = QueueSpec{};
  qs.nq = nq;
  for (int i = 0; i < nq; ++i) {
    items.insert(items.end(), lists[size_t(i)].begin(), lists[size_t(i)].end());
    qs.off[i + 1] = int32_t(items.size());
  }
  for (int i = nq + 1; i <= kMaxQueues; ++i) qs.off[i] = int32_t(items.size());
}

void upload_items(rf_batch* b) {
  build_items(b, b->order, b->xcd_queues ? kMaxQueues : 1, b->nseg, int32_t(b->n / kTimes), b->hitems, b->qs);
  RF_CHECK(b->hitems.size() <= b->items_cap, "batch: work list larger than its buffer");
  RF_HIP(hipMemcpy(b->items, b->hitems.data(), sizeof(WorkItem) * b->hitems.size(), hipMemcpyHostToDevice));
  drop_graphs(b);
}

// reference series of every (segment, reference) and their FP16 split
void enqueue_reference(rf_ctx* ctx, rf_batch* b, const void* xf) {
  condition_data(ctx, &b->grid, static_cast<const double2*>(xf), b->psd, b->q, b->nseg);
  fft_inverse_tmpl_f32(ctx, &b->grid, b->q, b->coef, b->nref, b->moment, b->zref, b->nseg * b->nref, b->fa,
                       b->fb);
  split_launch(ctx, b->zref, b->n, b->maxbits, b->zs, b->zinv, b->nseg * b->nref);
}

// the persistent reconstruction over every work item with the fused read-out
void enqueue_recon(rf_ctx* ctx, rf_batch* b, float thr, rf_peak* peaks, rf_trigger* trig, int64_t cap) {
  const int64_t np = int64_t(b->nseg) * b->ktotal;
  fill_u64(ctx, b->packed, 0ull, np + 1);
  PeakOut po{};
  po.packed = b->packed;
  po.count = reinterpret_cast<unsigned long long*>(b->packed + np);
  po.trig = trig;
  po.cap = cap;
  po.thr2 = thr * thr;
  po.seg = 0;
  po.nk = b->ktotal;
  queue_launch(ctx, b->nblocks, b->zs, b->n, b->nref, b->tiles, b->items, b->qs, b->counter, b->b16,
               b->gflag, b->colscale, b->slot_kernel, b->zinv, po);
  peaks_finalize(ctx, b->packed, np, peaks);
}

template <typename F>
hipGraphExec_t capture(rf_ctx* ctx, F&& enqueue) {
  hipGraph_t graph = nullptr;
  RF_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  try {
    enqueue();
  } catch (...) {
    hipGraph_t g2 = nullptr;
    (void)hipStreamEndCapture(ctx->stream, &g2);
    if (g2) (void)hipGraphDestroy(g2);
    throw;
  }
  RF_HIP(hipStreamEndCapture(ctx->stream, &graph));
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) throw Error{RF_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
  return exec;
}

std::string signature(const rf_batch* b) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) arch = prop.gcnArchName;
  int64_t steps = 0, smin = 0, smax = 0;
  for (int32_t t : b->order) {
    const int64_t k = b->htiles[size_t(t)].t.ksteps;
    steps += k;
    smin = smin == 0 ? k : std::min(smin, k);
    smax = std::max(smax, k);
  }
  std::ostringstream os;
  os << "arch=" << arch << ";n=" << b->n << ";seg=" << b->nseg << ";ref=" << b->nref << ";k=" << b->ktotal
     << ";tiles=" << b->order.size() << ";steps=" << steps << "," << smin << "," << smax;
  std::string s = os.str();
  for (char& c : s)
    if (c == ' ') c = '_';
  return s;
}

}  // namespace
}  // namespace rf

using namespace rf;

extern "C" {

rf_status rf_batch_create(rf_ctx* ctx, const rf_grid* grid, const double* psd, int32_t nref,
                          const rf_tmpl* refs, rf_kernels* const* ksets, int32_t nseg, rf_batch** out) {
  if (!ctx) return RF_E_INVAL;
  rf_batch* b = nullptr;
  rf_status st;
  try {
    RF_HIP(hipSetDevice(ctx->device));
    validate_grid(grid);
    RF_CHECK(psd && refs && ksets && out, "rf_batch_create: null pointer");
    RF_CHECK(nref >= 1 && nseg >= 1, "rf_batch_create: need nref >= 1 and nseg >= 1");
    RF_CHECK(int64_t(nseg) * nref <= 65535, "rf_batch_create: nseg * nref must be <= 65535");
    *out = nullptr;
    b = new rf_batch();
    b->device = ctx->device;
    b->grid = *grid;
    b->nseg = nseg;
    b->nref = nref;
    b->n = grid->n;
    b->psd = psd;
    std::vector<Tf2Coef> coef(nref);
    int64_t b16_total = 0, slot_total = 0, gflag_total = 0;
    for (int r = 0; r < nref; ++r) {
      RF_CHECK(refs[r].m1 > 0 && refs[r].m2 > 0, "rf_batch_create: template masses must be positive");
      coef[r] = tf2_coef(refs[r]);
      const rf_kernels* K = ksets[r];
      RF_CHECK(K != nullptr, "rf_batch_create: null kernel set");
      RF_CHECK(K->device == ctx->device, "rf_batch_create: kernel set on another device");
      for (const TileDev& T : K->tiles) {
        RF_CHECK(T.ksteps * 16 <= b->n, "rf_batch_create: kernel support longer than the segment");
        b16_total += T.ksteps * kB16PerStep;
      }
      slot_total += int64_t(K->tiles.size()) * kTileKernels;
      gflag_total += K->gflag_total;
    }
    // global slot arrays and tiles: group r's kernels get global indices kbase[r] + k
    b->b16 = dev_alloc<__half>(size_t(b16_total + int64_t(kOperandPadSteps) * kB16PerStep), "batch: device allocation failed");
    fill_u32(ctx, reinterpret_cast<uint32_t*>(b->b16 + b16_total), 0u, int64_t(kOperandPadSteps) * kB16PerStep / 2);
    b->colscale = dev_alloc<float>(size_t(slot_total), "batch: device allocation failed");
    b->slot_kernel = dev_alloc<int32_t>(size_t(slot_total), "batch: device allocation failed");
    b->gflag = dev_alloc<uint32_t>(size_t(std::max<int64_t>(gflag_total, 1)), "batch: device allocation failed");
    int64_t b16_off = 0, slot_off = 0, gflag_off = 0;
    int32_t kb = 0;
    std::vector<int32_t> host_slots;
    for (int r = 0; r < nref; ++r) {
      const rf_kernels* K = ksets[r];
      b->kbase.push_back(kb);
      const int64_t nslots = int64_t(K->tiles.size()) * kTileKernels;
      std::vector<int32_t> sk(static_cast<size_t>(nslots));
      RF_HIP(hipMemcpy(sk.data(), K->slot_kernel, sizeof(int32_t) * nslots, hipMemcpyDeviceToHost));
      for (auto& v : sk)
        if (v >= 0) v += kb;
      RF_HIP(hipMemcpy(b->slot_kernel + slot_off, sk.data(), sizeof(int32_t) * nslots, hipMemcpyHostToDevice));
      RF_HIP(hipMemcpy(b->colscale + slot_off, K->colscale16, sizeof(float) * nslots, hipMemcpyDeviceToDevice));
      int64_t own = 0;
      for (const TileDev& T : K->tiles) own = std::max(own, T.b16_off + T.ksteps * kB16PerStep);
      if (own > 0)
        RF_HIP(hipMemcpy(b->b16 + b16_off, K->b16, sizeof(__half) * own, hipMemcpyDeviceToDevice));
      if (K->gflag_total > 0)
        RF_HIP(hipMemcpy(b->gflag + gflag_off, K->gflag, sizeof(uint32_t) * K->gflag_total,
                         hipMemcpyDeviceToDevice));
      for (const TileDev& T : K->tiles) {
        BatchTile bt{};
        bt.t = T;
        bt.t.b16_off += b16_off;
        bt.t.gflag_off += gflag_off;
        bt.t.first += int32_t(slot_off);
        bt.ref = r;
        b->htiles.push_back(bt);
        b->max_ksteps = std::max(b->max_ksteps, T.ksteps);
      }
      b16_off += own;
      gflag_off += K->gflag_total;
      slot_off += nslots;
      kb += K->nk;
    }
    b->ktotal = kb;
    // work list: every (segment, tile, time block), longest tiles first; length
    // buckets split at the tertiles of the tile lengths
    for (size_t i = 0; i < b->htiles.size(); ++i)
      if (b->htiles[i].t.ksteps > 0) b->order.push_back(int32_t(i));
    // longest work first: a paired tile's step costs half a step of the others
    auto work = [&](int t) { return b->htiles[size_t(t)].t.ksteps * (b->htiles[size_t(t)].t.pair ? 1 : 2); };
    std::stable_sort(b->order.begin(), b->order.end(), [&](int a, int c) { return work(a) > work(c); });
    if (!b->order.empty()) {
      std::vector<int64_t> ks;
      for (int32_t t : b->order) ks.push_back(b->htiles[t].t.ksteps);
      std::sort(ks.begin(), ks.end());
      b->bucket_hi[0] = ks[(ks.size() - 1) / 3];
      b->bucket_hi[1] = ks[2 * (ks.size() - 1) / 3];
    }
    b->bucket_hi_tertiles[0] = b->bucket_hi[0];
    b->bucket_hi_tertiles[1] = b->bucket_hi[1];
    const int32_t ntb = int32_t(b->n / kTimes);
    const double nitems = double(b->order.size()) * nseg * ntb;
    RF_CHECK(nitems < double(INT32_MAX), "rf_batch_create: too many work items");
    b->items_cap = std::max<size_t>(size_t(nitems), 1);
    b->tiles = dev_alloc<BatchTile>(b->htiles.size(), "batch: device allocation failed");
    RF_HIP(hipMemcpy(b->tiles, b->htiles.data(), sizeof(BatchTile) * b->htiles.size(), hipMemcpyHostToDevice));
    b->items = dev_alloc<WorkItem>(b->items_cap, "batch: device allocation failed");
    upload_items(b);
    b->coef = dev_alloc<Tf2Coef>(size_t(nref), "batch: device allocation failed");
    RF_HIP(hipMemcpy(b->coef, coef.data(), sizeof(Tf2Coef) * nref, hipMemcpyHostToDevice));
    b->moment = dev_alloc<double>(1, "batch: device allocation failed");
    band_moment(ctx, grid, psd, b->moment);
    const size_t ns = size_t(nseg) * nref;
    int64_t jlo, jhi;
    band_limits(grid, &jlo, &jhi);
    b->q = dev_alloc<float2>(size_t(nseg) * size_t(jhi - jlo + 1), "batch: device allocation failed");
    b->zref = dev_alloc<float2>(ns * size_t(b->n), "batch: device allocation failed");
    b->zs = dev_alloc<__half>(ns * 4 * size_t(b->n), "batch: device allocation failed");
    b->maxbits = dev_alloc<uint32_t>(ns, "batch: device allocation failed");
    b->zinv = dev_alloc<float>(ns, "batch: device allocation failed");
    b->packed = dev_alloc<uint64_t>(size_t(nseg) * b->ktotal + 1, "batch: device allocation failed");
    b->counter = dev_alloc<uint32_t>(kMaxQueues, "batch: device allocation failed");
    b->nblocks = queue_blocks(ctx->device);
    // FFT scratch owned by the batch: the captured graph references it
    b->fa = dev_alloc<float2>(ns * size_t(b->n), "batch: device allocation failed");
    b->fb = dev_alloc<float2>(ns * size_t(b->n), "batch: device allocation failed");
    b->xf_own = dev_alloc<double2>(size_t(nseg) * size_t(b->n / 2 + 1), "batch: device allocation failed");
    b->peaks_own = dev_alloc<rf_peak>(size_t(nseg) * size_t(b->ktotal), "batch: device allocation failed");
    RF_HIP(hipEventCreate(&b->ev0));
    RF_HIP(hipEventCreate(&b->ev1));
    RF_HIP(hipStreamSynchronize(ctx->stream));
    *out = b;
    st = RF_OK;
  } catch (const Error& e) {
    ctx->last_error = e.msg;
    st = e.code;
  } catch (...) {
    ctx->last_error = "rf_batch_create: unexpected exception";
    st = RF_E_HIP;
  }
  if (st != RF_OK && b) free_batch(b);
  return st;
}

rf_status rf_batch_info(const rf_batch* b, int32_t* ktotal, int64_t* nitems, int32_t* kbase,
                        int32_t* chunk_per_bucket) {
  if (!b) return RF_E_INVAL;
  if (ktotal) *ktotal = b->ktotal;
  if (nitems) *nitems = int64_t(b->hitems.size());
  if (kbase)
    for (int r = 0; r < b->nref; ++r) kbase[r] = b->kbase[r];
  if (chunk_per_bucket)
    for (int i = 0; i < 3; ++i) chunk_per_bucket[i] = b->chunk_for_bucket[i];
  return RF_OK;
}

rf_status rf_batch_set_chunks(rf_batch* b, const int32_t* chunk_per_bucket) {
  if (!b || !chunk_per_bucket) return RF_E_INVAL;
  rf_batch_tuning t{};
  rf_batch_get_tuning(b, &t);
  for (int i = 0; i < 3; ++i) t.chunk[i] = chunk_per_bucket[i];
  return rf_batch_set_tuning(b, &t);
}

rf_status rf_batch_get_tuning(const rf_batch* b, rf_batch_tuning* t) {
  if (!b || !t) return RF_E_INVAL;
  *t = rf_batch_tuning{};
  for (int i = 0; i < 3; ++i) {
    t->chunk[i] = b->chunk_for_bucket[i];
    t->blocks[i] = b->blocks_for_bucket[i];
  }
  t->xcd_queues = b->xcd_queues;
  t->bucket_hi[0] = b->bucket_hi[0];
  t->bucket_hi[1] = b->bucket_hi[1];
  return RF_OK;
}

rf_status rf_batch_set_tuning(rf_batch* b, const rf_batch_tuning* t) {
  if (!b || !t) return RF_E_INVAL;
  for (int i = 0; i < 3; ++i) {
    if (t->chunk[i] != 256 && t->chunk[i] != 512 && t->chunk[i] != 1024) return RF_E_INVAL;
    if (t->blocks[i] != 1 && t->blocks[i] != 2 && t->blocks[i] != 4) return RF_E_INVAL;
  }
  if (t->xcd_queues != 0 && t->xcd_queues != 1) return RF_E_INVAL;
  if (t->bucket_hi[0] < 0 || t->bucket_hi[1] < t->bucket_hi[0]) return RF_E_INVAL;
  try {
    RF_HIP(hipSetDevice(b->device));
    for (int i = 0; i < 3; ++i) {
      b->chunk_for_bucket[i] = t->chunk[i];
      b->blocks_for_bucket[i] = t->blocks[i];
    }
    b->xcd_queues = t->xcd_queues;
    b->bucket_hi[0] = t->bucket_hi[0];
    b->bucket_hi[1] = t->bucket_hi[1];
    upload_items(b);
  } catch (const Error& e) {
    return e.code;
  }
  return RF_OK;
}

rf_status rf_batch_autotune(rf_ctx* ctx, rf_batch* b, const void* xf_segs, const char* cache_path) {
  if (!ctx || !b || !xf_segs) return RF_E_INVAL;
  WorkItem* trial = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  rf_status st = RF_OK;
  try {
    RF_HIP(hipSetDevice(ctx->device));
    const std::string sig = signature(b);
    // cached choice?
    if (cache_path) {
      std::ifstream in(cache_path);
      std::string line;
      while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string sg;
        rf_batch_tuning t{};
        if ((ls >> sg >> t.chunk[0] >> t.chunk[1] >> t.chunk[2] >> t.blocks[0] >> t.blocks[1] >> t.blocks[2] >>
             t.xcd_queues >> t.bucket_hi[0] >> t.bucket_hi[1]) &&
            sg == sig)
          return rf_batch_set_tuning(b, &t);
      }
    }
    // trial launches on the batch's data with the fused read-out into scratch, on
    // the buckets set at creation
    b->bucket_hi[0] = b->bucket_hi_tertiles[0];
    b->bucket_hi[1] = b->bucket_hi_tertiles[1];
    enqueue_reference(ctx, b, xf_segs);
    const int64_t np = int64_t(b->nseg) * b->ktotal;
    PeakOut po{};
    po.packed = b->packed;
    po.count = reinterpret_cast<unsigned long long*>(b->packed + np);
    po.trig = nullptr;
    po.cap = 0;
    po.thr2 = 1e30f;
    po.nk = b->ktotal;
    trial = dev_alloc<WorkItem>(b->items_cap, "batch: device allocation failed");
    RF_HIP(hipEventCreate(&e0));
    RF_HIP(hipEventCreate(&e1));
    // best of three launches of a trial list
    auto time_list = [&](const std::vector<WorkItem>& items, const QueueSpec& qs) {
      RF_HIP(hipMemcpy(trial, items.data(), sizeof(WorkItem) * items.size(), hipMemcpyHostToDevice));
      float best = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        fill_u64(ctx, b->packed, 0ull, np + 1);
        RF_HIP(hipEventRecord(e0, ctx->stream));
        queue_launch(ctx, b->nblocks, b->zs, b->n, b->nref, b->tiles, trial, qs, b->counter, b->b16, b->gflag,
                     b->colscale, b->slot_kernel, b->zinv, po);
        RF_HIP(hipEventRecord(e1, ctx->stream));
        RF_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        RF_HIP(hipEventElapsedTime(&ms, e0, e1));
        best = std::min(best, ms);
      }
      return best;
    };
    auto one_queue = [](size_t count) {
      QueueSpec qs{};
      qs.nq = 1;
      for (int i = 1; i <= kMaxQueues; ++i) qs.off[i] = int32_t(count);
      return qs;
    };
    const int32_t ntb = int32_t(b->n / kTimes);
    // Candidates come in order of less memory traffic first (longer window chunks,
    // more time blocks per item: fewer operand and window reloads and fewer item
    // starts; per-XCD queues: a tile's operand stays in one L2), and a later one
    // must be faster by more than 1 % to replace an earlier one: at a near tie the
    // launch keeps the setting that moves less data.
    auto better = [](float ms, float best) { return ms < 0.99f * best; };
    // (1) per bucket, chunk x blocks per item on the same sampled time blocks: about
    // four per workgroup slot, in groups of four consecutive blocks spread over the
    // bucket's (tile, segment, block) space
    const int cand_chunk[3] = {1024, 512, 256};
    const int cand_blocks[3] = {4, 2, 1};
    for (int bk = 0; bk < 3; ++bk) {
      struct Group { int32_t seg, tile, q0, len; };
      std::vector<Group> all;
      for (int32_t t : b->order) {
        if (bucket_of(b, b->htiles[t].t.ksteps) != bk) continue;
        for (int32_t sg = 0; sg < b->nseg; ++sg)
          for (int32_t q = 0; q < ntb; q += 4) all.push_back(Group{sg, t, q, std::min(4, ntb - q)});
      }
      if (all.empty()) continue;
      const size_t want = size_t(std::max(1, b->nblocks));
      const size_t stride = std::max<size_t>(1, all.size() / want);
      std::vector<Group> groups;
      for (size_t i = 0; i < all.size() && groups.size() < want; i += stride) groups.push_back(all[i]);
      float best = 1e30f;
      for (int c : cand_chunk)
        for (int nb : cand_blocks) {
          std::vector<WorkItem> items;
          for (const Group& g : groups)
            for (int32_t q = g.q0; q < g.q0 + g.len; q += nb)
              items.push_back(WorkItem{g.seg, g.tile, q, c, std::min(nb, g.q0 + g.len - q), 0});
          const float ms = time_list(items, one_queue(items.size()));
          if (better(ms, best)) {
            best = ms;
            b->chunk_for_bucket[bk] = c;
            b->blocks_for_bucket[bk] = nb;
          }
        }
    }
    // (2) one queue or one per XCD, with the chosen settings, on whole runs of time
    // blocks of up to eight tiles spread over the order (one per XCD queue), segment 0
    {
      std::vector<int32_t> pick;
      const size_t nt = b->order.size();
      for (int i = 0; i < kMaxQueues && size_t(i) < nt; ++i) pick.push_back(b->order[size_t(i) * nt / kMaxQueues]);
      const int32_t run = std::min<int32_t>(ntb, std::max(16, int32_t(16 * size_t(b->nblocks) / std::max<size_t>(pick.size(), 1))));
      float best = 1e30f;
      for (int x = 1; x >= 0; --x) {
        std::vector<WorkItem> items;
        QueueSpec qs{};
        build_items(b, pick, x ? kMaxQueues : 1, 1, run, items, qs);
        const float ms = time_list(items, qs);
        if (better(ms, best)) {
          best = ms;
          b->xcd_queues = x;
        }
      }
    }
    upload_items(b);
    if (cache_path) {
      std::ofstream outf(cache_path, std::ios::app);
      outf << sig;
      for (int i = 0; i < 3; ++i) outf << " " << b->chunk_for_bucket[i];
      for (int i = 0; i < 3; ++i) outf << " " << b->blocks_for_bucket[i];
      outf << " " << b->xcd_queues << " " << b->bucket_hi[0] << " " << b->bucket_hi[1] << "\n";
    }
  } catch (const Error& e) {
    ctx->last_error = e.msg;
    st = e.code;
  } catch (...) {
    ctx->last_error = "rf_batch_autotune: unexpected exception";
    st = RF_E_HIP;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (trial) {
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(trial);
  }
  return st;
}

rf_status rf_batch_run(rf_ctx* ctx, rf_batch* b, const void* xf_segs, float thr, rf_peak* peaks,
                       rf_trigger* trig, int64_t cap, int64_t* ntrig) {
  if (!ctx || !b) return RF_E_INVAL;
  try {
    RF_HIP(hipSetDevice(ctx->device));
    RF_CHECK(xf_segs && peaks && ntrig, "rf_batch_run: null pointer");
    RF_CHECK(cap >= 0 && (cap == 0 || trig), "rf_batch_run: bad trigger buffer");
    RF_CHECK(std::isfinite(thr) && thr >= 0, "rf_batch_run: bad threshold");
    RF_CHECK(ctx->stream != nullptr, "rf_batch_run: needs a non-null stream (graph capture)");
    if (!b->exec || !b->exec_ref || b->g_cap != cap || b->g_thr != thr) {
      drop_graphs(b);
      if (cap > b->trig_cap) {
        RF_HIP(hipStreamSynchronize(ctx->stream));
        if (b->trig_own) (void)hipFree(b->trig_own);
        b->trig_own = nullptr;
        b->trig_cap = 0;
        b->trig_own = dev_alloc<rf_trigger>(size_t(cap), "batch: device allocation failed");
        b->trig_cap = cap;
      }
      b->exec_ref = capture(ctx, [&] { enqueue_reference(ctx, b, b->xf_own); });
      b->exec = capture(ctx, [&] { enqueue_recon(ctx, b, thr, b->peaks_own, cap > 0 ? b->trig_own : nullptr, cap); });
      b->g_cap = cap;
      b->g_thr = thr;
      ++b->captures;
    }
    const int64_t np = int64_t(b->nseg) * b->ktotal;
    RF_HIP(hipMemcpyAsync(b->xf_own, xf_segs, sizeof(double2) * size_t(b->nseg) * size_t(b->n / 2 + 1),
                          hipMemcpyDeviceToDevice, ctx->stream));
    RF_HIP(hipGraphLaunch(b->exec_ref, ctx->stream));
    RF_HIP(hipEventRecord(b->ev0, ctx->stream));
    RF_HIP(hipGraphLaunch(b->exec, ctx->stream));
    RF_HIP(hipEventRecord(b->ev1, ctx->stream));
    ++b->replays;
    unsigned long long cnt = 0;
    RF_HIP(hipMemcpyAsync(&cnt, b->packed + np, sizeof(cnt), hipMemcpyDeviceToHost, ctx->stream));
    RF_HIP(hipStreamSynchronize(ctx->stream));
    RF_HIP(hipMemcpyAsync(peaks, b->peaks_own, sizeof(rf_peak) * size_t(np), hipMemcpyDeviceToDevice, ctx->stream));
    const int64_t nrec = std::min<int64_t>(int64_t(cnt), cap);
    if (nrec > 0)
      RF_HIP(hipMemcpyAsync(trig, b->trig_own, sizeof(rf_trigger) * size_t(nrec), hipMemcpyDeviceToDevice,
                            ctx->stream));
    RF_HIP(hipStreamSynchronize(ctx->stream));
    RF_HIP(hipEventElapsedTime(&b->last_recon_ms, b->ev0, b->ev1));
    *ntrig = int64_t(cnt);
    if (int64_t(cnt) > cap) throw Error{RF_E_OVERFLOW, "rf_batch_run: trigger buffer overflow"};
  } catch (const Error& e) {
    ctx->last_error = e.msg;
    return e.code;
  } catch (...) {
    ctx->last_error = "rf_batch_run: unexpected exception";
    return RF_E_HIP;
  }
  return RF_OK;
}

rf_status rf_batch_graph_stats(const rf_batch* b, int64_t* captures, int64_t* replays, float* recon_ms) {
  if (!b) return RF_E_INVAL;
  if (captures) *captures = b->captures;
  if (replays) *replays = b->replays;
  if (recon_ms) *recon_ms = b->last_recon_ms;
  return RF_OK;
}

rf_status rf_batch_free(rf_batch* b) {
  if (!b) return RF_E_INVAL;
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  free_batch(b);
  return RF_OK;
}

}  // extern "C"
