// Batched reconstruction: several data segments x several reference groups,
// each group with its own (uneven) set of truncated kernels.  Per call, one
// device sequence -- reference matched filters of every (segment, reference),
// split of every reference series, one persistent split-FP16 reconstruction
// launch over all (segment, tile, time block) work items with the fused
// peak/threshold read-out, peak finalisation -- captured once in a hipGraph
// and replayed.  The graph reads and writes only buffers the batch owns (the
// caller's data are copied in before a replay, the read-out copied out after
// it), so a replay does not depend on the caller's pointers.  Work items are
// ordered longest tile first so the queue ends on short items; the chunk size
// of each item comes from an autotuner that times the candidate chunk sizes
// per kernel-length bucket on the device.
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
  // chunk size per kernel-length bucket (taps)
  int chunk_for_bucket[3] = {512, 512, 512};
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

int bucket_of(int64_t ksteps) { return ksteps <= 64 ? 0 : (ksteps <= 512 ? 1 : 2); }

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

void upload_items(rf_batch* b) {
  for (auto& it : b->hitems) it.chunk = b->chunk_for_bucket[bucket_of(b->htiles[it.tile].t.ksteps)];
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
  queue_launch(ctx, b->nblocks, b->zs, b->n, b->nref, b->tiles, b->items, int(b->hitems.size()),
               b->counter, b->b16, b->gflag, b->colscale, b->slot_kernel, b->zinv, po);
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
  int64_t counts[3] = {0, 0, 0};
  for (const auto& t : b->htiles) counts[bucket_of(t.t.ksteps)] += t.t.ksteps;
  std::ostringstream os;
  os << "arch=" << arch << ";n=" << b->n << ";seg=" << b->nseg << ";ref=" << b->nref
     << ";k=" << b->ktotal << ";steps=" << counts[0] << "," << counts[1] << "," << counts[2];
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
    // work list: every (segment, tile, time block), longest tiles first
    std::vector<int32_t> order(b->htiles.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = int32_t(i);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return b->htiles[a].t.ksteps > b->htiles[c].t.ksteps; });
    const int32_t ntb = int32_t(b->n / kTimes);
    for (int32_t t : order) {
      if (b->htiles[t].t.ksteps == 0) continue;
      for (int32_t s = 0; s < nseg; ++s)
        for (int32_t q = 0; q < ntb; ++q) b->hitems.push_back(WorkItem{s, t, q, int32_t(kChunk)});
    }
    RF_CHECK(b->hitems.size() < size_t(INT32_MAX), "rf_batch_create: too many work items");
    b->tiles = dev_alloc<BatchTile>(b->htiles.size(), "batch: device allocation failed");
    RF_HIP(hipMemcpy(b->tiles, b->htiles.data(), sizeof(BatchTile) * b->htiles.size(), hipMemcpyHostToDevice));
    b->items = dev_alloc<WorkItem>(b->hitems.size(), "batch: device allocation failed");
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
    b->counter = dev_alloc<uint32_t>(1, "batch: device allocation failed");
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
  for (int i = 0; i < 3; ++i) {
    const int c = chunk_per_bucket[i];
    if (c != 256 && c != 512 && c != 1024) return RF_E_INVAL;
  }
  try {
    RF_HIP(hipSetDevice(b->device));
    for (int i = 0; i < 3; ++i) b->chunk_for_bucket[i] = chunk_per_bucket[i];
    upload_items(b);
  } catch (const Error& e) {
    return e.code;
  }
  return RF_OK;
}

rf_status rf_batch_autotune(rf_ctx* ctx, rf_batch* b, const void* xf_segs, const char* cache_path) {
  if (!ctx || !b || !xf_segs) return RF_E_INVAL;
  try {
    RF_HIP(hipSetDevice(ctx->device));
    const std::string sig = signature(b);
    // cached choice?
    if (cache_path) {
      std::ifstream in(cache_path);
      std::string line;
      while (std::getline(in, line)) {
        std::istringstream ls(line);
        std::string s;
        int c0, c1, c2;
        if ((ls >> s >> c0 >> c1 >> c2) && s == sig) {
          const int32_t cs[3] = {c0, c1, c2};
          return rf_batch_set_chunks(b, cs);
        }
      }
    }
    // time every candidate on each bucket's own items (fused read-out into scratch)
    enqueue_reference(ctx, b, xf_segs);
    const int64_t np = int64_t(b->nseg) * b->ktotal;
    PeakOut po{};
    po.packed = b->packed;
    po.count = reinterpret_cast<unsigned long long*>(b->packed + np);
    po.trig = nullptr;
    po.cap = 0;
    po.thr2 = 1e30f;
    po.nk = b->ktotal;
    WorkItem* scratch = dev_alloc<WorkItem>(b->hitems.size(), "batch: device allocation failed");
    hipEvent_t e0, e1;
    RF_HIP(hipEventCreate(&e0));
    RF_HIP(hipEventCreate(&e1));
    const int cand[3] = {256, 512, 1024};
    for (int bk = 0; bk < 3; ++bk) {
      std::vector<WorkItem> sub;
      for (const auto& it : b->hitems)
        if (bucket_of(b->htiles[it.tile].t.ksteps) == bk) sub.push_back(it);
      if (sub.empty()) continue;
      // at most ~4 items per workgroup slot keeps the tuning runs short
      const size_t cap_items = size_t(b->nblocks) * 4;
      if (sub.size() > cap_items) sub.resize(cap_items);
      float best = 1e30f;
      for (int c : cand) {
        for (auto& it : sub) it.chunk = c;
        RF_HIP(hipMemcpy(scratch, sub.data(), sizeof(WorkItem) * sub.size(), hipMemcpyHostToDevice));
        float ms = 0.f;
        for (int rep = 0; rep < 2; ++rep) {
          fill_u64(ctx, b->packed, 0ull, np + 1);
          RF_HIP(hipEventRecord(e0, ctx->stream));
          queue_launch(ctx, b->nblocks, b->zs, b->n, b->nref, b->tiles, scratch, int(sub.size()),
                       b->counter, b->b16, b->gflag, b->colscale, b->slot_kernel, b->zinv, po);
          RF_HIP(hipEventRecord(e1, ctx->stream));
          RF_HIP(hipEventSynchronize(e1));
          RF_HIP(hipEventElapsedTime(&ms, e0, e1));
        }
        if (ms < best) {
          best = ms;
          b->chunk_for_bucket[bk] = c;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(scratch);
    upload_items(b);
    if (cache_path) {
      std::ofstream outf(cache_path, std::ios::app);
      outf << sig << " " << b->chunk_for_bucket[0] << " " << b->chunk_for_bucket[1] << " "
           << b->chunk_for_bucket[2] << "\n";
    }
  } catch (const Error& e) {
    ctx->last_error = e.msg;
    return e.code;
  } catch (...) {
    ctx->last_error = "rf_batch_autotune: unexpected exception";
    return RF_E_HIP;
  }
  return RF_OK;
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
