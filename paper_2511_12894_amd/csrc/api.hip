// C-ABI entry points of librf: argument checks, workspace, scheduling of the
// kernels in fft.hip, spectra.hip and recon.hip.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>

#include "recon.h"

// Scratch of snr_reconstruct_noalloc, for callers that cannot allocate: the
// FP16 split planes of the reference series (4 x n halves) with the split's
// maximum bits and inverse scale, then the peak keys and trigger count of the
// fused read-out.  One copy per device, held until the process ends; every
// call on a device shares it (calls that overlap on one device race).
namespace rf {
constexpr int64_t kNoAllocMaxN = int64_t(1) << 21;
constexpr int32_t kNoAllocMaxKernels = 4096;
constexpr size_t kNoAllocSplitBytes = sizeof(__half) * 4 * size_t(kNoAllocMaxN) + 256;
constexpr size_t kNoAllocBytes = kNoAllocSplitBytes + sizeof(uint64_t) * (size_t(kNoAllocMaxKernels) + 1);
constexpr int kMaxDevices = 64;
}  // namespace rf
static __device__ __align__(256) unsigned char scratch[rf::kNoAllocBytes];

namespace rf {

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

void* DevBuf::ensure(size_t n) {
  if (n <= bytes && p) return p;
  release();
  if (hipMalloc(&p, n) != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();
    throw Error{RF_E_NOMEM, "device allocation of " + std::to_string(n) + " bytes failed"};
  }
  bytes = n;
  return p;
}

void validate_grid(const rf_grid* g) {
  RF_CHECK(g != nullptr, "grid is NULL");
  RF_CHECK(is_pow2(g->n) && g->n >= 256 && g->n <= (int64_t(1) << 24),
           "grid.n must be a power of two in [2^8, 2^24]");
  RF_CHECK(std::isfinite(g->fs) && g->fs > 0, "grid.fs must be positive");
  RF_CHECK(g->df_high > 0 && g->df_low_max > 0, "taper widths must be positive");
  RF_CHECK(g->f_low - g->df_low_max > 0, "need f_low - df_low_max > 0");
  RF_CHECK(g->f_high > g->f_low, "need f_high > f_low");
  RF_CHECK(g->f_high + g->df_high <= 0.5 * g->fs * (1 + 1e-15), "need f_high + df_high <= fs / 2");
}

namespace {

void validate_tmpl(const rf_tmpl& t) {
  RF_CHECK(std::isfinite(t.m1) && std::isfinite(t.m2) && t.m1 > 0 && t.m2 > 0,
           "template masses must be positive");
}

// Small per-call tables: staged in a host copy owned by the context (so the
// source outlives an asynchronous copy), then copied on the context stream.
template <typename T>
T* upload(rf_ctx* ctx, int slot, const T* host, size_t count) {
  T* d = static_cast<T*>(ctx->ws[slot].ensure(sizeof(T) * std::max<size_t>(count, 1)));
  std::vector<char>& stage = ctx->host_stage[slot];
  stage.assign(reinterpret_cast<const char*>(host), reinterpret_cast<const char*>(host + count));
  RF_HIP(hipMemcpyAsync(d, stage.data(), sizeof(T) * count, hipMemcpyHostToDevice, ctx->stream));
  return d;
}

void sync(rf_ctx* ctx) { RF_HIP(hipStreamSynchronize(ctx->stream)); }

// Device address of `scratch` on each device (the host-side name is not one):
// looked up once per device, with that device current, by rf_ctx_create.
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_lookup(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess) g_scratch_ptr[device] = p;
  return e;
}

char* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return static_cast<char*>(g_scratch_ptr[device]);
}

// Work buffers of one reconstruction: split planes (+ max bits, inverse scale)
// and the fused read-out's peak keys (+ trigger count).
struct ReconScratch {
  char* split;
  uint64_t* packed;
};

double pow2_scale_for(double maxabs) {
  if (!(maxabs > 0)) return 1.0;
  int ex = 0;
  std::frexp(maxabs, &ex);
  return std::ldexp(1.0, 14 - ex);   // maxabs * s in [2^13, 2^14)
}

void free_kernels(rf_kernels* k) {
  if (!k) return;
  for (void* p : {(void*)k->taps64, (void*)k->tiles_dev, (void*)k->b32, (void*)k->b16,
                  (void*)k->colscale32, (void*)k->colscale16, (void*)k->slot_kernel, (void*)k->gflag})
    if (p) (void)hipFree(p);
  delete k;
}

}  // namespace

void free_kernel_set(rf_kernels* k) { free_kernels(k); }

void copy_sync(rf_ctx* ctx, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  RF_HIP(hipMemcpyAsync(dst, src, bytes, kind, ctx->stream));
  RF_HIP(hipStreamSynchronize(ctx->stream));
}

// Tiles, packed operands and device copies of a kernel set whose per-kernel
// fields (m_lo, len, off, norm_ratio, kscale) and FP64 taps (host, concatenated
// at off) are filled in.  Synchronises.
void finalize_kernel_set(rf_ctx* ctx, rf_kernels* K, const std::vector<double>& taps_host) {
  const int32_t nk = K->nk;
  K->total_taps = int64_t(taps_host.size());
  K->taps64 = dev_alloc<double>(size_t(K->total_taps));
  if (K->total_taps)
    RF_HIP(hipMemcpy(K->taps64, taps_host.data(), sizeof(double) * taps_host.size(), hipMemcpyHostToDevice));

  // tiles: kernels sorted by first tap, 32 per tile, union support per tile; a
  // last tile of at most 16 kernels is paired (each kernel in two columns, the
  // second 32 taps later), so it costs half a tile's matrix products
  std::vector<int32_t> order(nk);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return K->m_lo[a] < K->m_lo[b]; });
  const int ntiles = (nk + kTileKernels - 1) / kTileKernels;
  std::vector<int32_t> slot(size_t(ntiles) * kTileKernels, -1);
  std::vector<float> cs32(slot.size(), 0.f), cs16(slot.size(), 0.f);
  int64_t b32_total = 0, b16_total = 0, gflag_total = 0;
  K->tiles.clear();
  K->max_ksteps = 0;
  for (int t = 0; t < ntiles; ++t) {
    TileDev T{};
    T.first = t * kTileKernels;
    T.count = std::min(kTileKernels, nk - t * kTileKernels);
    int64_t lo = INT64_MAX, hi = INT64_MIN;
    for (int i = 0; i < T.count; ++i) {
      const int k = order[T.first + i];
      slot[T.first + i] = k;
      cs32[T.first + i] = float(K->norm_ratio[k]);
      cs16[T.first + i] = float(K->norm_ratio[k] / K->kscale[k]);
      if (K->len[k] > 0) {
        lo = std::min(lo, K->m_lo[k]);
        hi = std::max(hi, K->m_lo[k] + K->len[k]);
      }
    }
    if (lo == INT64_MAX) {
      T.m0 = 0;
      T.ksteps = 0;
    } else {
      T.m0 = lo & ~int64_t(3);            // a multiple of 4: the window refill moves 4-sample blocks
      auto steps_for = [&](int64_t end) { return ((end - T.m0 + 16 * kStepAlign - 1) / (16 * kStepAlign)) * kStepAlign; };
      T.ksteps = steps_for(hi);
      if (T.count <= kPairKernels && steps_for(hi + kPairShift) * 16 <= K->n_build) {
        T.pair = 1;
        T.ksteps = steps_for(hi + kPairShift);
      }
    }
    T.b32_off = b32_total;
    T.b16_off = b16_total;
    T.gflag_off = gflag_total;
    b32_total += T.ksteps * kB32PerStep;
    b16_total += T.ksteps * kB16PerStep;
    gflag_total += (T.ksteps + 15) / 16;
    K->max_ksteps = std::max(K->max_ksteps, T.ksteps);
    K->tiles.push_back(T);
  }
  K->tiles_dev = dev_alloc<TileDev>(K->tiles.size());
  K->slot_kernel = dev_alloc<int32_t>(slot.size());
  K->colscale32 = dev_alloc<float>(slot.size());
  K->colscale16 = dev_alloc<float>(slot.size());
  K->b32 = dev_alloc<float>(size_t(b32_total + int64_t(kOperandPadSteps) * kB32PerStep));
  K->b16 = dev_alloc<__half>(size_t(b16_total + int64_t(kOperandPadSteps) * kB16PerStep));
  fill_u32(ctx, reinterpret_cast<uint32_t*>(K->b32 + b32_total), 0u, int64_t(kOperandPadSteps) * kB32PerStep);
  fill_u32(ctx, reinterpret_cast<uint32_t*>(K->b16 + b16_total), 0u, int64_t(kOperandPadSteps) * kB16PerStep / 2);
  K->gflag_total = gflag_total;
  K->gflag = dev_alloc<uint32_t>(size_t(std::max<int64_t>(gflag_total, 1)));
  fill_u32(ctx, K->gflag, 0u, std::max<int64_t>(gflag_total, 1));
  RF_HIP(hipMemcpy(K->tiles_dev, K->tiles.data(), sizeof(TileDev) * K->tiles.size(), hipMemcpyHostToDevice));
  RF_HIP(hipMemcpy(K->slot_kernel, slot.data(), sizeof(int32_t) * slot.size(), hipMemcpyHostToDevice));
  RF_HIP(hipMemcpy(K->colscale32, cs32.data(), sizeof(float) * cs32.size(), hipMemcpyHostToDevice));
  RF_HIP(hipMemcpy(K->colscale16, cs16.data(), sizeof(float) * cs16.size(), hipMemcpyHostToDevice));
  if (K->max_ksteps > 0) {
    int64_t* off_d = dev_alloc<int64_t>(size_t(nk) * 2);
    int64_t* mlo_d = off_d + nk;
    int32_t* len_d = dev_alloc<int32_t>(size_t(nk));
    double* ks_d = dev_alloc<double>(size_t(nk));
    RF_HIP(hipMemcpy(off_d, K->off.data(), sizeof(int64_t) * nk, hipMemcpyHostToDevice));
    RF_HIP(hipMemcpy(mlo_d, K->m_lo.data(), sizeof(int64_t) * nk, hipMemcpyHostToDevice));
    RF_HIP(hipMemcpy(len_d, K->len.data(), sizeof(int32_t) * nk, hipMemcpyHostToDevice));
    RF_HIP(hipMemcpy(ks_d, K->kscale.data(), sizeof(double) * nk, hipMemcpyHostToDevice));
    pack_launch(ctx, K, off_d, mlo_d, len_d, ks_d, K->tiles_dev, ntiles, K->max_ksteps);
    sync(ctx);
    (void)hipFree(off_d);
    (void)hipFree(len_d);
    (void)hipFree(ks_d);
  }
}

namespace {

// FNV-1a, 64 bit, over a byte range, continued from h
uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= 1099511628211ull;
  }
  return h;
}
constexpr uint64_t kFnvBasis = 14695981039346656037ull;
constexpr char kSetTag[8] = {'R', 'F', 'K', 'S', 'E', 'T', '0', '1'};

// Sequential writer / reader of the kernel-set file, hashing the bytes after the tag.
struct SetWriter {
  std::FILE* f;
  uint64_t h = kFnvBasis;
  void put(const void* p, size_t n) {
    RF_CHECK(n == 0 || std::fwrite(p, 1, n, f) == n, "rf_kernels_save: write failed");
    h = fnv1a(h, p, n);
  }
};
struct SetReader {
  std::FILE* f;
  uint64_t h = kFnvBasis;
  void get(void* p, size_t n) {
    RF_CHECK(n == 0 || std::fread(p, 1, n, f) == n, "rf_kernels_load: file shorter than its header states");
    h = fnv1a(h, p, n);
  }
};
struct FileCloser {
  std::FILE* f;
  ~FileCloser() {
    if (f) std::fclose(f);
  }
};

}  // namespace

}  // namespace rf

using namespace rf;

extern "C" {

rf_status rf_ctx_create(int device, void* hip_stream, rf_ctx** out) {
  if (!out) return RF_E_INVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return RF_E_INVAL;
  rf_ctx* c = new (std::nothrow) rf_ctx();
  if (!c) return RF_E_NOMEM;
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (device >= kMaxDevices || hipSetDevice(device) != hipSuccess || scratch_lookup(device) != hipSuccess) {
    delete c;
    return RF_E_HIP;
  }
  *out = c;
  return RF_OK;
}

rf_status rf_ctx_destroy(rf_ctx* ctx) {
  if (!ctx) return RF_E_INVAL;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& b : ctx->ws) b.release();
  delete ctx;
  return RF_OK;
}

const char* rf_last_error(const rf_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

rf_status mf_ref_snr(rf_ctx* ctx, const rf_grid* grid, const void* xf, const double* psd,
                     const rf_tmpl* tmpl, int32_t nt, void* z, double* sigma) {
  if (!ctx) return RF_E_INVAL;
  return guarded(ctx, [&] {
    validate_grid(grid);
    RF_CHECK(xf && psd && tmpl && z, "mf_ref_snr: null pointer");
    RF_CHECK(nt >= 1, "mf_ref_snr: nt must be >= 1");
    const int64_t n = grid->n;
    std::vector<Tf2Coef> coef(nt);
    for (int i = 0; i < nt; ++i) {
      validate_tmpl(tmpl[i]);
      coef[i] = tf2_coef(tmpl[i]);
    }
    Tf2Coef* coef_dev = upload(ctx, WS_COEF, coef.data(), coef.size());
    double* moment = static_cast<double*>(ctx->ws[WS_SCALAR].ensure(64));
    band_moment(ctx, grid, psd, moment);
    // conditioned data once, then the templates in batches (FFT scratch up to 8 GiB); each
    // template's spectrum is formed inside the first transform pass and never stored
    int64_t jlo, jhi;
    band_limits(grid, &jlo, &jhi);
    float2* q = static_cast<float2*>(ctx->ws[WS_Y].ensure(sizeof(float2) * size_t(jhi - jlo + 1)));
    condition_data(ctx, grid, static_cast<const double2*>(xf), psd, q);
    // at most 2^30 / n templates a batch, split evenly (no small last batch)
    const int cap = int(std::max<int64_t>(1, std::min<int64_t>(nt, (int64_t(1) << 30) / n)));
    const int nbatch = (nt + cap - 1) / cap;
    const int per = (nt + nbatch - 1) / nbatch;
    float2* zo = static_cast<float2*>(z);
    for (int t0 = 0; t0 < nt; t0 += per) {
      const int cnt = std::min(per, nt - t0);
      fft_inverse_tmpl_f32(ctx, grid, q, coef_dev + t0, cnt, moment, zo + int64_t(t0) * n, cnt);
    }
    if (sigma) {
      double mom = 0;
      RF_HIP(hipMemcpyAsync(&mom, moment, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
      sync(ctx);
      const double df = grid->fs / double(n);
      for (int i = 0; i < nt; ++i) sigma[i] = coef[i].amp * std::sqrt(4.0 * df * mom);
    }
  });
}

rf_status snr_reconstruct_factored_batch(rf_ctx* ctx, const rf_grid* grid, const void* xf_segs, int32_t nseg,
                                         const double* psd, int32_t nset, const rf_factored* const* sets,
                                         const rf_tmpl* refs, rf_prec prec, const rf_peak_args* out) {
  if (!ctx) return RF_E_INVAL;
  return guarded(ctx, [&] {
    validate_grid(grid);
    RF_CHECK(xf_segs && psd && sets && refs && out, "snr_reconstruct_factored_batch: null pointer");
    RF_CHECK(nseg >= 1 && nset >= 1, "snr_reconstruct_factored_batch: need nseg >= 1 and nset >= 1");
    RF_CHECK(prec == RF_PREC_FP32 || prec == RF_PREC_SPLIT_FP16, "snr_reconstruct_factored_batch: bad precision");
    RF_CHECK(out->peaks && out->ntrig && out->cap >= 0 && (out->cap == 0 || out->trig),
             "snr_reconstruct_factored_batch: bad read-out arguments");
    RF_CHECK(std::isfinite(out->thr) && out->thr >= 0, "snr_reconstruct_factored_batch: bad threshold");
    const int64_t n = grid->n;
    std::vector<int32_t> kbase(static_cast<size_t>(nset) + 1, 0);
    std::vector<Tf2Coef> coef(static_cast<size_t>(nset));
    for (int r = 0; r < nset; ++r) {
      RF_CHECK(sets[r] != nullptr, "snr_reconstruct_factored_batch: null set");
      const FactoredView v = factored_view(sets[r]);
      RF_CHECK(v.device == ctx->device, "snr_reconstruct_factored_batch: set on another device");
      RF_CHECK(v.n == n, "snr_reconstruct_factored_batch: set built for another series length");
      RF_CHECK(!(v.large && prec != RF_PREC_SPLIT_FP16),
               "snr_reconstruct_factored_batch: large sets mix in split FP16 only");
      RF_CHECK(int64_t(kbase[r]) + v.nk <= INT32_MAX, "snr_reconstruct_factored_batch: too many kernels");
      kbase[r + 1] = kbase[r] + v.nk;
      validate_tmpl(refs[r]);
      coef[r] = tf2_coef(refs[r]);
    }
    const int64_t ktot = kbase[nset];
    RF_CHECK(int64_t(nseg) * ktot < (int64_t(1) << 40), "snr_reconstruct_factored_batch: too many series");
    Tf2Coef* coef_dev = upload(ctx, WS_COEF, coef.data(), coef.size());
    double* moment = static_cast<double*>(ctx->ws[WS_SCALAR].ensure(64));
    band_moment(ctx, grid, psd, moment);
    int64_t jlo, jhi;
    band_limits(grid, &jlo, &jhi);
    float2* q = static_cast<float2*>(ctx->ws[WS_Y].ensure(sizeof(float2) * size_t(jhi - jlo + 1)));
    float2* zref = static_cast<float2*>(ctx->ws[WS_ZREF].ensure(sizeof(float2) * size_t(n)));
    const int64_t np = int64_t(nseg) * ktot;
    uint64_t* packed = static_cast<uint64_t*>(ctx->ws[WS_PEAK].ensure(sizeof(uint64_t) * size_t(np + 1)));
    fill_u64(ctx, packed, 0ull, np + 1);
    PeakOut po{};
    po.packed = packed;
    po.count = reinterpret_cast<unsigned long long*>(packed + np);
    po.trig = out->trig;
    po.cap = out->cap;
    po.thr2 = out->thr * out->thr;
    po.nk = int32_t(ktot);
    const double2* xs = static_cast<const double2*>(xf_segs);
    for (int32_t sg = 0; sg < nseg; ++sg) {
      condition_data(ctx, grid, xs + int64_t(sg) * (n / 2 + 1), psd, q);
      for (int r = 0; r < nset; ++r) {
        fft_inverse_tmpl_f32(ctx, grid, q, coef_dev + r, 1, moment, zref, 1);
        po.seg = sg;
        po.tmpl0 = kbase[r];
        factored_enqueue(ctx, sets[r], zref, n, prec, nullptr, &po);
      }
    }
    trig_finish(ctx, out->trig, po.count, out->cap);
    peaks_finalize(ctx, packed, np, out->peaks);
    unsigned long long c = 0;
    RF_HIP(hipMemcpyAsync(&c, po.count, sizeof(c), hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    *out->ntrig = int64_t(c);
    if (int64_t(c) > out->cap) throw Error{RF_E_OVERFLOW, "snr_reconstruct_factored_batch: trigger buffer overflow"};
  });
}

rf_status mf_snr_peaks(rf_ctx* ctx, const rf_grid* grid, const void* xf, const double* psd,
                       const rf_tmpl* tmpl, int32_t nt, const rf_peak_args* out) {
  if (!ctx) return RF_E_INVAL;
  return guarded(ctx, [&] {
    validate_grid(grid);
    RF_CHECK(xf && psd && tmpl && out, "mf_snr_peaks: null pointer");
    RF_CHECK(nt >= 1, "mf_snr_peaks: nt must be >= 1");
    RF_CHECK(out->peaks && out->ntrig && out->cap >= 0 && (out->cap == 0 || out->trig),
             "mf_snr_peaks: bad read-out arguments");
    RF_CHECK(std::isfinite(out->thr) && out->thr >= 0, "mf_snr_peaks: bad threshold");
    const int64_t n = grid->n;
    std::vector<Tf2Coef> coef(nt);
    for (int i = 0; i < nt; ++i) {
      validate_tmpl(tmpl[i]);
      coef[i] = tf2_coef(tmpl[i]);
    }
    Tf2Coef* coef_dev = upload(ctx, WS_COEF, coef.data(), coef.size());
    double* moment = static_cast<double*>(ctx->ws[WS_SCALAR].ensure(64));
    band_moment(ctx, grid, psd, moment);
    int64_t jlo, jhi;
    band_limits(grid, &jlo, &jhi);
    float2* q = static_cast<float2*>(ctx->ws[WS_Y].ensure(sizeof(float2) * size_t(jhi - jlo + 1)));
    condition_data(ctx, grid, static_cast<const double2*>(xf), psd, q);
    uint64_t* packed = static_cast<uint64_t*>(ctx->ws[WS_PEAK].ensure(sizeof(uint64_t) * (nt + 1)));
    fill_u64(ctx, packed, 0ull, nt + 1);
    PeakOut po{};
    po.packed = packed;
    po.count = reinterpret_cast<unsigned long long*>(packed + nt);
    po.trig = out->trig;
    po.cap = out->cap;
    po.thr2 = out->thr * out->thr;
    po.seg = 0;
    po.nk = nt;
    // templates in batches (two transform scratch buffers of up to 8 GiB each)
    // at most 2^30 / n templates a batch, split evenly (no small last batch)
    const int cap = int(std::max<int64_t>(1, std::min<int64_t>(nt, (int64_t(1) << 30) / n)));
    const int nbatch = (nt + cap - 1) / cap;
    const int per = (nt + nbatch - 1) / nbatch;
    for (int t0 = 0; t0 < nt; t0 += per) {
      const int cnt = std::min(per, nt - t0);
      po.tmpl0 = t0;
      fft_inverse_tmpl_peaks_f32(ctx, grid, q, coef_dev + t0, cnt, moment, cnt, po);
    }
    peaks_finalize(ctx, packed, nt, out->peaks);
    trig_finish(ctx, out->trig, po.count, out->cap);   // the passes wrote raw (re, im)
    unsigned long long c = 0;
    RF_HIP(hipMemcpyAsync(&c, po.count, sizeof(c), hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    *out->ntrig = int64_t(c);
    if (int64_t(c) > out->cap) throw Error{RF_E_OVERFLOW, "mf_snr_peaks: trigger buffer overflow"};
  });
}

rf_status ratio_kernel_build(rf_ctx* ctx, const rf_grid* grid, const double* psd, rf_tmpl ref,
                             const rf_tmpl* nbr, int32_t nk, double thr, rf_thr_unit unit,
                             int64_t n_build, rf_kernels** out) {
  if (!ctx) return RF_E_INVAL;
  rf_kernels* K = nullptr;
  rf_status st = guarded(ctx, [&] {
    validate_grid(grid);
    RF_CHECK(psd && nbr && out, "ratio_kernel_build: null pointer");
    RF_CHECK(nk >= 1, "ratio_kernel_build: nk must be >= 1");
    RF_CHECK(std::isfinite(thr) && thr > 0, "ratio_kernel_build: threshold must be positive");
    RF_CHECK(unit == RF_THR_PER_SECOND || unit == RF_THR_PER_TAP, "ratio_kernel_build: bad unit");
    const int64_t nb = n_build == 0 ? grid->n : n_build;
    RF_CHECK(is_pow2(nb) && nb >= 256 && nb <= grid->n, "ratio_kernel_build: n_build must be a power of two in [2^8, n]");
    validate_tmpl(ref);
    *out = nullptr;
    K = new rf_kernels();
    K->device = ctx->device;
    K->nk = nk;
    K->n_build = nb;
    K->fs = grid->fs;

    // host scalars: taper widths (section II.C) and amplitude ratios
    const Tf2Coef cref = tf2_coef(ref);
    const double tpr = tf2_dtdf(cref, grid->f_low);
    std::vector<Tf2Coef> ct(nk);
    std::vector<RatioParam> par(nk);
    K->df_low.resize(nk);
    for (int k = 0; k < nk; ++k) {
      validate_tmpl(nbr[k]);
      ct[k] = tf2_coef(nbr[k]);
      const double d = std::fabs(tf2_dtdf(ct[k], grid->f_low) - tpr);
      double dfl = d > 0 ? 1.0 / std::sqrt(d) : grid->df_low_max;
      if (dfl > grid->df_low_max) dfl = grid->df_low_max;
      K->df_low[k] = dfl;
      par[k].amp_ratio = ct[k].amp / cref.amp;
      par[k].df_low = dfl;
    }
    // template norms through the band moment (section II.A normalisation)
    double* moment = static_cast<double*>(ctx->ws[WS_SCALAR].ensure(64));
    band_moment(ctx, grid, psd, moment);
    double mom = 0;
    RF_HIP(hipMemcpyAsync(&mom, moment, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    const double df = grid->fs / double(grid->n);
    RF_CHECK(std::isfinite(mom) && mom > 0, "ratio_kernel_build: PSD band moment is not positive");
    const double nref = cref.amp * std::sqrt(4.0 * df * mom);
    K->norm_ratio.resize(nk);
    for (int k = 0; k < nk; ++k) K->norm_ratio[k] = nref / (ct[k].amp * std::sqrt(4.0 * df * mom));

    const double thr_tap = unit == RF_THR_PER_SECOND ? thr / grid->fs : thr;
    Tf2Coef* ref_dev = upload(ctx, WS_COEF, &cref, 1);
    // neighbours in batches bounded by ~512 MiB of FP64 spectra
    const int per = int(std::max<int64_t>(1, std::min<int64_t>(nk, (int64_t(1) << 25) / nb)));
    double2* spec = static_cast<double2*>(ctx->ws[WS_BUILD].ensure(sizeof(double2) * size_t(nb) * per));
    double2* wout = static_cast<double2*>(ctx->ws[WS_Y].ensure(sizeof(double2) * size_t(nb) * per));
    char* scan = static_cast<char*>(ctx->ws[WS_SCAN].ensure(size_t(per) * 64 + 4096));
    int32_t* lo_d = reinterpret_cast<int32_t*>(scan);
    int32_t* hi_d = lo_d + per;
    uint32_t* mx_d = reinterpret_cast<uint32_t*>(hi_d + per);
    Tf2Coef* tgt_dev = static_cast<Tf2Coef*>(ctx->ws[WS_TGT].ensure(sizeof(Tf2Coef) * per + sizeof(RatioParam) * per));
    RatioParam* par_dev = reinterpret_cast<RatioParam*>(tgt_dev + per);
    std::vector<double> taps_host;
    K->m_lo.resize(nk);
    K->len.resize(nk);
    K->off.resize(nk);
    K->kscale.resize(nk);
    std::vector<int32_t> lo_h(per), hi_h(per);
    std::vector<uint32_t> mx_h(per);
    std::vector<int64_t> offc(per);
    std::vector<double> chunk_taps;
    for (int k0 = 0; k0 < nk; k0 += per) {
      const int cnt = std::min(per, nk - k0);
      RF_HIP(hipMemcpyAsync(tgt_dev, ct.data() + k0, sizeof(Tf2Coef) * cnt, hipMemcpyHostToDevice, ctx->stream));
      RF_HIP(hipMemcpyAsync(par_dev, par.data() + k0, sizeof(RatioParam) * cnt, hipMemcpyHostToDevice, ctx->stream));
      // (the host vectors live until the synchronisation below)
      ratio_spectrum(ctx, grid, nb, ref_dev, tgt_dev, par_dev, spec, cnt);
      fft_inverse_f64(ctx, spec, wout, nb, cnt);
      fill_u32(ctx, reinterpret_cast<uint32_t*>(lo_d), 0x7FFFFFFFu, cnt);
      fill_u32(ctx, reinterpret_cast<uint32_t*>(hi_d), 0x80000000u, cnt);
      fill_u32(ctx, mx_d, 0u, cnt);
      support_scan(ctx, wout, nb, cnt, thr_tap, lo_d, hi_d, mx_d);
      RF_HIP(hipMemcpyAsync(lo_h.data(), lo_d, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, ctx->stream));
      RF_HIP(hipMemcpyAsync(hi_h.data(), hi_d, sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, ctx->stream));
      RF_HIP(hipMemcpyAsync(mx_h.data(), mx_d, sizeof(uint32_t) * cnt, hipMemcpyDeviceToHost, ctx->stream));
      sync(ctx);
      int64_t tot = 0;
      for (int i = 0; i < cnt; ++i) {
        const int k = k0 + i;
        if (lo_h[i] == 0x7FFFFFFF) {
          K->m_lo[k] = 0;
          K->len[k] = 0;
        } else {
          K->m_lo[k] = lo_h[i];
          K->len[k] = hi_h[i] - lo_h[i] + 1;
        }
        float mxf;
        std::memcpy(&mxf, &mx_h[i], 4);
        K->kscale[k] = pow2_scale_for(double(mxf));
        offc[i] = tot;
        tot += K->len[k];
      }
      if (tot > 0) {
        double* dst = static_cast<double*>(ctx->ws[WS_SPLIT].ensure(sizeof(double) * size_t(tot)));
        std::vector<int32_t> mlo32(cnt), len32(cnt);
        for (int i = 0; i < cnt; ++i) {
          mlo32[i] = int32_t(K->m_lo[k0 + i]);
          len32[i] = K->len[k0 + i];
        }
        int64_t* off_d = reinterpret_cast<int64_t*>(ctx->ws[WS_PEAK].ensure(size_t(cnt) * 16 + 64));
        int32_t* mlo_d = reinterpret_cast<int32_t*>(off_d + cnt);
        int32_t* len_d = mlo_d + cnt;
        RF_HIP(hipMemcpyAsync(off_d, offc.data(), sizeof(int64_t) * cnt, hipMemcpyHostToDevice, ctx->stream));
        RF_HIP(hipMemcpyAsync(mlo_d, mlo32.data(), sizeof(int32_t) * cnt, hipMemcpyHostToDevice, ctx->stream));
        RF_HIP(hipMemcpyAsync(len_d, len32.data(), sizeof(int32_t) * cnt, hipMemcpyHostToDevice, ctx->stream));
        gather_taps(ctx, wout, nb, cnt, off_d, mlo_d, len_d, dst);
        chunk_taps.resize(size_t(tot));
        RF_HIP(hipMemcpyAsync(chunk_taps.data(), dst, sizeof(double) * size_t(tot), hipMemcpyDeviceToHost, ctx->stream));
        sync(ctx);
      }
      const int64_t base = int64_t(taps_host.size());
      for (int i = 0; i < cnt; ++i) K->off[k0 + i] = base + offc[i];
      taps_host.insert(taps_host.end(), chunk_taps.begin(), chunk_taps.begin() + tot);
    }
    finalize_kernel_set(ctx, K, taps_host);
    *out = K;
  });
  if (st != RF_OK && K) {
    free_kernels(K);
    if (out) *out = nullptr;
  }
  return st;
}

rf_status rf_kernels_save(rf_ctx* ctx, const rf_kernels* k, const char* path) {
  if (!ctx) return RF_E_INVAL;
  return guarded(ctx, [&] {
    RF_CHECK(k && path, "rf_kernels_save: null pointer");
    RF_CHECK(k->device == ctx->device, "rf_kernels_save: kernel set on another device");
    std::vector<double> taps(static_cast<size_t>(k->total_taps));
    if (k->total_taps > 0)
      copy_sync(ctx, taps.data(), k->taps64, sizeof(double) * taps.size(), hipMemcpyDeviceToHost);
    std::FILE* f = std::fopen(path, "wb");
    RF_CHECK(f != nullptr, std::string("rf_kernels_save: cannot open ") + path);
    FileCloser fc{f};
    RF_CHECK(std::fwrite(kSetTag, 1, 8, f) == 8, "rf_kernels_save: write failed");
    SetWriter w{f};
    const int32_t version = 1, nk = k->nk;
    const size_t n = size_t(nk);
    w.put(&version, 4);
    w.put(&nk, 4);
    w.put(&k->n_build, 8);
    w.put(&k->fs, 8);
    w.put(&k->total_taps, 8);
    w.put(k->m_lo.data(), 8 * n);
    w.put(k->len.data(), 4 * n);
    w.put(k->off.data(), 8 * n);
    w.put(k->norm_ratio.data(), 8 * n);
    w.put(k->df_low.data(), 8 * n);
    w.put(k->kscale.data(), 8 * n);
    w.put(taps.data(), 8 * taps.size());
    const uint64_t h = w.h;
    RF_CHECK(std::fwrite(&h, 1, 8, f) == 8, "rf_kernels_save: write failed");
    fc.f = nullptr;
    RF_CHECK(std::fclose(f) == 0, "rf_kernels_save: write failed");
  });
}

rf_status rf_kernels_load(rf_ctx* ctx, const char* path, rf_kernels** out) {
  if (out) *out = nullptr;
  if (!ctx) return RF_E_INVAL;
  rf_kernels* K = nullptr;
  rf_status st = guarded(ctx, [&] {
    RF_CHECK(path && out, "rf_kernels_load: null pointer");
    std::FILE* f = std::fopen(path, "rb");
    RF_CHECK(f != nullptr, std::string("rf_kernels_load: cannot open ") + path);
    FileCloser fc{f};
    char tag[8];
    RF_CHECK(std::fread(tag, 1, 8, f) == 8 && std::memcmp(tag, kSetTag, 8) == 0,
             "rf_kernels_load: not a kernel-set file");
    SetReader r{f};
    int32_t version = 0, nk = 0;
    int64_t n_build = 0, total = 0;
    double fs = 0;
    r.get(&version, 4);
    r.get(&nk, 4);
    r.get(&n_build, 8);
    r.get(&fs, 8);
    r.get(&total, 8);
    RF_CHECK(version == 1, "rf_kernels_load: unknown version");
    RF_CHECK(nk >= 1 && nk <= (1 << 24), "rf_kernels_load: bad kernel count");
    RF_CHECK(is_pow2(n_build) && n_build >= 256 && n_build <= (int64_t(1) << 24), "rf_kernels_load: bad n_build");
    RF_CHECK(std::isfinite(fs) && fs > 0, "rf_kernels_load: bad sampling rate");
    RF_CHECK(total >= 0 && total <= int64_t(nk) * n_build, "rf_kernels_load: bad tap count");
    K = new rf_kernels();
    K->device = ctx->device;
    K->nk = nk;
    K->n_build = n_build;
    K->fs = fs;
    const size_t n = size_t(nk);
    K->m_lo.resize(n);
    K->len.resize(n);
    K->off.resize(n);
    K->norm_ratio.resize(n);
    K->df_low.resize(n);
    K->kscale.resize(n);
    r.get(K->m_lo.data(), 8 * n);
    r.get(K->len.data(), 4 * n);
    r.get(K->off.data(), 8 * n);
    r.get(K->norm_ratio.data(), 8 * n);
    r.get(K->df_low.data(), 8 * n);
    r.get(K->kscale.data(), 8 * n);
    for (size_t i = 0; i < n; ++i) {
      RF_CHECK(K->len[i] >= 0 && K->len[i] <= n_build, "rf_kernels_load: bad kernel length");
      RF_CHECK(K->off[i] >= 0 && K->off[i] + K->len[i] <= total, "rf_kernels_load: taps outside the file");
      RF_CHECK(K->m_lo[i] > -n_build && K->m_lo[i] < n_build, "rf_kernels_load: bad first tap");
      RF_CHECK(std::isfinite(K->norm_ratio[i]) && K->norm_ratio[i] > 0, "rf_kernels_load: bad norm ratio");
      RF_CHECK(std::isfinite(K->df_low[i]) && K->df_low[i] >= 0, "rf_kernels_load: bad taper width");
      int ex = 0;
      RF_CHECK(std::isfinite(K->kscale[i]) && K->kscale[i] > 0 && std::frexp(K->kscale[i], &ex) == 0.5,
               "rf_kernels_load: bad FP16 scale");
    }
    std::vector<double> taps(static_cast<size_t>(total));
    r.get(taps.data(), 8 * taps.size());
    uint64_t h = 0;
    RF_CHECK(std::fread(&h, 1, 8, f) == 8 && h == r.h, "rf_kernels_load: hash mismatch (file damaged)");
    RF_CHECK(std::fgetc(f) == EOF, "rf_kernels_load: bytes after the hash");
    finalize_kernel_set(ctx, K, taps);
    *out = K;
  });
  if (st != RF_OK && K) {
    free_kernels(K);
    if (out) *out = nullptr;
  }
  return st;
}

rf_status rf_kernels_info(const rf_kernels* k, int32_t* nk, int64_t* m_lo, int32_t* len,
                          double* norm_ratio, double* df_low) {
  if (!k) return RF_E_INVAL;
  if (nk) *nk = k->nk;
  for (int i = 0; i < k->nk; ++i) {
    if (m_lo) m_lo[i] = k->m_lo[i];
    if (len) len[i] = k->len[i];
    if (norm_ratio) norm_ratio[i] = k->norm_ratio[i];
    if (df_low) df_low[i] = k->df_low[i];
  }
  return RF_OK;
}

rf_status rf_kernels_split_steps(const rf_kernels* k, int32_t chunk, int64_t* corr_steps, int64_t* all_steps) {
  if (!k || chunk < 256 || chunk > 1024 || chunk % 256 != 0) return RF_E_INVAL;
  if (hipSetDevice(k->device) != hipSuccess) return RF_E_HIP;
  std::vector<uint32_t> flags(size_t(std::max<int64_t>(k->gflag_total, 1)), 0u);
  if (k->gflag_total > 0 && hipMemcpy(flags.data(), k->gflag, sizeof(uint32_t) * size_t(k->gflag_total),
                                      hipMemcpyDeviceToHost) != hipSuccess)
    return RF_E_HIP;
  int64_t corr = 0, all = 0;
  for (const rf::TileDev& T : k->tiles) {
    const int64_t ntaps = T.ksteps * 16;
    const int64_t per = T.pair ? 2 : 1;     // a paired tile's step is half a step's products
    all += T.ksteps / per;                  // ksteps: a multiple of 8
    // the corrections run over chunks of kCorrChunk taps, whatever `chunk` is
    for (int64_t t0 = 0; t0 < ntaps; t0 += rf::kCorrChunk) {
      const int64_t b = std::min<int64_t>(t0 + rf::kCorrChunk, ntaps);
      uint32_t need = 0;
      for (int64_t g = t0 / 256; g < (b + 255) / 256; ++g) need |= flags[size_t(T.gflag_off + g)];
      if (need & 1) corr += (b - t0) / 16 / per;   // bit 1: the correction products
    }
  }
  if (corr_steps) *corr_steps = corr;
  if (all_steps) *all_steps = all;
  return RF_OK;
}

rf_status rf_kernels_taps_fp64(const rf_kernels* k, int32_t idx, double* host_out) {
  if (!k || idx < 0 || idx >= k->nk || (!host_out && k->len[idx] > 0)) return RF_E_INVAL;
  if (k->len[idx] == 0) return RF_OK;
  if (hipSetDevice(k->device) != hipSuccess) return RF_E_HIP;
  if (hipMemcpy(host_out, k->taps64 + k->off[idx], sizeof(double) * size_t(k->len[idx]),
                hipMemcpyDeviceToHost) != hipSuccess)
    return RF_E_HIP;
  return RF_OK;
}

rf_status rf_kernels_free(rf_kernels* k) {
  if (!k) return RF_E_INVAL;
  (void)hipSetDevice(k->device);
  (void)hipDeviceSynchronize();
  free_kernels(k);
  return RF_OK;
}

}  // extern "C"

namespace rf {
namespace {

void check_reconstruct_args(const rf_kernels* K, const void* z_ref, int64_t n, rf_prec prec, const void* z_out,
                            const rf_peak_args* fused, const char* who) {
  // messages are built only on failure (the no-allocation entry point shares this)
  RF_CHECK(K && z_ref, std::string(who) + ": null pointer");
  RF_CHECK(z_out || fused, std::string(who) + ": need z_out or fused read-out");
  RF_CHECK(prec == RF_PREC_FP32 || prec == RF_PREC_SPLIT_FP16, std::string(who) + ": bad precision");
  RF_CHECK(is_pow2(n) && n >= 256 && n <= (int64_t(1) << 24),
           std::string(who) + ": n must be a power of two in [2^8, 2^24]");
  for (const TileDev& T : K->tiles)
    RF_CHECK(T.ksteps * 16 <= n, std::string(who) + ": kernel support longer than the segment");
  if (fused) {
    RF_CHECK(fused->peaks && fused->ntrig && fused->cap >= 0 && (fused->cap == 0 || fused->trig),
             std::string(who) + ": bad fused read-out arguments");
    RF_CHECK(std::isfinite(fused->thr) && fused->thr >= 0, std::string(who) + ": bad threshold");
  }
}

// snr_reconstruct on the given work buffers (split: 4 n halves + 256 bytes,
// packed: nk + 1 keys); arguments already checked.
void reconstruct_on(rf_ctx* ctx, const rf_kernels* K, const void* z_ref, int64_t n, rf_prec prec, void* z_out,
                    const rf_peak_args* fused, const ReconScratch& ws, const char* who) {
  PeakOut po{};
  if (fused) {
    fill_u64(ctx, ws.packed, 0ull, K->nk + 1);
    po.packed = ws.packed;
    po.count = reinterpret_cast<unsigned long long*>(ws.packed + K->nk);
    po.trig = fused->trig;
    po.cap = fused->cap;
    po.thr2 = fused->thr * fused->thr;
    po.seg = 0;
    po.nk = K->nk;
  }
  const void* src = z_ref;
  const float* zinv = nullptr;
  if (prec == RF_PREC_SPLIT_FP16) {
    uint32_t* mx = reinterpret_cast<uint32_t*>(ws.split + sizeof(__half) * 4 * size_t(n));
    float* inv = reinterpret_cast<float*>(mx + 16);
    split_launch(ctx, static_cast<const float2*>(z_ref), n, mx, reinterpret_cast<__half*>(ws.split), inv);
    src = ws.split;
    zinv = inv;
  }
  if (!K->tiles.empty())
    recon_launch(ctx, prec, src, n, K->tiles_dev, int(K->tiles.size()), K, zinv, static_cast<float2*>(z_out), po,
                 fused != nullptr);
  if (fused) {
    peaks_finalize(ctx, ws.packed, K->nk, fused->peaks);
    unsigned long long cnt = 0;
    RF_HIP(hipMemcpyAsync(&cnt, po.count, sizeof(cnt), hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    *fused->ntrig = int64_t(cnt);
    if (int64_t(cnt) > fused->cap) throw Error{RF_E_OVERFLOW, std::string(who) + ": trigger buffer overflow"};
  }
}

}  // namespace
}  // namespace rf

extern "C" {

rf_status snr_reconstruct(rf_ctx* ctx, const rf_kernels* K, const void* z_ref, int64_t n,
                          rf_prec prec, void* z_out, const rf_peak_args* fused) {
  if (!ctx) return RF_E_INVAL;
  return guarded(ctx, [&] {
    check_reconstruct_args(K, z_ref, n, prec, z_out, fused, "snr_reconstruct");
    ReconScratch ws{nullptr, nullptr};
    if (fused) ws.packed = static_cast<uint64_t*>(ctx->ws[WS_PEAK].ensure(sizeof(uint64_t) * (K->nk + 1)));
    if (prec == RF_PREC_SPLIT_FP16)
      ws.split = static_cast<char*>(ctx->ws[WS_SPLIT].ensure(sizeof(__half) * 4 * size_t(n) + 256));
    reconstruct_on(ctx, K, z_ref, n, prec, z_out, fused, ws, "snr_reconstruct");
  });
}

rf_status snr_reconstruct_noalloc(rf_ctx* ctx, const rf_kernels* K, const void* z_ref, int64_t n,
                                  rf_prec prec, void* z_out, const rf_peak_args* fused) {
  if (!ctx) return RF_E_INVAL;
  return guarded(ctx, [&] {
    check_reconstruct_args(K, z_ref, n, prec, z_out, fused, "snr_reconstruct_noalloc");
    RF_CHECK(n <= kNoAllocMaxN, "snr_reconstruct_noalloc: n above the scratch limit of 2^21 samples");
    RF_CHECK(K->nk <= kNoAllocMaxKernels, "snr_reconstruct_noalloc: more than 4096 kernels");
    char* base = scratch_of(ctx->device);
    RF_CHECK(base != nullptr, "snr_reconstruct_noalloc: no scratch address for this device");
    ReconScratch ws{base, reinterpret_cast<uint64_t*>(base + kNoAllocSplitBytes)};
    reconstruct_on(ctx, K, z_ref, n, prec, z_out, fused, ws, "snr_reconstruct_noalloc");
  });
}

rf_status snr_peaks(rf_ctx* ctx, const void* z, int32_t nt, int64_t n, float thr, rf_peak* peaks,
                    rf_trigger* trig, int64_t cap, int64_t* ntrig) {
  if (!ctx) return RF_E_INVAL;
  return guarded(ctx, [&] {
    RF_CHECK(z && peaks && ntrig, "snr_peaks: null pointer");
    RF_CHECK(nt >= 1 && n >= 1 && n <= (int64_t(1) << 30), "snr_peaks: bad sizes");
    RF_CHECK(cap >= 0 && (cap == 0 || trig), "snr_peaks: bad trigger buffer");
    RF_CHECK(std::isfinite(thr) && thr >= 0, "snr_peaks: bad threshold");
    uint64_t* packed = static_cast<uint64_t*>(ctx->ws[WS_PEAK].ensure(sizeof(uint64_t) * (nt + 1)));
    fill_u64(ctx, packed, 0ull, nt + 1);
    PeakOut po{};
    po.packed = packed;
    po.count = reinterpret_cast<unsigned long long*>(packed + nt);
    po.trig = trig;
    po.cap = cap;
    po.thr2 = thr * thr;
    po.seg = 0;
    po.nk = nt;
    peaks_launch(ctx, static_cast<const float2*>(z), nt, n, po);
    peaks_finalize(ctx, packed, nt, peaks);
    unsigned long long cnt = 0;
    RF_HIP(hipMemcpyAsync(&cnt, po.count, sizeof(cnt), hipMemcpyDeviceToHost, ctx->stream));
    sync(ctx);
    *ntrig = int64_t(cnt);
    if (int64_t(cnt) > cap) throw Error{RF_E_OVERFLOW, "snr_peaks: trigger buffer overflow"};
  });
}

}  // extern "C"
