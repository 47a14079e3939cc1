/*
 * librf -- ratio-filter reconstruction of matched-filter SNR series on one
 * MI355X (gfx950).  C ABI; every pointer argument is a plain host or device
 * pointer as stated per argument; no C++ types cross this boundary.
 *
 * Method: Murakami, Ghosh, Morisaki, "Efficient Reconstruction of
 * Matched-Filter Signal-to-Noise Ratio Time Series from Nearby Templates for
 * Compact Binary Coalescences Searches", arXiv 2511.12894.
 *
 * Conventions (section II): a~(f) = int a(t) exp(-2 pi i f t) dt.  A data
 * segment holds n samples at rate fs (n a power of two, 2^8 <= n <= 2^24);
 * frequency series hold bins j = 0..n/2 at f_j = j fs / n.  The analysis band
 * is B = { j : f_low <= f_j <= f_high } (the S_n = +inf convention of
 * section II.A).  Complex values are interleaved (re, im).
 *
 * Streams: every call enqueues its work on the stream given to
 * rf_ctx_create.  A call that returns host data (sigma, counts, supports)
 * synchronises that stream before it returns; the others do not.
 *
 * Errors: every call returns an rf_status and never aborts; RF_E_INVAL is
 * returned for null pointers, sizes out of range or an inconsistent grid,
 * before any work is enqueued.  After an error the outputs are undefined and
 * the context stays usable; rf_last_error gives a message.
 */
#ifndef RF_H
#define RF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RF_OK = 0,
  RF_E_INVAL = 1,        /* bad argument                                      */
  RF_E_NOMEM = 2,        /* device or host allocation failed                  */
  RF_E_HIP = 3,          /* a HIP runtime call failed                         */
  RF_E_UNSUPPORTED = 4,  /* valid request this build does not implement       */
  RF_E_OVERFLOW = 5      /* trigger buffer too small; true count is returned  */
} rf_status;

typedef struct rf_ctx rf_ctx;           /* device, borrowed stream, workspace */
typedef struct rf_kernels rf_kernels;   /* truncated ratio kernels on device  */

/* Non-spinning template in detector-frame solar masses; TaylorF2 phase to
 * 3.5PN with Newtonian amplitude, coalescence time and phase zero. */
typedef struct { double m1, m2; } rf_tmpl;

/* Segment sampling and analysis band (section II.A), taper widths (section
 * II.C: df_high = 53 Hz, df_low capped at df_low_max = 5 Hz).  Requirements:
 * n a power of two in [2^8, 2^24]; 0 < f_low - df_low_max;
 * f_low < f_high; f_high + df_high <= fs / 2. */
typedef struct {
  double fs;
  int64_t n;
  double f_low, f_high;
  double df_high, df_low_max;
} rf_grid;

/* Unit of the truncation threshold (section II.D): the paper's 1/s on
 * r(t) = fs * w, or a bare value on the tap w itself. */
typedef enum { RF_THR_PER_SECOND = 0, RF_THR_PER_TAP = 1 } rf_thr_unit;

/* Arithmetic of the reconstruction: plain FP32 (FP32 matrix cores), or
 * z = z_hi + z_lo, w = w_hi + w_lo in FP16 with the three products
 * hi*hi + hi*lo + lo*hi accumulated in FP32. */
typedef enum { RF_PREC_FP32 = 0, RF_PREC_SPLIT_FP16 = 1 } rf_prec;

/* Peak of one series: max_m |z[m]| and the smallest m attaining it.  The
 * comparison is made on |z|^2 = re*re + im*im in FP32 (no fused multiply-add). */
typedef struct { float max_absz; int32_t argmax; } rf_peak;

/* One threshold crossing |z[idx]| > thr of series `tmpl` of segment `seg`. */
typedef struct { int32_t tmpl, seg, idx; float absz, argz; } rf_trigger;

/* Fused read-out for snr_reconstruct (all pointers device except ntrig). */
typedef struct {
  float thr;              /* trigger threshold on |z| (> thr)                 */
  rf_peak* peaks;         /* device [nk]: peak of each reconstructed series   */
  rf_trigger* trig;       /* device [cap]: triggers, unspecified order         */
  int64_t cap;            /* capacity of trig (>= 0)                          */
  int64_t* ntrig;         /* host: number of triggers found (may exceed cap)  */
} rf_peak_args;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream; borrowed, not destroyed).
 * *out receives the context; free it with rf_ctx_destroy. */
rf_status rf_ctx_create(int device, void* hip_stream, rf_ctx** out);
rf_status rf_ctx_destroy(rf_ctx* ctx);
/* Message of the last failed call on ctx (static storage owned by ctx). */
const char* rf_last_error(const rf_ctx* ctx);

/* Complex matched-filter SNR series of nt templates (section II.A, equation
 * matched_filter; for the reference template, equation snr_ref):
 *   N_h^2 = 4 df sum_B |h~_j|^2 / S_j,
 *   z[m]  = sum_{j in B} (4 df / N_h) x~_j conj(h~_j) / S_j exp(2 pi i j m / n),
 * i.e. the SNR for coalescence time m / fs, circular in the segment.
 *   xf    device complex128 [n/2+1]: data x~(f_j) (read only)
 *   psd   device double [n/2+1]: one-sided S_n(f_j) > 0 on B (read only)
 *   tmpl  host [nt] templates; nt >= 1
 *   z     device complex64 [nt][n] (written)
 *   sigma host double [nt] or NULL: N_h of each template (then the call syncs)
 * FP64 template phase (reduced to [-pi, pi] in FP64), FP32 exponential,
 * amplitude and FFT; each template's spectrum is formed inside the first
 * transform pass and never stored. */
rf_status mf_ref_snr(rf_ctx* ctx, const rf_grid* grid, const void* xf, const double* psd,
                     const rf_tmpl* tmpl, int32_t nt, void* z, double* sigma);

/* Direct matched filtering with the read-out only (the comparator of section
 * IV: every template filtered on its own, equation matched_filter): the same
 * series as mf_ref_snr, bit for bit, but the last transform pass reads each
 * one out (running peak of |z|, crossings |z| > out->thr) instead of storing it.
 *   xf, psd, tmpl, nt   as mf_ref_snr
 *   out->peaks   device rf_peak [nt]; out->trig device rf_trigger [out->cap]
 *                (seg = 0, unspecified order); *out->ntrig host count (may
 *                exceed cap).
 * Synchronises; RF_E_OVERFLOW when the count exceeds cap. */
rf_status mf_snr_peaks(rf_ctx* ctx, const rf_grid* grid, const void* xf, const double* psd,
                       const rf_tmpl* tmpl, int32_t nt, const rf_peak_args* out);

/* Exact truncated ratio kernels of nk targets against one reference
 * (sections II.B-II.D):
 *   R~_j = W(f_j) (B_k/B_ref)(f_j) exp(-i (Psi_k - Psi_ref)(f_j)), j = 0..nb/2,
 *   w    = inverse real DFT of R~ over nb = n_build points (FP64),
 *   kept taps: signed indices [m_lo, m_hi] spanning every |w| >= thr/fs
 *   (RF_THR_PER_SECOND) or |w| >= thr (RF_THR_PER_TAP), all taps in between kept;
 *   norm_ratio = N_ref / N_k.
 * W is equation (window) with df_high from the grid and
 * df_low = min(df_low_max, |dtau'(f_low)|^(-1/2)) per target.
 *   psd     device double [n/2+1] (for the norms)
 *   ref     reference template; nbr host [nk] targets, nk >= 1
 *   n_build power of two, 2^8 <= n_build <= n (0 means n)
 *   *out    receives the kernel set (device memory owned by the set).
 * Synchronises the stream. */
rf_status ratio_kernel_build(rf_ctx* ctx, const rf_grid* grid, const double* psd, rf_tmpl ref,
                             const rf_tmpl* nbr, int32_t nk, double thr, rf_thr_unit unit,
                             int64_t n_build, rf_kernels** out);

/* Host copies of the kernel-set layout: any pointer may be NULL.
 * nk: count; m_lo[nk], len[nk] (len = m_hi - m_lo + 1, 0 if nothing reaches
 * the threshold); norm_ratio[nk] = N_ref / N_k; df_low[nk] taper widths. */
rf_status rf_kernels_info(const rf_kernels* k, int32_t* nk, int64_t* m_lo, int32_t* len,
                          double* norm_ratio, double* df_low);
/* FP64 taps of kernel idx into host_out[len[idx]]. */
rf_status rf_kernels_taps_fp64(const rf_kernels* k, int32_t idx, double* host_out);
/* Work of the split-FP16 reconstruction with window chunks of `chunk` taps (a
 * multiple of 256 in [256, 1024]; single calls use 1024): *all_steps receives the
 * number of 16-tap steps over all tiles, *corr_steps the number of those that
 * carry the two correction products, both in units of a 32-kernel tile's step
 * (kernels sorted by first tap fill tiles of 32; a last tile of at most 16
 * kernels is paired: each kernel also sits in a second column 32 taps later,
 * its support extended by 32 taps, and one of its steps counts one half).  A
 * step takes the hi*hi product alone when no column of its tile has a tap with
 * |w| s_k >= 1/2 (s_k the kernel's FP16 scale; such taps are below 2^-14 of the
 * kernel's largest) in the 512-tap block, counted from the tile's first tap,
 * that holds the step.  Neither count depends on `chunk` (the correction pass
 * uses 512-tap chunks whatever the first pass uses); it is checked for validity
 * only.  Either pointer may be NULL.  Synchronises (reads the tiles' granule
 * flags). */
rf_status rf_kernels_split_steps(const rf_kernels* k, int32_t chunk, int64_t* corr_steps, int64_t* all_steps);
rf_status rf_kernels_free(rf_kernels* k);
/* Kernel sets stored and reused (section II.B: the ratio kernels are computed
 * once and kept; the storage figure of section IV is what such a file holds).
 * rf_kernels_save writes k to the file at `path` (created or replaced): an
 * 8-byte tag "RFKSET01", then in the host's byte order (little-endian) int32
 * version 1, int32 nk, int64 n_build, double fs, int64 total_taps, the per-kernel
 * arrays m_lo (int64), len (int32), off (int64, first tap in the concatenated
 * taps), norm_ratio, df_low and kscale (double, the FP16 scale s_k), the FP64
 * taps (total_taps doubles), and a 64-bit FNV-1a hash of every byte after the
 * tag.  rf_kernels_load reads such a file into a new set on ctx's device (tiles
 * and packed operands rebuilt as ratio_kernel_build makes them) and stores its
 * handle in *out; the caller frees it with rf_kernels_free.  Errors:
 * RF_E_INVAL for null pointers, a file that cannot be opened, read or written,
 * and a file that is not a kernel set (tag, version, sizes, hash, or field
 * ranges: lengths within n_build, taps inside the file, finite positive norm
 * ratios and scales); RF_E_NOMEM / RF_E_HIP as elsewhere; *out is NULL after a
 * failed load.  Both synchronise ctx's stream. */
rf_status rf_kernels_save(rf_ctx* ctx, const rf_kernels* k, const char* path);
rf_status rf_kernels_load(rf_ctx* ctx, const char* path, rf_kernels** out);

/* Reconstructed SNR series of every kernel's target (section II.B, equation
 * convolution, on the circular segment):
 *   z_k[m] = (N_ref / N_k) sum_{s = m_lo}^{m_hi} z_ref[(m + s) mod n] w_k[s].
 *   z_ref  device complex64 [n] (from mf_ref_snr of the reference)
 *   n      segment length (power of two, >= the kernels' n_build)
 *   prec   RF_PREC_FP32 (FP32 operands, FP32 partial sums of 32 taps added in
 *          FP64) or RF_PREC_SPLIT_FP16 (z and w split into FP16 hi + lo parts
 *          after power-of-two scales; hi*hi everywhere, hi*lo + lo*hi where a
 *          kernel of the tile has large taps, see rf_kernels_split_steps; FP32
 *          partial sums added in FP64, of at most 128 taps where a kernel of
 *          the tile has taps above 1/64..1/32 of its largest, longer elsewhere)
 *   z_out  device complex64 [nk][n], or NULL to skip the series
 *   fused  NULL, or peak/trigger read-out of every series (then the call syncs);
 *          at least one of z_out and fused must be non-NULL.
 * Returns RF_E_OVERFLOW when fused->cap is exceeded (counts still valid). */
rf_status snr_reconstruct(rf_ctx* ctx, const rf_kernels* k, const void* z_ref, int64_t n,
                          rf_prec prec, void* z_out, const rf_peak_args* fused);

/* snr_reconstruct without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and results, bit for bit, with the work
 * buffers (FP16 split planes of z_ref, the read-out's peak keys) in a static
 * device array of the library, 16 MiB + 33 KiB per device, held until the
 * process ends.  Limits: n <= 2^21 and at most 4096 kernels (RF_E_INVAL
 * beyond).  Every call on one device shares that array, so calls that overlap
 * on a device (other streams or threads) race; calls in one stream are
 * ordered.  Arguments otherwise as snr_reconstruct. */
rf_status snr_reconstruct_noalloc(rf_ctx* ctx, const rf_kernels* k, const void* z_ref, int64_t n,
                                  rf_prec prec, void* z_out, const rf_peak_args* fused);

/* Peak and threshold read-out of nt series of n samples (section IV reads
 * the peak SNR of each series):
 *   z      device complex64 [nt][n]
 *   peaks  device rf_peak [nt]
 *   trig   device rf_trigger [cap] (seg = 0), unspecified order
 *   ntrig  host: number of crossings |z| > thr (may exceed cap).
 * Synchronises; RF_E_OVERFLOW when the count exceeds cap. */
rf_status snr_peaks(rf_ctx* ctx, const void* z, int32_t nt, int64_t n, float thr, rf_peak* peaks,
                    rf_trigger* trig, int64_t cap, int64_t* ntrig);

/* ---- batched form (many references, uneven neighbour sets, several segments) ----
 *
 * A batch holds nref reference groups (each a template and its kernel set from
 * ratio_kernel_build on the same grid) and nseg data segments.  One call of
 * rf_batch_run computes, for every segment s and reference r, the reference
 * series (as mf_ref_snr) and the reconstructed series of every kernel of group
 * r (as snr_reconstruct with RF_PREC_SPLIT_FP16), reading them out only
 * through the fused peak/threshold read-out -- the series are not stored.  The
 * device work is one captured hipGraph whose reconstruction is a single
 * persistent launch over all (segment, tile, time block) work items, longest
 * tiles first (captured as two graphs, the reference series and the
 * reconstruction with its read-out, replayed back to back).  The graphs read
 * and write only buffers of the batch: each run copies the caller's data in
 * before the replay and the read-out out after it, so new pointers do not
 * re-capture them; a new cap or thr, or new launch settings, do.  Kernel k of
 * group r has global index kbase[r] + k.  The batch borrows psd and the kernel
 * sets' contents are copied (the sets may be freed afterwards); it owns its
 * device buffers (about 24 bytes per sample per (segment, reference)). */
typedef struct rf_batch rf_batch;

/* psd: device double [n/2+1], must outlive the batch; refs: host [nref];
 * ksets: host [nref]; nseg * nref <= 65535.  Synchronises the stream. */
rf_status rf_batch_create(rf_ctx* ctx, const rf_grid* grid, const double* psd, int32_t nref,
                          const rf_tmpl* refs, rf_kernels* const* ksets, int32_t nseg,
                          rf_batch** out);
/* Launch settings of the persistent reconstruction.  Tiles (32 kernels each)
 * fall into three length buckets: bucket 0 holds tiles of at most bucket_hi[0]
 * 16-tap steps, bucket 1 at most bucket_hi[1], bucket 2 the rest (at creation
 * the bounds are the tertiles of the batch's own tile lengths).  Per bucket:
 * the window chunk (taps staged per LDS window and accumulated between FP64
 * folds: 256, 512 or 1024; it changes the rounding order only) and the number
 * of consecutive 256-time blocks one work item covers (1, 2 or 4).
 * xcd_queues = 1 deals the tiles, longest first, to 8 work queues in turn (one
 * per XCD, workgroups being dispatched to the XCDs in turn) so that a tile's
 * operands are fetched into one XCD's L2; a workgroup drains its own queue and
 * then takes the others' remaining items.  None of these changes a result but
 * the chunk. */
typedef struct {
  int32_t chunk[3];
  int32_t blocks[3];
  int32_t xcd_queues;
  int32_t pad;
  int64_t bucket_hi[2];
} rf_batch_tuning;
/* Host copies (any pointer may be NULL): total kernels, work items, kbase[nref],
 * chosen chunk sizes (taps) of the three tile-length buckets. */
rf_status rf_batch_info(const rf_batch* b, int32_t* ktotal, int64_t* nitems, int32_t* kbase,
                        int32_t* chunk_per_bucket);
/* Set the chunk sizes (each 256, 512 or 1024) without timing, the other settings kept. */
rf_status rf_batch_set_chunks(rf_batch* b, const int32_t* chunk_per_bucket);
/* Read or set every launch setting (no timing); RF_E_INVAL for a value outside
 * the sets above or bucket bounds that are negative or decreasing. */
rf_status rf_batch_get_tuning(const rf_batch* b, rf_batch_tuning* t);
rf_status rf_batch_set_tuning(rf_batch* b, const rf_batch_tuning* t);
/* Choose the settings by timing with the data xf_segs (device complex128
 * [nseg][n/2+1]): per bucket every chunk x blocks pair on the same sampled
 * time blocks (about four per workgroup of the launch, in runs of four spread
 * over the bucket's tiles, segments and times; best of three launches each),
 * then one queue against one per XCD on runs of time blocks of up to eight
 * tiles spread over the lengths; the buckets are the creation's tertiles.  The
 * candidates are tried in order of less memory traffic (chunks 1024, 512, 256;
 * blocks 4, 2, 1; per-XCD queues before one queue) and a later one is taken only
 * when more than 1 % faster.  When cache_path is given, a line keyed by the
 * batch's shape and the device name is read if present (no timing) or
 * appended.  Synchronises. */
rf_status rf_batch_autotune(rf_ctx* ctx, rf_batch* b, const void* xf_segs, const char* cache_path);
/* xf_segs: device complex128 [nseg][n/2+1]; peaks: device rf_peak [nseg][ktotal];
 * trig: device rf_trigger [cap] (tmpl = global kernel index, seg = segment);
 * ntrig: host.  Needs a non-NULL stream in ctx (graph capture).  Synchronises;
 * RF_E_OVERFLOW when the crossings exceed cap. */
rf_status rf_batch_run(rf_ctx* ctx, rf_batch* b, const void* xf_segs, float thr, rf_peak* peaks,
                       rf_trigger* trig, int64_t cap, int64_t* ntrig);
/* Host copies (any may be NULL): number of graph captures and of replays
 * since the batch was created, and the duration in ms of the last run's
 * reconstruction graph (the persistent launch with its read-out), from HIP
 * events recorded around it on the context's stream. */
rf_status rf_batch_graph_stats(const rf_batch* b, int64_t* captures, int64_t* replays, float* recon_ms);
rf_status rf_batch_free(rf_batch* b);

/* ---- learned kernels: an MLP predicting ratio kernels in an SVD basis ----
 *
 * The analytic ratio kernel of a pair, h[m] = (1/nb) sum_{j<=nb/2} c_j R~_j
 * e^{2 pi i j m/nb} (c_0 = c_{nb/2} = 1, else 2; w = Re h is the exact kernel
 * of ratio_kernel_build), is taken on the tap window (-window/2, window/2].
 * A surrogate holds: the leading `rank` left singular vectors U of the
 * training kernels (randomized range finder, Cholesky-QR applied twice), and an
 * MLP 4 -> 256 -> 256 -> 256 -> 2 rank (exact GELU) from the standardised
 * features (tau0_ref, tau3_ref, tau0_k - tau0_ref, tau3_k - tau3_ref) (Newtonian
 * and 1.5PN chirp times at f_low) to the coefficients U^H h / scale (real parts,
 * then imaginary parts).  The exact FP64 build provides the training data and
 * the fallback.  Not part of the paper: an extension for storage and build
 * time; its error is always measured against the exact kernels. */
typedef struct rf_surrogate rf_surrogate;

/* Training set: npair pairs (refs[p], nbrs[p]) (host), kernels built exactly
 * on grid (grid.n = build length), window taps (power of two, <= n), rank = 64.
 * omega: device double [npair][nomega] standard-normal draws for the range
 * finder (rank <= nomega <= 256), supplied by the caller.  Synchronises. */
rf_status rf_surrogate_create(rf_ctx* ctx, const rf_grid* grid, const rf_tmpl* refs, const rf_tmpl* nbrs,
                              int32_t npair, int32_t window, int32_t rank, const double* omega,
                              int32_t nomega, rf_surrogate** out);
/* Host copies (any may be NULL): window, rank, numerical rank of the training
 * kernels, their singular values [numerical rank], coefficient scale, steps. */
rf_status rf_surrogate_info(const rf_surrogate* s, int32_t* window, int32_t* rank, int32_t* numerical_rank,
                            double* svals, double* out_scale, int64_t* steps_trained);
/* Parameters: device float [165760], packed W1 [256][4], b1, W2 [256][256], b2,
 * W3 [256][256], b3, W4 [128][256], b4.  set_params also resets Adam state. */
rf_status rf_surrogate_set_params(rf_ctx* ctx, rf_surrogate* s, const float* theta);
rf_status rf_surrogate_get_params(rf_ctx* ctx, const rf_surrogate* s, float* theta);
/* Training rows the surrogate was built with: x device float [npair][4]
 * (standardised features), t device float [npair][128] (targets); either may
 * be NULL.  Synchronises. */
rf_status rf_surrogate_dataset(rf_ctx* ctx, const rf_surrogate* s, float* x, float* t);
/* Loss (mean squared error over rows x 128 outputs) and its gradient for inputs
 * x (device float [rows][4], standardised) and targets t (device [rows][128]);
 * grad_out: device float [165760].  Synchronises. */
rf_status rf_surrogate_grad(rf_ctx* ctx, rf_surrogate* s, const float* x, const float* t, int32_t rows,
                            float* loss_host, float* grad_out);
/* Adam (0.9, 0.999, 1e-8; moments and bias correction continue across calls
 * until set_params) with a cosine learning-rate decay from lr to 0 over this
 * call's `steps` steps, one captured graph per step, batches of training rows
 * order[step][0..batch) (device int32, supplied by the caller).  loss_host:
 * host float [steps] or NULL.  Needs a non-NULL stream.  Synchronises. */
rf_status rf_surrogate_train(rf_ctx* ctx, rf_surrogate* s, const int32_t* order, int32_t steps, int32_t batch,
                             float lr, float* loss_host);
/* Predicted coefficients U^H h of the pairs (ref, nbr[k]): device complex128 [nk][rank]. */
rf_status rf_surrogate_predict(rf_ctx* ctx, rf_surrogate* s, rf_tmpl ref, const rf_tmpl* nbr, int32_t nk,
                               void* coeffs);
/* Exact coefficients U^H h of the pairs (ref, nbr[k]) (kernels built exactly on
 * the training grid): device complex128 [nk][rank].  Synchronises. */
rf_status rf_surrogate_project(rf_ctx* ctx, rf_surrogate* s, rf_tmpl ref, const rf_tmpl* nbr, int32_t nk,
                               void* coeffs);
/* Learned predictive coding of the coefficients (not in the paper): the exact
 * coefficients c = U^H h of the pairs (ref, nbr[k]) are stored as residual
 * codes against the network's prediction p (use_network = 1) or as plain
 * codes (use_network = 0, p = 0):
 *   r = c - p,  scale_k = max_j max(|Re r_j|, |Im r_j|) / qmax  (FP32),
 *   code = round(r / scale_k) in [-qmax, qmax],  qmax = 2^(bits-1) - 1,
 * bits 8 or 16; codes device int8 / int16 [nk][2 rank] (real parts, then
 * imaginary parts), scales device float [nk].  Decoding gives c~ = p + code
 * scale_k (device complex128 [nk][rank]) for rf_surrogate_kernels, so a kernel
 * costs 2 rank codes + one scale instead of its taps; the network shrinks the
 * range the codes must span.  Both synchronise. */
rf_status rf_surrogate_encode(rf_ctx* ctx, rf_surrogate* s, rf_tmpl ref, const rf_tmpl* nbr, int32_t nk,
                              int32_t bits, int32_t use_network, void* codes, float* scales);
rf_status rf_surrogate_decode(rf_ctx* ctx, rf_surrogate* s, rf_tmpl ref, const rf_tmpl* nbr, int32_t nk,
                              int32_t bits, int32_t use_network, const void* codes, const float* scales,
                              void* coeffs);
/* Kernel set of the targets nbr[k] of ref from the surrogate: w = Re(U c) on
 * the window, truncated as ratio_kernel_build truncates, with c the network's
 * prediction, or coeffs (device complex128 [nk][rank]) when not NULL.  A kernel
 * whose support reaches the window edge is replaced by the exact one.  With a check segment
 * (check_grid sharing fs and band, check_xf device complex128 [n_c/2+1],
 * check_psd device double [n_c/2+1]): each kernel's reconstructed series on it
 * is compared with direct matched filtering; where max |dz| > tol the exact
 * FP64 kernel replaces it.  fallback: host int32 [nk] (1 = exact), check_err:
 * host float [nk] (0 without a check); either may be NULL.  Synchronises. */
rf_status rf_surrogate_kernels(rf_ctx* ctx, rf_surrogate* s, const rf_grid* grid, const double* psd, rf_tmpl ref,
                               const rf_tmpl* nbr, int32_t nk, const void* coeffs, double thr, rf_thr_unit unit,
                               const rf_grid* check_grid, const void* check_xf, const double* check_psd,
                               double tol, rf_kernels** out, int32_t* fallback, float* check_err);
rf_status rf_surrogate_free(rf_surrogate* s);

/* ---- factored reconstruction through a basis of a kernel set ----
 *
 * Every kernel of a set is replaced by its projection on the set's leading
 * J-dimensional subspace: with W the kernels on their union support and
 * W W^T = V diag(lambda) V^T, w~_k = sum_{j<J} V[k][j] b_j, b_j = sum_k V[k][j] w_k
 * (the best rank-J approximation).  The correlation of sec. II.B (eq.
 * `convolution`) then splits into J basis correlations y_j = z_ref (*) b_j, done
 * with one forward and J inverse FFTs of length n, and a mixing product
 * z~_k = (N_ref / N_k) sum_j V[k][j] y_j on the matrix cores.  Not in the paper.
 */
typedef struct rf_factored rf_factored;

/* Basis of the kernel set K for series of grid->n samples (a multiple of 256)
 * and grid's band.  J is the smallest basis size whose largest per-kernel
 * relative residual ||w_k - w~_k|| / ||w_k|| is at most tol, capped at jmax
 * (1..512) and at the number of kernels (1..1024); tol <= 0 takes the cap.
 * Sets of more than 256 kernels or 128 basis vectors mix in split FP16 only,
 * by a tiled product (128 kernels x 128 times per workgroup); the basis
 * correlations take J x n complex64 of device memory, the basis spectra
 * J x (band bins).  Synchronises. */
rf_status rf_factored_build(rf_ctx* ctx, const rf_kernels* K, const rf_grid* grid, double tol, int32_t jmax,
                            rf_factored** out);
/* Host copies (any may be NULL): basis size J, union support (first tap m0,
 * length), Gram eigenvalues lambda [nk] (descending), per-kernel relative
 * residuals [nk]. */
rf_status rf_factored_info(const rf_factored* F, int32_t* J, int64_t* m0, int64_t* len, double* lambda,
                           double* resid);
/* As snr_reconstruct with the projected kernels: z_ref device complex64 [n]
 * (n as built), band-limited to the build grid's band (a matched-filter series
 * is); prec selects the mixing product: RF_PREC_FP32 (FP32 matrix cores) or
 * RF_PREC_SPLIT_FP16 (hi/lo FP16 parts of both operands after power-of-two
 * scales, three products, FP32 accumulation); the basis transforms are FP32
 * either way (RF_E_UNSUPPORTED for RF_PREC_FP32 on a large set).  z_out
 * device complex64 [nk][n] or NULL; fused read-out as in snr_reconstruct.
 * Synchronises when fused. */
rf_status snr_reconstruct_factored(rf_ctx* ctx, const rf_factored* F, const void* z_ref, int64_t n, rf_prec prec,
                                   void* z_out, const rf_peak_args* fused);
/* Many segments and sets in one call (sec. II.B per reference; the batching is
 * an implementation form): for every segment s < nseg of xf_segs (device
 * complex128 [nseg][n/2+1], the whitened data as for mf_ref_snr) and every set
 * r < nset, the matched-filter series of reference refs[r] (as mf_ref_snr
 * computes it) and the factored reconstruction of set sets[r] from it (as
 * snr_reconstruct_factored with the fused read-out), all enqueued on ctx's
 * stream with one synchronisation at the end.  Every set must be built for
 * grid->n samples and reside on ctx's device.  out->peaks: device rf_peak
 * [nseg][ktot], ktot = the sets' kernel counts summed, kernel k of set r at
 * index kbase_r + k (kbase_r = the counts of sets 0..r-1); trigger records
 * carry (kbase_r + k, s, sample, |z|, arg z); overflow as in snr_peaks.  The
 * peaks and triggers equal those of the per-(segment, set) calls bit for bit.
 * The conditioned data are formed once per segment. */
rf_status snr_reconstruct_factored_batch(rf_ctx* ctx, const rf_grid* grid, const void* xf_segs, int32_t nseg,
                                         const double* psd, int32_t nset, const rf_factored* const* sets,
                                         const rf_tmpl* refs, rf_prec prec, const rf_peak_args* out);
rf_status rf_factored_free(rf_factored* F);

/* ---- blocked frequency-domain reconstruction (overlap-save) ----
 *
 * The correlation of sec. II.B (eq. `convolution`) with the exact truncated
 * kernels, computed per block of H = 4096 outputs with transforms of
 * B = 8192 points (sec. IV computes it with an FFT convolution of this kind on
 * the CPU).  Each kernel is cut into P_k partitions of H taps aligned to a
 * 2048-tap grid from the set's first tap; its partition spectra (B complex
 * values each) are built once in FP64 and kept in FP32.  A reconstruction
 * transforms every input block once (exp(-) DFT) and, per kernel and block,
 * sums the products with the partition spectra and inverse transforms.  Not
 * the paper's data layout.
 */
typedef struct rf_ols rf_ols;

/* Plan for kernel set K on series of n samples (a power of two in
 * [4096, 2^24], at least the kernels' build length): partition spectra of
 * every kernel and the block-spectrum buffers (2 x 2n complex64 at most).
 * Kernels of more than 4 partitions (over about 14k taps) work but read their
 * spectra from the cache per block.  Synchronises. */
rf_status rf_ols_build(rf_ctx* ctx, const rf_kernels* K, int64_t n, rf_ols** out);
/* Host copies (any may be NULL): transform length B, hop H, largest partition
 * count, partitions of each kernel [nk], bytes of partition spectra. */
rf_status rf_ols_info(const rf_ols* O, int32_t* block, int32_t* hop, int32_t* pmax, int32_t* parts,
                      int64_t* spectra_bytes);
/* As snr_reconstruct (same kernels, same output and fused read-out), for the
 * n the plan was built for; FP32 transforms and products.  Synchronises when
 * fused. */
rf_status snr_reconstruct_ols(rf_ctx* ctx, const rf_ols* O, const void* z_ref, int64_t n, void* z_out,
                              const rf_peak_args* fused);
rf_status rf_ols_free(rf_ols* O);

/* ---- template bank organisation (host only, no device work) ----
 *
 * Section III.A (template bank construction): sets of one reference and its
 * dependent templates.  The bank, ordered by chirp mass, is halved again and
 * again until every subset's durations differ by at most max_spread (10 s in
 * the paper); subsets of more than max_size templates (500) are halved along
 * symmetric mass ratio until none is larger; each set's reference minimises
 * the summed absolute duration difference to the set (a median duration: the
 * lower one for an even count, the first in the set's order among equal
 * durations).  Odd counts put the smaller half first; sorts are stable from
 * bank order.
 */
/* tau[i] = t_c - t(f_low) of template t[i] (TaylorF2, sec. II.C), seconds. */
rf_status rf_template_durations(const rf_tmpl* t, int64_t n, double f_low, double* tau);
/* t[n], tau[n] host inputs (any durations, e.g. from rf_template_durations);
 * group[n] receives each template's set; reference[] (room for n entries)
 * the bank index of each set's reference; *ngroups the number of sets.  Sets
 * are numbered in chirp-mass order, then symmetric-mass-ratio order. */
rf_status rf_bank_organise(const rf_tmpl* t, const double* tau, int64_t n, double max_spread, int32_t max_size,
                           int32_t* group, int64_t* reference, int32_t* ngroups);

#ifdef __cplusplus
}
#endif

#endif /* RF_H */
