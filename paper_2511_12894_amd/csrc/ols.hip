// Blocked frequency-domain reconstruction (overlap-save): the correlation of
// sec. II.B eq. `convolution`,
//     z_k[m] = c_k sum_s z_ref[(m + s) mod n] w_k[s],   c_k = N_ref / N_k,
// computed block by block with transforms short enough to live in LDS.  The
// paper's CPU reconstruction (sec. IV) is an FFT convolution of this class
// (overlap-add); here every kernel's partition spectra are built once per set.
//
// Blocks of H = 4096 outputs, transforms of B = 2H points.  With M0 the set's
// first tap and G = H / 2, kernel k is cut into P_k partitions of H taps
// starting at M0 + o_k, o_k = a_k G the largest multiple of G not past its
// first tap (a_k = 2 e_k + phi_k).  The input blocks
//     x^phi_c[i] = z_ref[(c H + M0 + phi G + i) mod n],   i < B,  phi in {0, 1},
// give for t < H (t + v < 2H: no wrap inside a block)
//     z_k[b H + t] = sum_{p < P_k} sum_{v < H} x^{phi_k}_{b + e_k + p}[t + v] w_{k,p}[v],
//     w_{k,p}[v] = c_k w_k[M0 + o_k + p H + v]  (zero off the kernel's support),
// and in the frequency domain, per block and kernel,
//     z_k[b H + t] = IDFT( sum_p X^{phi_k}_{b + e_k + p} . W_{k,p} )[t],
//     X = DFT(x) (exp -),  W_{k,p}[f] = (1 / B) sum_v w_{k,p}[v] e^{+2 pi i f v / B},
// IDFT the unnormalised exp(+) sum.  The W are built once per set in FP64
// (stored FP32, P_k B values per kernel); the X once per reconstruction (both
// phases, n / H blocks each: x_c depends on c only through c H mod n).
//
// Mixing kernel: one workgroup of 512 threads per work item (kernel, run of
// consecutive blocks); a thread owns the 16 frequencies j + 512 q, which are
// exactly the inputs of the first radix-16 stage of a Stockham inverse
// transform, so the products never pass through LDS.  The 8192-point transform
// then takes two more radix-16 stages in LDS (two buffers used in turn, three
// barriers a block) and the half of the final radix-2 stage that gives the H
// valid outputs, written straight to the series (runs of 512 consecutive
// samples) and fed to the fused read-out.  Kernels of at most four partitions keep their
// spectra in registers for the whole work item; longer ones read them from the
// cache per block.  Workgroups of one wave of items share the run of blocks,
// so the block spectra come from L2.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "recon.h"

// Every rounding of the transforms is spelled out (explicit fused multiply-adds,
// no contraction by the compiler), so the kernel's variants (series stored or
// not) produce bit-identical series and read-outs.
#pragma clang fp contract(off)

struct rf_ols {
  int device = 0;
  int64_t n = 0;
  int32_t nk = 0;
  int32_t pmax = 0;
  int64_t M0 = 0;
  int nphase = 0;                 // block-spectrum sets in use (1 or 2)
  int phase_slot[2] = {-1, -1};   // set index of each phase
  std::vector<int32_t> P, phase, e;
  std::vector<int64_t> wofs;      // offset of kernel k's spectra in W (float2)
  int64_t wtotal = 0;
  float2* W = nullptr;            // [sum_k P_k][B] partition spectra
  void* meta = nullptr;           // device OlsKernel [nk]
  float2* X = nullptr;            // [nphase][n / H][B] block spectra
};

namespace rf {
namespace {

constexpr int kOB = 8192;        // transform length
constexpr int kOH = 4096;        // outputs per block (hop)
constexpr int kOG = 2048;        // alignment grid of the partitions
constexpr int kOT = 512;         // threads per workgroup; thread j owns frequencies j + 512 q, q < 16
constexpr int kPReg = 4;         // partitions kept in registers
constexpr int kOChunk = 16;      // blocks per work item
constexpr int kPadN = kOB + kOB / 16;

struct OlsKernel {
  int64_t wofs;
  int32_t P, slot, e, pad;
};

// one float2 of padding every 16: the strided stage writes hit distinct banks
__device__ inline int pad(int i) { return i + (i >> 4); }

// Spectra (block and partition) are stored thread-major: frequency
// f = j + 512 q at 16 j + q, so a thread's 16 values are 128 contiguous bytes.
__host__ __device__ inline int perm(int f) { return ((f & 511) << 4) | (f >> 9); }

__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
__device__ inline float2 cmac(float2 acc, float2 a, float2 b) {
  return make_float2(fmaf(-a.y, b.y, fmaf(a.x, b.x, acc.x)), fmaf(a.y, b.x, fmaf(a.x, b.y, acc.y)));
}
__device__ inline float2 mul_i(float2 a) { return make_float2(-a.y, a.x); }
__device__ inline float2 conj2(float2 a) { return make_float2(a.x, -a.y); }

// in-register DFTs with kernel exp(+2 pi i / R)
__device__ inline void dft4(float2& a, float2& b, float2& c, float2& d) {
  const float2 t0 = cadd(a, c), t1 = csub(a, c), t2 = cadd(b, d), t3 = mul_i(csub(b, d));
  a = cadd(t0, t2);
  c = csub(t0, t2);
  b = cadd(t1, t3);
  d = csub(t1, t3);
}
__device__ inline void dft8(float2* v) {
  float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4(e0, e1, e2, e3);
  dft4(o0, o1, o2, o3);
  const float h = 0.70710678118654752f;
  o1 = make_float2(h * (o1.x - o1.y), h * (o1.x + o1.y));      // * e^{+i pi / 4}
  o2 = mul_i(o2);                                              // * e^{+i pi / 2}
  o3 = make_float2(-h * (o3.x + o3.y), h * (o3.x - o3.y));     // * e^{+3 i pi / 4}
  v[0] = cadd(e0, o0);
  v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1);
  v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2);
  v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3);
  v[7] = csub(e3, o3);
}
// e^{+i pi k / 8}, k < 8
__device__ inline float2 w16(int k) {
  const float c1 = 0.92387953251128676f, s1 = 0.38268343236508977f, h = 0.70710678118654752f;
  switch (k) {
    case 1: return make_float2(c1, s1);
    case 2: return make_float2(h, h);
    case 3: return make_float2(s1, c1);
    case 4: return make_float2(0.f, 1.f);
    case 5: return make_float2(-s1, c1);
    case 6: return make_float2(-h, h);
    case 7: return make_float2(-c1, s1);
    default: return make_float2(1.f, 0.f);
  }
}
__device__ inline void dft16(float2* v) {
  float2 ev[8], od[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    ev[i] = v[2 * i];
    od[i] = v[2 * i + 1];
  }
  dft8(ev);
  dft8(od);
#pragma unroll
  for (int k = 1; k < 8; ++k) od[k] = cmul(od[k], w16(k));
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    v[k] = cadd(ev[k], od[k]);
    v[k + 8] = csub(ev[k], od[k]);
  }
}

// e^{+2 pi i k / B} = hi[k >> 6] lo[k & 63] from two small LDS tables
struct Twiddle {
  float2 lo[64];
  float2 hi[128];
};
__device__ inline void twiddle_init(Twiddle& tw) {
  for (int i = threadIdx.x; i < 192; i += blockDim.x) {
    double sn, cs;
    if (i < 64) {
      sincospi(2.0 * i / kOB, &sn, &cs);
      tw.lo[i] = make_float2(float(cs), float(sn));
    } else {
      sincospi(2.0 * 64 * (i - 64) / kOB, &sn, &cs);
      tw.hi[i - 64] = make_float2(float(cs), float(sn));
    }
  }
}
__device__ inline float2 twiddle(const Twiddle& tw, int k) { return cmul(tw.hi[k >> 6], tw.lo[k & 63]); }

// v[q] *= w^q, q = 1..15, from w and w^4 (each a table value): w^{4a + b} = (w^4)^a w^b
__device__ inline void twiddle_powers(float2* v, float2 w1, float2 w4) {
  const float2 w2 = cmul(w1, w1), w3 = cmul(w2, w1);
  const float2 w8 = cmul(w4, w4), w12 = cmul(w8, w4);
  const float2 lo[4] = {make_float2(1.f, 0.f), w1, w2, w3};
  const float2 hi[4] = {make_float2(1.f, 0.f), w4, w8, w12};
#pragma unroll
  for (int q = 1; q < 16; ++q) {
    const float2 t = (q & 3) == 0 ? hi[q >> 2] : ((q >> 2) == 0 ? lo[q & 3] : cmul(hi[q >> 2], lo[q & 3]));
    v[q] = cmul(v[q], t);
  }
}

// Stockham inverse transform of 8192 points after its first radix-16 stage
// (which wrote a[pad(16 j + q)] and was followed by a barrier): radix 16 at
// sub-lengths 16 (a -> b) and 256 (b -> a) in LDS, one barrier after each
// (ping-pong buffers: a stage never overwrites what another thread still
// reads), then the half of the final radix-2 stage that gives outputs
// t < 4096 from a: out[i] = output j + 512 i, i < 8.  With full = true the
// other half too (out[8 + i] = output 4096 + j + 512 i).  Buffer b is free on
// return; a until every thread has passed the next barrier.
template <bool FULL>
__device__ inline void finish_transform(float2* a, float2* b, const Twiddle& tw, float2 (&out)[FULL ? 16 : 8]) {
  const int j = threadIdx.x;
#pragma unroll
  for (int st = 0; st < 2; ++st) {
    const int ns = st == 0 ? 16 : 256;
    const int step = st == 0 ? 32 : 2;          // B / (ns R)
    const int k = j & (ns - 1);
    const float2* src = st == 0 ? a : b;
    float2* dst = st == 0 ? b : a;
    float2 v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = src[pad(j + 512 * q)];
    twiddle_powers(v, twiddle(tw, k * step), twiddle(tw, 4 * k * step));
    dft16(v);
    const int d = (j / ns) * ns * 16 + k;
#pragma unroll
    for (int q = 0; q < 16; ++q) dst[pad(d + q * ns)] = v[q];
    __syncthreads();
  }
  const float2* s = a;
  // radix 2 at sub-length 4096: output t = a + w^t b, t + 4096 = a - w^t b
  const float2 wj = twiddle(tw, j);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int t = j + 512 * i;
    const float2 a = s[pad(t)], b = cmul(s[pad(t + 4096)], cmul(wj, w16(i)));
    out[i] = cadd(a, b);
    if constexpr (FULL) out[8 + i] = csub(a, b);
  }
}

// 16 values of a thread-major spectrum (128 contiguous bytes)
__device__ inline void load16(const float2* p, float2 (&v)[16]) {
  const float4* p4 = reinterpret_cast<const float4*>(p);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float4 u = p4[i];
    v[2 * i] = make_float2(u.x, u.y);
    v[2 * i + 1] = make_float2(u.z, u.w);
  }
}

// Block spectra: X[slot][c] = DFT_{exp -}(x^phi_c) = conj(IDFT(conj x)), one
// workgroup per (block c, phase set), stored thread-major.
__global__ __launch_bounds__(kOT) void k_ols_blocks(const float2* __restrict__ z, int64_t n, int64_t M0,
                                                    int phase0, float2* __restrict__ X) {
  __shared__ float2 s[2][kPadN];
  __shared__ Twiddle tw;
  const int j = threadIdx.x;
  const int64_t c = blockIdx.x;
  const int phi = phase0 + int(blockIdx.y);   // phases in use are consecutive (0, 1 or both)
  const int64_t nb = n / kOH;
  const int64_t base = (c * kOH + M0 + int64_t(phi) * kOG) & (n - 1);
  twiddle_init(tw);
  float2 v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) v[q] = conj2(z[(base + j + 512 * q) & (n - 1)]);
  dft16(v);
#pragma unroll
  for (int q = 0; q < 16; ++q) s[0][pad(16 * j + q)] = v[q];
  __syncthreads();
  float2 o[16];
  finish_transform<true>(s[0], s[1], tw, o);
  float2* out = X + (int64_t(blockIdx.y) * nb + c) * kOB;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    out[perm(j + 512 * i)] = conj2(o[i]);
    out[perm(4096 + j + 512 * i)] = conj2(o[8 + i]);
  }
}

// partition p of kernel k (scaled by c_k), zero padded to B, in FP64 for the transform
__global__ void k_ols_place(const double* __restrict__ taps, const int64_t* __restrict__ pk,
                            int64_t M0, double2* __restrict__ buf) {
  // pk[5 i ..]: off_k, m_lo_k, len_k, o_k + p H, bits of c_k
  const int i = blockIdx.y;
  const int64_t off = pk[5 * i], mlo = pk[5 * i + 1], len = pk[5 * i + 2], start = pk[5 * i + 3];
  const double ck = __longlong_as_double(pk[5 * i + 4]);
  for (int v = blockIdx.x * 256 + threadIdx.x; v < kOB; v += gridDim.x * 256) {
    double w = 0.0;
    if (v < kOH) {
      const int64_t l = M0 + start + v - mlo;
      if (l >= 0 && l < len) w = ck * taps[off + l];
    }
    buf[int64_t(i) * kOB + v] = make_double2(w, 0.0);
  }
}

// W = transform / B in FP32, thread-major
__global__ void k_ols_store(const double2* __restrict__ tr, int count, float2* __restrict__ W) {
  const double inv = 1.0 / kOB;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < int64_t(count) * kOB;
       i += int64_t(gridDim.x) * 256) {
    const int64_t part = i / kOB;
    const int f = int(i % kOB);
    W[part * kOB + perm(f)] = make_float2(float(tr[i].x * inv), float(tr[i].y * inv));
  }
}

template <bool WREG, bool STORE, bool FUSED>
__global__ __launch_bounds__(kOT, 1) void k_ols_mix(const float2* __restrict__ X, const float2* __restrict__ W,
                                                    const OlsKernel* __restrict__ meta, int nk, int64_t n,
                                                    float2* __restrict__ zout, PeakOut po) {
  __shared__ float2 s[2][kPadN];
  __shared__ Twiddle tw;
  __shared__ Best wbest[kOT / 64];
  int par = 0;                    // buffer roles swap every block
  const int j = threadIdx.x;
  const int64_t nb = n / kOH;
  const int64_t nchunks = (nb + kOChunk - 1) / kOChunk;
  const int64_t items = nchunks * nk;
  twiddle_init(tw);
  __syncthreads();
  for (int64_t item = blockIdx.x; item < items; item += gridDim.x) {
    const int k = int(item % nk);
    const int64_t b0 = (item / nk) * kOChunk, b1 = b0 + kOChunk < nb ? b0 + kOChunk : nb;
    const OlsKernel mk = meta[k];
    const float2* Xs = X + int64_t(mk.slot) * nb * kOB + 16 * j;
    const float2* Wk = W + mk.wofs + 16 * j;
    float2 wr[WREG ? kPReg : 1][16];
    if (WREG) {
#pragma unroll
      for (int p = 0; p < kPReg; ++p) {
        if (p < mk.P) load16(Wk + int64_t(p) * kOB, wr[p]);
        else
#pragma unroll
          for (int q = 0; q < 16; ++q) wr[p][q] = make_float2(0.f, 0.f);
      }
    }
    Best run{-1.f, INT32_MAX};
    for (int64_t b = b0; b < b1; ++b) {
      // products at this thread's frequencies j + 512 q, summed over the partitions
      float2 v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = make_float2(0.f, 0.f);
      if (WREG) {
#pragma unroll
        for (int p = 0; p < kPReg; ++p)
          if (p < mk.P) {
            float2 x[16];
            load16(Xs + ((b + mk.e + p) & (nb - 1)) * kOB, x);
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = cmac(v[q], x[q], wr[p][q]);
          }
      } else {
        for (int p = 0; p < mk.P; ++p) {
          float2 x[16], w[16];
          load16(Xs + ((b + mk.e + p) & (nb - 1)) * kOB, x);
          load16(Wk + int64_t(p) * kOB, w);
#pragma unroll
          for (int q = 0; q < 16; ++q) v[q] = cmac(v[q], x[q], w[q]);
        }
      }
      dft16(v);
      // a = the buffer the previous block's transform left free (its last
      // stage read the other one); one barrier before the next stage reads it
      float2* a = s[par];
      float2* bb = s[par ^ 1];
      par ^= 1;
#pragma unroll
      for (int q = 0; q < 16; ++q) a[pad(16 * j + q)] = v[q];
      __syncthreads();
      float2 o[8];
      finish_transform<false>(a, bb, tw, o);
      const int64_t m0 = b * kOH + j;            // outputs m0 + 512 i, i < 8
      if (STORE) {
        float2* zr = zout + int64_t(k) * n + m0;
#pragma unroll
        for (int i = 0; i < 8; ++i) zr[512 * i] = o[i];
      }
      if (FUSED) {
        // running peak of this thread's outputs; crossings recorded in place
        uint32_t cross = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const float a2 = abs2_rn(o[i].x, o[i].y);
          run = better(run, Best{a2, int32_t(m0 + 512 * i)});
          if (a2 > po.thr2) cross |= 1u << i;
        }
        if (cross) {
#pragma unroll
          for (int i = 0; i < 8; ++i)
            if ((cross >> i) & 1u) {
              const unsigned long long sl = atomicAdd(po.count, 1ull);
              if (int64_t(sl) < po.cap) {
                rf_trigger tr;          // (re, im) for now; finished by trig_finish
                tr.tmpl = k;
                tr.seg = po.seg;
                tr.idx = int32_t(m0 + 512 * i);
                tr.absz = o[i].x;
                tr.argz = o[i].y;
                po.trig[sl] = tr;
              }
            }
        }
      }
    }
    if (FUSED) {
      // the item's peak: wave shuffles, then one wave over the per-wave results
      for (int off = 32; off > 0; off >>= 1) {
        const Best ob{__shfl_xor(run.a2, off), __shfl_xor(run.idx, off)};
        run = better(run, ob);
      }
      if ((j & 63) == 0) wbest[j >> 6] = run;
      __syncthreads();
      if (j == 0)
        for (int w = 1; w < kOT / 64; ++w) run = better(run, wbest[w]);
      __syncthreads();
    }
    if (FUSED && j == 0 && run.a2 >= 0.f) {
      const uint64_t key = (uint64_t(__float_as_uint(run.a2)) << 32) | uint64_t(0xFFFFFFFFu - uint32_t(run.idx));
      atomicMax(reinterpret_cast<unsigned long long*>(po.packed + int64_t(po.seg) * po.nk + k),
                (unsigned long long)key);
    }
  }
}

void free_ols(rf_ols* O) {
  if (!O) return;
  for (void* p : {(void*)O->W, O->meta, (void*)O->X})
    if (p) (void)hipFree(p);
  delete O;
}

unsigned gridsize(int64_t work, int64_t cap) {
  return unsigned(std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, cap)));
}

}  // namespace
}  // namespace rf

using namespace rf;

extern "C" {

rf_status rf_ols_build(rf_ctx* ctx, const rf_kernels* K, int64_t n, rf_ols** out) {
  if (!ctx) return RF_E_INVAL;
  rf_ols* O = nullptr;
  rf_status st = guarded(ctx, [&] {
    RF_CHECK(K && out, "rf_ols_build: null pointer");
    *out = nullptr;
    RF_CHECK(K->device == ctx->device, "rf_ols_build: kernel set on another device");
    RF_CHECK(is_pow2(n) && n >= kOH && n <= (int64_t(1) << 24), "rf_ols_build: n must be a power of two in [4096, 2^24]");
    RF_CHECK(n >= K->n_build, "rf_ols_build: n shorter than the kernels' build length");
    const int nk = K->nk;
    RF_CHECK(nk >= 1, "rf_ols_build: empty kernel set");
    O = new rf_ols();
    O->device = ctx->device;
    O->n = n;
    O->nk = nk;
    int64_t M0 = INT64_MAX;
    for (int k = 0; k < nk; ++k)
      if (K->len[k] > 0) M0 = std::min(M0, K->m_lo[k]);
    if (M0 == INT64_MAX) M0 = 0;
    O->M0 = M0;
    O->P.assign(nk, 0);
    O->phase.assign(nk, 0);
    O->e.assign(nk, 0);
    O->wofs.assign(nk, 0);
    bool used[2] = {false, false};
    int64_t total = 0;
    for (int k = 0; k < nk; ++k) {
      O->wofs[k] = total * kOB;
      if (K->len[k] <= 0) continue;
      const int64_t d = K->m_lo[k] - M0, a = d / kOG, o = a * kOG;
      const int64_t P = (d - o + K->len[k] + kOH - 1) / kOH;
      RF_CHECK(P <= 4096, "rf_ols_build: kernel support too long");
      O->P[k] = int32_t(P);
      O->phase[k] = int32_t(a & 1);
      O->e[k] = int32_t((a >> 1) % (n / kOH));
      used[a & 1] = true;
      O->pmax = std::max<int32_t>(O->pmax, int32_t(P));
      total += P;
    }
    if (!used[0] && !used[1]) used[0] = true;
    for (int ph = 0; ph < 2; ++ph)
      if (used[ph]) O->phase_slot[ph] = O->nphase++;
    O->wtotal = total;
    O->W = dev_alloc<float2>(size_t(std::max<int64_t>(total, 1)) * kOB, "overlap-save: device allocation failed");
    // partition spectra in FP64 batches
    if (total > 0) {
      const int per = 128;
      double2* buf = static_cast<double2*>(ctx->ws[WS_BUILD].ensure(sizeof(double2) * size_t(kOB) * per));
      double2* tr = static_cast<double2*>(ctx->ws[WS_Y].ensure(sizeof(double2) * size_t(kOB) * per));
      int64_t* pk = static_cast<int64_t*>(ctx->ws[WS_SCAN].ensure(sizeof(int64_t) * 5 * per));
      std::vector<int64_t> h;
      int64_t done = 0;
      auto flush = [&] {
        const int cnt = int(h.size() / 5);
        if (!cnt) return;
        copy_sync(ctx, pk, h.data(), sizeof(int64_t) * h.size(), hipMemcpyHostToDevice);
        hipLaunchKernelGGL(k_ols_place, dim3(kOB / 256, unsigned(cnt)), dim3(256), 0, ctx->stream, K->taps64, pk,
                           M0, buf);
        RF_HIP(hipGetLastError());
        fft_inverse_f64(ctx, buf, tr, kOB, cnt);
        hipLaunchKernelGGL(k_ols_store, dim3(gridsize(int64_t(cnt) * kOB, 4096)), dim3(256), 0, ctx->stream, tr,
                           cnt, O->W + done * kOB);
        RF_HIP(hipGetLastError());
        RF_HIP(hipStreamSynchronize(ctx->stream));
        done += cnt;
        h.clear();
      };
      for (int k = 0; k < nk; ++k) {
        if (O->P[k] == 0) continue;
        const int64_t a = (K->m_lo[k] - M0) / kOG;
        for (int p = 0; p < O->P[k]; ++p) {
          int64_t cbits;
          const double ck = K->norm_ratio[k];
          std::memcpy(&cbits, &ck, sizeof(cbits));
          h.insert(h.end(), {K->off[k], K->m_lo[k], int64_t(K->len[k]), a * kOG + int64_t(p) * kOH, cbits});
          if (int(h.size() / 5) == per) flush();
        }
      }
      flush();
    }
    std::vector<OlsKernel> mk(nk);
    for (int k = 0; k < nk; ++k)
      mk[k] = OlsKernel{O->wofs[k], O->P[k], O->P[k] ? O->phase_slot[O->phase[k]] : 0, O->e[k], 0};
    O->meta = dev_alloc<OlsKernel>(size_t(nk), "overlap-save: device allocation failed");
    copy_sync(ctx, O->meta, mk.data(), sizeof(OlsKernel) * nk, hipMemcpyHostToDevice);
    O->X = dev_alloc<float2>(size_t(O->nphase) * size_t(n / kOH) * kOB, "overlap-save: device allocation failed");
    *out = O;
  });
  if (st != RF_OK && O) free_ols(O);
  return st;
}

rf_status rf_ols_info(const rf_ols* O, int32_t* block, int32_t* hop, int32_t* pmax, int32_t* parts,
                      int64_t* spectra_bytes) {
  if (!O) return RF_E_INVAL;
  if (block) *block = kOB;
  if (hop) *hop = kOH;
  if (pmax) *pmax = O->pmax;
  if (parts)
    for (int k = 0; k < O->nk; ++k) parts[k] = O->P[k];
  if (spectra_bytes) *spectra_bytes = O->wtotal * kOB * int64_t(sizeof(float2));
  return RF_OK;
}

rf_status snr_reconstruct_ols(rf_ctx* ctx, const rf_ols* O, const void* z_ref, int64_t n, void* z_out,
                              const rf_peak_args* fused) {
  if (!ctx) return RF_E_INVAL;
  return guarded(ctx, [&] {
    RF_CHECK(O && z_ref, "snr_reconstruct_ols: null pointer");
    RF_CHECK(O->device == ctx->device, "snr_reconstruct_ols: plan on another device");
    RF_CHECK(n == O->n, "snr_reconstruct_ols: series length differs from the build");
    RF_CHECK(z_out || fused, "snr_reconstruct_ols: need z_out or fused read-out");
    if (fused) {
      RF_CHECK(fused->peaks && fused->ntrig && fused->cap >= 0 && (fused->cap == 0 || fused->trig),
               "snr_reconstruct_ols: bad fused read-out arguments");
      RF_CHECK(std::isfinite(fused->thr) && fused->thr >= 0, "snr_reconstruct_ols: bad threshold");
    }
    PeakOut po{};
    uint64_t* packed = nullptr;
    if (fused) {
      packed = static_cast<uint64_t*>(ctx->ws[WS_PEAK].ensure(sizeof(uint64_t) * (O->nk + 1)));
      fill_u64(ctx, packed, 0ull, O->nk + 1);
      po.packed = packed;
      po.count = reinterpret_cast<unsigned long long*>(packed + O->nk);
      po.trig = fused->trig;
      po.cap = fused->cap;
      po.thr2 = fused->thr * fused->thr;
      po.seg = 0;
      po.nk = O->nk;
    }
    const int64_t nb = n / kOH;
    const int phase0 = O->phase_slot[0] >= 0 ? 0 : 1;
    hipLaunchKernelGGL(k_ols_blocks, dim3(unsigned(nb), unsigned(O->nphase)), dim3(kOT), 0, ctx->stream,
                       static_cast<const float2*>(z_ref), n, O->M0, phase0, O->X);
    RF_HIP(hipGetLastError());
    int dev = 0, cus = 0;
    RF_HIP(hipGetDevice(&dev));
    RF_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t items = ((nb + kOChunk - 1) / kOChunk) * O->nk;
    const unsigned grid = unsigned(std::max<int64_t>(1, std::min<int64_t>(items, cus)));
    float2* zo = static_cast<float2*>(z_out);
    const bool wreg = O->pmax <= kPReg;
#define RF_OLS(WR, S, FU)                                                                                  \
  hipLaunchKernelGGL((k_ols_mix<WR, S, FU>), dim3(grid), dim3(kOT), 0, ctx->stream, O->X, O->W,          \
                     static_cast<const OlsKernel*>(O->meta), O->nk, n, zo, po)
    if (wreg) {
      if (zo && fused) RF_OLS(true, true, true);
      else if (zo) RF_OLS(true, true, false);
      else RF_OLS(true, false, true);
    } else {
      if (zo && fused) RF_OLS(false, true, true);
      else if (zo) RF_OLS(false, true, false);
      else RF_OLS(false, false, true);
    }
#undef RF_OLS
    RF_HIP(hipGetLastError());
    if (fused) {
      trig_finish(ctx, fused->trig, po.count, fused->cap);
      peaks_finalize(ctx, packed, O->nk, fused->peaks);
      unsigned long long cnt = 0;
      RF_HIP(hipMemcpyAsync(&cnt, po.count, sizeof(cnt), hipMemcpyDeviceToHost, ctx->stream));
      RF_HIP(hipStreamSynchronize(ctx->stream));
      *fused->ntrig = int64_t(cnt);
      if (int64_t(cnt) > fused->cap) throw Error{RF_E_OVERFLOW, "snr_reconstruct_ols: trigger buffer overflow"};
    }
  });
}

rf_status rf_ols_free(rf_ols* O) {
  if (!O) return RF_E_INVAL;
  (void)hipSetDevice(O->device);
  (void)hipDeviceSynchronize();
  free_ols(O);
  return RF_OK;
}

}  // extern "C"
