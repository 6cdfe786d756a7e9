// HIP kernels (gfx950) of the encrypted-SpMV library.
//
// Layout in HBM: polynomials limb-major, [poly][limb][N] u64 residues in [0, q) (NTT form unless
// stated); scratch between kernels of one key switch is held as balanced doubles.  A limb-level
// transform runs in one workgroup (the transform policies below): N = 16384 keeps half a limb in
// LDS (68 KiB, two workgroups per CU), smaller rings the whole limb, with compile-time register
// rounds whose first and last rounds read and write global memory directly.
#include "hs_device.hpp"
#include "kernels.hpp"
#include "extra.hpp"

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>

namespace hs {

__constant__ u64 c_cdt[20];

#define SMEM() extern __shared__ double smem[]

__device__ __forceinline__ ModD mod_of(const ModTab& t) { return ModD{t.q, t.qinv}; }

// Galois automorphism X -> X^g as an index map on NTT-form limbs:
// NTT(sigma_g a)[k] = NTT(a)[pi(k)], 2 bitrev(pi(k)) + 1 = g (2 bitrev(k) + 1) mod 2N.
__device__ __forceinline__ u32 galois_index(u32 k, u32 g, int logn) {
  const u32 n2m = (2u << logn) - 1;
  const u32 e = 2 * brev_bits(k, logn) + 1;
  const u32 e2 = (u32)(((u64)g * e) & n2m);
  return brev_bits((e2 - 1) >> 1, logn);
}

__device__ __forceinline__ void store_canon(u64* out, const double* s, int n, ModD m, int nt) {
  for (int i = threadIdx.x; i < n; i += nt) out[i] = d2u(canon(s[lpad(i)], m));
}

// ------------------------------------------------------------------ limb-transform policies
// How a workgroup of XF::NT threads runs one length-N transform from an element source in(e)
// (|x| <= q) to an element sink out(e, x) (balanced x, |x| <= 2.9 q forward with the half-limb
// policy's 8-byte twiddles, 2.375 q + 1 with the others, 0.625 q inverse).  Every element is read
// once and written once, each by one thread; the functions end without a barrier, so a caller
// that reuses LDS synchronises first.  fwd_seg leaves the result
// in LDS and hands it to seg(base, count) in one or two segments (element base + e at
// s[lpad(e)]), ending with a barrier.
//   XfRuntime<NT>: any N <= 16 NT, limb in LDS, runtime log N (small rings)
//   XfStatic<NT> : N = 16 NT, compile-time rounds, first/last round on the source/sink directly
//   XfSplit      : N = 16384 with 512 threads and half-limb LDS (two workgroups per CU)
template <int NT_>
struct XfRuntime {
  static constexpr int NT = NT_;
  int logn;
  template <class In, class Out>
  __device__ __forceinline__ void fwd(const In& in, const Out& out, double* s, const double2* __restrict__ tw, const double* __restrict__ twc, ModD m,
                                      int tid = threadIdx.x) const {
    const int n = 1 << logn;
    for (int i = threadIdx.x; i < n; i += NT) s[lpad(i)] = in(i);
    __syncthreads();
    lds_ntt_fwd<NT>(s, logn, tw, m);
    for (int i = threadIdx.x; i < n; i += NT) out(i, s[lpad(i)]);
  }
  template <class In, class Seg>
  __device__ __forceinline__ void fwd_seg(const In& in, const Seg& seg, double* s, const double2* __restrict__ tw, const double* __restrict__ twc, ModD m,
                                          int tid = threadIdx.x) const {
    const int n = 1 << logn;
    for (int i = threadIdx.x; i < n; i += NT) s[lpad(i)] = in(i);
    __syncthreads();
    lds_ntt_fwd<NT>(s, logn, tw, m);
    seg(0, n);
    __syncthreads();
  }
  template <class In, class Out>
  __device__ __forceinline__ void inv(const In& in, const Out& out, double* s, const double2* __restrict__ tw, double2 ninv, ModD m, int tid = threadIdx.x) const {
    const int n = 1 << logn;
    for (int i = threadIdx.x; i < n; i += NT) s[lpad(i)] = in(i);
    __syncthreads();
    lds_ntt_inv<NT>(s, logn, tw, ninv, m);
    for (int i = threadIdx.x; i < n; i += NT) out(i, s[lpad(i)]);
  }
};
template <int NT_>
struct XfStatic {
  static constexpr int NT = NT_;
  static constexpr int LOGN = static_logn(NT_);
  template <class In, class Out>
  __device__ __forceinline__ void fwd(const In& in, const Out& out, double* s, const double2* __restrict__ tw, const double* __restrict__ twc, ModD m,
                                      int tid = threadIdx.x) const {
    ntt_fwd_c<LOGN, NT>(elem_in(in), elem_out(out), s, tw, m, tid);
  }
  template <class In, class Seg>
  __device__ __forceinline__ void fwd_seg(const In& in, const Seg& seg, double* s, const double2* __restrict__ tw, const double* __restrict__ twc, ModD m,
                                          int tid = threadIdx.x) const {
    ntt_fwd_c<LOGN, NT>(elem_in(in), LdsIO{s}, s, tw, m, tid);
    __syncthreads();
    seg(0, 1 << LOGN);
    __syncthreads();
  }
  template <class In, class Out>
  __device__ __forceinline__ void inv(const In& in, const Out& out, double* s, const double2* __restrict__ tw, double2 ninv, ModD m, int tid = threadIdx.x) const {
    ntt_inv_c<LOGN, NT>(elem_in(in), elem_out(out), s, tw, ninv, m, tid);
  }
};
struct XfSplit {
  static constexpr int NT = kSplitNT;
  template <class In, class Out>
  __device__ __forceinline__ void fwd(const In& in, const Out& out, double* s, const double2* __restrict__ tw, const double* __restrict__ twc, ModD m,
                                      int tid = threadIdx.x) const {
    ntt_fwd_split(in, out, s, tw, twc, m, tid);
  }
  template <class In, class Seg>
  __device__ __forceinline__ void fwd_seg(const In& in, const Seg& seg, double* s, const double2* __restrict__ tw, const double* __restrict__ twc, ModD m,
                                          int tid = threadIdx.x) const {
    ntt_fwd_split_seg(in, seg, s, tw, twc, m, tid);
  }
  template <class In, class Out>
  __device__ __forceinline__ void inv(const In& in, const Out& out, double* s, const double2* __restrict__ tw, double2 ninv, ModD m, int tid = threadIdx.x) const {
    ntt_inv_split(in, out, s, tw, ninv, m, tid);
  }
};
// Kernels on these policies keep to 128 VGPRs so that the split form fits two workgroups per CU.
#define HS_XF_KERNEL template <class XF> __global__ void __launch_bounds__(XF::NT) __attribute__((amdgpu_waves_per_eu(4)))

// ------------------------------------------------------------------ standalone NTT
// One workgroup per limb: poly b / nl, limb b % nl, modulus index mod0 + limb (in place).
HS_XF_KERNEL k_ntt(u64* data, int nl, int mod0, int inverse, const ModTab* __restrict__ tab, int logn, XF xf) {
  SMEM();
  const int n = 1 << logn;
  const int b = blockIdx.x;
  const ModTab t = tab[mod0 + b % nl];
  const ModD m = mod_of(t);
  u64* p = data + (size_t)b * n;
  auto in = [p](int i) { return u2d(p[i]); };
  auto out = [p, m](int i, double x) { p[i] = d2u(canon(x, m)); };
  if (inverse) xf.inv(in, out, smem, t.iv, t.ninv, m);
  else xf.fwd(in, out, smem, t.fw, t.fwc, m);
}

// One workgroup of 1024 threads per N = 2^15 limb (in place, canonical u64 in and out), for
// batches of many limbs (the exact ciphertext product's transforms): the half-limb schedule of
// N = 2^14 with twice the threads.  Forward: stage 0 pairs e with e + 2^14 in registers as the
// limb is read (thread t owns elements t + 1024 k of both halves, k < 16, exactly its register
// group of stages 1..4); each half then runs stages 5..14 through LDS (radix-8 rounds at stages
// 5, 8, 11 with two tasks per thread, stage 14 as a radix-2 round into the output) while the other
// half waits in registers.  Inverse: the mirror image (per half stages 0..9 through LDS, 10..13
// in registers; stage 14 and the 1/N scaling on both halves at the end).  LDS: one half limb
// (136 KiB), one workgroup per CU.
static constexpr int kN15Logn = 15, kN15NT = 1024;
__host__ __device__ constexpr int n15_lds_doubles() { return lds_doubles(1 << (kN15Logn - 1)); }

__global__ void __launch_bounds__(kN15NT) __attribute__((amdgpu_waves_per_eu(4)))
k_ntt15(u64* data, int nl, int mod0, int inverse, const ModTab* __restrict__ tab, NttRows rows) {
  SMEM();
  constexpr int LOGN = kN15Logn, NT = kN15NT, H = 1 << (LOGN - 1), EH = H / NT;
  static_assert(EH == 16, "16 elements per thread and half");
  const int b = blockIdx.x;
  const ModTab t = tab[mod0 + b % nl];
  const ModD m = mod_of(t);
  // the row's source and destination (the same limb of `data` unless the row map says otherwise;
  // every element is read before any is written, so in place is fine)
  const u64* src = data + ((size_t)b << LOGN);
  u64* p = data + ((size_t)b << LOGN);
  if (rows.mode != 0) {
    const int i = b / rows.per, q = b % rows.per;
    if (rows.mode == 1) src = (q < rows.split ? rows.opA[i] + ((size_t)q << LOGN) : rows.opB[i] + ((size_t)(q - rows.split) << LOGN));
    else if (rows.out[i]) p = rows.out[i] + ((size_t)q << LOGN);
  }
  const int tid = threadIdx.x;
  const LdsHalf<LOGN - 1> Lh{smem};
  if (!inverse) {
    const double2* tw = t.fw;
    const double* twc = t.fwc;
    auto out = [p, m](int i, double x) { gst(p + i, d2u(canon(x, m))); };
    double a[EH], c[EH];
#pragma unroll
    for (int k = 0; k < EH; k++) {
      a[k] = u2d(gld(src + tid + k * NT));
      c[k] = u2d(gld(src + tid + k * NT + H));
    }
    const double2 w1 = ldtw(tw, 1);
#pragma unroll
    for (int k = 0; k < EH; k++) {
      const double tt = mul_tw(c[k], w1.x, w1.y, m);
      c[k] = a[k] - tt;
      a[k] = a[k] + tt;
    }
    ct_group<4, 1>(a, 0, tw, m);
    Lh.template put<4, 10>(a, tid);
    __syncthreads();
    fwd_round_gc<LOGN, NT, 5, 3, 2>(Lh, Lh, twc, m, 0, tid);
    __syncthreads();
    fwd_round_gc<LOGN, NT, 8, 3, 2>(Lh, Lh, twc, m, 0, tid);
    __syncthreads();
    fwd_round_gc<LOGN, NT, 11, 3, 2>(Lh, Lh, twc, m, 0, tid);
    __syncthreads();
    fwd_round_gc<LOGN, NT, 14, 1, 8>(Lh, elem_out(out), twc, m, 0, tid);
    __syncthreads();
    ct_group<4, 1>(c, 1, tw, m);
    Lh.template put<4, 10>(c, H + tid);
    __syncthreads();
    fwd_round_gc<LOGN, NT, 5, 3, 2>(Lh, Lh, twc, m, 1 << 11, tid);
    __syncthreads();
    fwd_round_gc<LOGN, NT, 8, 3, 2>(Lh, Lh, twc, m, 1 << 11, tid);
    __syncthreads();
    fwd_round_gc<LOGN, NT, 11, 3, 2>(Lh, Lh, twc, m, 1 << 11, tid);
    __syncthreads();
    fwd_round_gc<LOGN, NT, 14, 1, 8>(Lh, elem_out(out), twc, m, 1 << 13, tid);
  } else {
    const double2* tw = t.iv;
    const double2 ninv = t.ninv;
    auto in = [src](int i) { return u2d(gld(src + i)); };
    double a[EH], c[EH];
    inv_round_g<LOGN, NT, 0, 3, 2, false>(elem_in(in), Lh, tw, ninv, m, 0, tid);
    __syncthreads();
    inv_round_g<LOGN, NT, 3, 3, 2, false>(Lh, Lh, tw, ninv, m, 0, tid);
    __syncthreads();
    inv_round_g<LOGN, NT, 6, 3, 2, false>(Lh, Lh, tw, ninv, m, 0, tid);
    __syncthreads();
    inv_round_g<LOGN, NT, 9, 1, 8, false>(Lh, Lh, tw, ninv, m, 0, tid);
    __syncthreads();
    Lh.template get<4, 10>(a, tid);
    gs_group<4, 10, LOGN, false>(a, 0, tw, ninv, m);
    __syncthreads();
    inv_round_g<LOGN, NT, 0, 3, 2, false>(elem_in(in), Lh, tw, ninv, m, 1 << 11, tid);
    __syncthreads();
    inv_round_g<LOGN, NT, 3, 3, 2, false>(Lh, Lh, tw, ninv, m, 1 << 11, tid);
    __syncthreads();
    inv_round_g<LOGN, NT, 6, 3, 2, false>(Lh, Lh, tw, ninv, m, 1 << 11, tid);
    __syncthreads();
    inv_round_g<LOGN, NT, 9, 1, 8, false>(Lh, Lh, tw, ninv, m, 1 << 13, tid);
    __syncthreads();
    Lh.template get<4, 10>(c, H + tid);
    gs_group<4, 10, LOGN, false>(c, 1, tw, ninv, m);
    // stage 14 with the scaling merged into its twiddle: w' = w / N mod q
    const double2 w = ldtw(tw, 1);
    const double wn = canon(mul_tw(w.x, ninv.x, ninv.y, m), m);
    const double wnq = wn / m.q;
#pragma unroll
    for (int k = 0; k < EH; k++) {
      const int e = tid + k * NT;
      const double x = a[k], y = c[k];
      gst(p + e, d2u(canon(mul_tw(x + y, ninv.x, ninv.y, m), m)));
      gst(p + e + H, d2u(canon(mul_tw(x - y, wn, wnq, m), m)));
    }
  }
}

// Forward transforms of many N = 2^14 limbs, software-pipelined: a grid of two workgroups per CU
// loops over the limbs (stride = grid size).  The half-limb schedule above holds both halves in
// registers after the first stage; once the first half has gone to LDS its registers are free, so
// the first-half words of the workgroup's next limb are read into them while the second half runs
// its LDS rounds (prefetching both halves would exceed the 128 registers that keep two workgroups
// on a CU).  The LDS rounds read the 8-byte twiddle table (ct_group_c): half the twiddle bytes,
// which come from L2 and are as many as the limb's own.  The last limb reloads itself: those
// words are not used.
__global__ void __launch_bounds__(kSplitNT) __attribute__((amdgpu_waves_per_eu(4)))
k_ntt_fwd_pipe(u64* data, i64 nlimbs, int nl, int mod0, const ModTab* __restrict__ tab) {
  SMEM();
  constexpr int LOGN = kSplitLogn, NT = kSplitNT, H = 1 << (LOGN - 1), EH = H / NT;
  const int tid = threadIdx.x;
  const i64 stride = gridDim.x;
  i64 b = blockIdx.x;
  if (b >= nlimbs) return;
  const LdsHalf<LOGN - 1> L{smem};
  u64 wa[EH], wb[EH];
#pragma unroll
  for (int k = 0; k < EH; k++) wa[k] = gld(data + ((size_t)b << LOGN) + tid + k * NT);
  for (; b < nlimbs; b += stride) {
    const ModTab t = tab[mod0 + (int)(b % nl)];
    const ModD m = mod_of(t);
    const double2* tw = t.fw;
    const double* twc = t.fwc;
    u64* p = data + ((size_t)b << LOGN);
#pragma unroll
    for (int k = 0; k < EH; k++) wb[k] = gld(p + tid + k * NT + H);
    auto out = [p, m](int i, double x) { gst(p + i, d2u(canon(x, m))); };
    double a[EH], c[EH];
    const double2 w1 = ldtw(tw, 1);
#pragma unroll
    for (int k = 0; k < EH; k++) {
      const double x = u2d(wa[k]), y = u2d(wb[k]);
      const double tt = mul_tw(y, w1.x, w1.y, m);
      a[k] = x + tt;
      c[k] = x - tt;
    }
    ct_group<4, 1>(a, 0, tw, m);
    L.template put<4, 9>(a, tid);
    __syncthreads();
    fwd_round_gc<LOGN, NT, 5, 3, 2>(L, L, twc, m, 0, tid);
    __syncthreads();
    fwd_round_gc<LOGN, NT, 8, 3, 2>(L, L, twc, m, 0, tid);
    __syncthreads();
    fwd_round_gc<LOGN, NT, 11, 3, 2>(L, elem_out(out), twc, m, 0, tid);
    __syncthreads();
    ct_group<4, 1>(c, 1, tw, m);
    L.template put<4, 9>(c, H + tid);
    const i64 nb = b + stride < nlimbs ? b + stride : b;
#pragma unroll
    for (int k = 0; k < EH; k++) wa[k] = gld(data + ((size_t)nb << LOGN) + tid + k * NT);
    __syncthreads();
    fwd_round_gc<LOGN, NT, 5, 3, 2>(L, L, twc, m, 1 << 10, tid);
    __syncthreads();
    fwd_round_gc<LOGN, NT, 8, 3, 2>(L, L, twc, m, 1 << 10, tid);
    __syncthreads();
    fwd_round_gc<LOGN, NT, 11, 3, 2>(L, elem_out(out), twc, m, 1 << 10, tid);
    __syncthreads();
  }
}

// Encryption's forward transforms with the prologue folded into their input: row b = (g, which, l)
// of [G][3][L] transforms U = u (which 0), E1 = e1 (1) or D0 = e0 + floor(Q m / t + 1/2) (2),
// reduced modulo q_l, into NTT form (the same values as the elementwise prologue followed by the
// plain transform, without writing and re-reading them).  Samples [G][3][N] = (u, e0, e1).
HS_XF_KERNEL k_enc_ntt(const u64* __restrict__ mcoef, const int* __restrict__ samples, u64* prep, int L, u64 t, u64 q_mod_t,
                       const double2* __restrict__ qdt, const ModTab* __restrict__ tab, int logn, XF xf) {
  SMEM();
  const int n = 1 << logn;
  const int b = blockIdx.x;
  const int l = b % L, which = (b / L) % 3, g = b / (3 * L);
  const ModTab tb = tab[l];
  const ModD m = mod_of(tb);
  const double q = tb.q;
  const int* u = samples + (size_t)g * 3 * n;
  const u64* mc = mcoef + (size_t)g * n;
  u64* p = prep + (size_t)b * n;
  auto out = [p, m](int i, double x) { p[i] = d2u(canon(x, m)); };
  if (which == 0) {
    xf.fwd([u, q](int i) { const int v = u[i]; return v < 0 ? (double)v + q : (double)v; }, out, smem, tb.fw, tb.fwc, m);
  } else if (which == 1) {
    const int* e1 = u + 2 * n;
    xf.fwd([e1, q](int i) { const int v = e1[i]; return v < 0 ? (double)v + q : (double)v; }, out, smem, tb.fw, tb.fwc, m);
  } else {
    const int* e0 = u + n;
    const double2 qd = qdt[l];
    const double tt = (double)t, th = (double)(t / 2);
    xf.fwd(
        [=](int i) {
          const u64 mv = mc[i];
          const double d1 = mul_tw((double)mv, qd.x, qd.y, m);
          // floor(((Q mod t) m + floor(t/2)) / t): the numerator is below 2^53 (t < 2^26), so the quotient of
          // exactly represented doubles is within 2^-18 of the true one and floor is exact
          const double d2 = floor(((double)(q_mod_t * mv) + th) / tt);
          return canon(reduce((double)e0[i] + d1 + d2, m), m);
        },
        out, smem, tb.fw, tb.fwc, m);
  }
}

// ------------------------------------------------------------------ sampling
// Small-integer samples (int32) of nobj polynomials: object o uses stream (seed, purpose,
// index0 + o * index_step) and is written at out + o * obj_stride.  kind 0: ternary, word i -> (w mod 3) - 1.  kind 1: discrete Gaussian by CDT,
// 64 bits (words 2i, 2i+1) per coefficient: top bit sign, low 63 bits r, |e| = #{k: T[k] <= r}.
__device__ __forceinline__ void sample_small_body(int* out, int nobj, i64 obj_stride, u64 seed, u32 purpose, u64 index0, u64 index_step, int kind,
                                                  int logn) {
  const int n = 1 << logn;
  const int per = kind == 0 ? 16 : 8;
  const int nblk = n / per;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= nobj * nblk) return;
  const int o = gid / nblk, blk = gid % nblk;
  u32 w[16];
  chacha_block(seed, purpose, index0 + (u64)o * index_step, (u32)blk, w);
  int* dst = out + (size_t)o * obj_stride + (size_t)blk * per;
  if (kind == 0) {
#pragma unroll
    for (int i = 0; i < 16; i++) dst[i] = (int)(w[i] % 3u) - 1;
  } else {
#pragma unroll
    for (int i = 0; i < 8; i++) {
      const u64 x = (u64)w[2 * i] | ((u64)w[2 * i + 1] << 32);
      const u64 r = x & 0x7fffffffffffffffULL;
      int mag = 0;
#pragma unroll
      for (int k = 0; k < 20; k++) mag += (c_cdt[k] <= r) ? 1 : 0;
      dst[i] = (x >> 63) ? -mag : mag;
    }
  }
}
__global__ void k_sample_small(int* out, int nobj, i64 obj_stride, u64 seed, u32 purpose, u64 index0, u64 index_step, int kind, int logn) {
  sample_small_body(out, nobj, obj_stride, seed, purpose, index0, index_step, kind, logn);
}
// The three sample polynomials of public-key encryption in one launch: object o (index o) gets
// u (ternary, purpose pu) at out[o][0], e0 and e1 (Gaussian, purposes pe0, pe1) at out[o][1..2];
// blockIdx.y selects the polynomial.
__global__ void k_sample_enc(int* out, int nobj, u64 seed, u32 pu, u32 pe0, u32 pe1, int logn) {
  const int job = blockIdx.y;
  const i64 n = (i64)1 << logn;
  sample_small_body(out + job * n, nobj, 3 * n, seed, job == 0 ? pu : job == 1 ? pe0 : pe1, 0, 1, job == 0 ? 0 : 1, logn);
}

// 128-bit little-endian value (w0..w3) mod q, q < 2^50.
__device__ __forceinline__ u64 u128_mod(u32 w0, u32 w1, u32 w2, u32 w3, u64 q, double2 r64, ModD m) {
  const u64 lo = (u64)w0 | ((u64)w1 << 32), hi = (u64)w2 | ((u64)w3 << 32);
  const double h = u2d(hi % q), l = u2d(lo % q);
  return d2u(canon(mul_tw(h, r64.x, r64.y, m) + l, m));  // hi * (2^64 mod q) + lo
}

// ------------------------------------------------------------------ keys
// Secret key: ternary s (purpose 1, index 0) in NTT form for every modulus of the chain.
template <int NT>
__global__ void __launch_bounds__(NT) k_sk_ntt(u64* sk, const int* s_coef, const ModTab* __restrict__ tab, int logn) {
  SMEM();
  const int n = 1 << logn;
  const ModTab t = tab[blockIdx.x];
  const ModD m = mod_of(t);
  for (int i = threadIdx.x; i < n; i += NT) smem[lpad(i)] = (double)s_coef[i];
  __syncthreads();
  lds_ntt_fwd<NT>(smem, logn, t.fw, m);
  store_canon(sk + (size_t)blockIdx.x * n, smem, n, m, NT);
}

// One limb of a key-switching (or public) key:  b = NTT(e) - a s + [in digit] P s',  a uniform in
// NTT form from stream (seed, purpose_a, idx_a), e from the Gaussian samples e_coef.
// s' mode: 0 none (public key), 1 Galois sigma_g(s) (NTT-domain index map), 2 s^2.

template <int NT>
__global__ void __launch_bounds__(NT) k_ksk_limb(const KskArgs* __restrict__ args, const ModTab* __restrict__ tab, int logn) {
  SMEM();
  const int n = 1 << logn;
  const KskArgs A = args[blockIdx.x];
  const ModTab t = tab[A.mod_index];
  const ModD m = mod_of(t);
  const u64 q = (u64)t.q;
  for (int i = threadIdx.x; i < n; i += NT) smem[lpad(i)] = (double)A.e_coef[i];
  __syncthreads();
  lds_ntt_fwd<NT>(smem, logn, t.fw, m);
  // each thread draws whole ChaCha blocks: block k gives coefficients 4k .. 4k+3
  for (int blk = threadIdx.x; blk < n / 4; blk += NT) {
    u32 w[16];
    chacha_block(A.seed, A.purpose_a, A.idx_a, (u32)blk, w);
#pragma unroll
    for (int c = 0; c < 4; c++) {
      const int i = blk * 4 + c;
      const u64 av = u128_mod(w[4 * c], w[4 * c + 1], w[4 * c + 2], w[4 * c + 3], q, A.r64, m);
      const double ad = u2d(av);
      const double s = u2d(A.sk[i]);
      double v = smem[lpad(i)] - mulmod(ad, s, m);
      if (A.sprime_mode == 1) {
        const double sp = u2d(A.sk[galois_index((u32)i, A.galois, logn)]);
        v += mul_tw(sp, A.pfac.x, A.pfac.y, m);
      } else if (A.sprime_mode == 2) {
        const double s2 = mulmod(s, s, m);
        v += mul_tw(s2, A.pfac.x, A.pfac.y, m);
      }
      A.b[i] = d2u(canon(v, m));
      A.a[i] = av;
    }
  }
}

// ------------------------------------------------------------------ slot packing + encoding
// Builds the slot vector of one plaintext and applies the inverse mod-t NTT (batch encoding):
// coefficients m in [0, t).  Slot k < h*c of chunk (start, c, h): block b = k / h, sorted row
// p = k % h; source value at CSSC entry CP[start + b] + p when p < NNZ[start + b], else 0.
//   mode 0: matrix values va[e];  mode 1: vector values v[ci[e]];  mode 2: mask (1 for k < h).

template <int NT>
__global__ void __launch_bounds__(NT) k_pack_encode(PackArgs A, const u32* __restrict__ slot_pos, const ModTab* __restrict__ tab, int tmod, int logn) {
  SMEM();
  const int n = 1 << logn;
  const int g = blockIdx.x;
  const int mode = A.mode == 3 ? (g < A.nG ? 0 : 2) : A.mode;
  // (start, c, h, cp_off, nnz_off, group, cp_off of slot row 1 or -1, nnz_off of slot row 1)
  const i64* cd = A.chunk + 8 * (A.mode == 3 && g >= A.nG ? g - A.nG : g);
  const i64 start = cd[0], cols = cd[1], h = cd[2];
  const ModTab t = tab[tmod];
  const ModD m = mod_of(t);
  const i64 tq = (i64)t.q;
  for (int k = threadIdx.x; k < n; k += NT) {
    const int srow = k >= n / 2;
    const i64 kk = k - srow * (n / 2);
    const i64 cpo = srow ? cd[6] : cd[3], nzo = srow ? cd[7] : cd[4];
    i64 val = 0;
    if (cpo < 0) {
      val = 0;   // no partition in this slot row
    } else if (mode == 2) {
      val = (kk < h) ? 1 : 0;
    } else if (kk < h * cols) {
      const i64 b = kk / h, p = kk % h;
      const i64 c0 = A.cp[cpo + start + b], c1 = A.cp[cpo + start + b + 1];
      if (p < c1 - c0) {
        const i64 e = nzo + c0 + p;
        val = (mode == 0) ? A.va[e] : A.v[A.ci[e]];
      }
    }
    val %= tq;
    if (val < 0) val += tq;
    smem[lpad(slot_pos[k])] = (double)val;
  }
  __syncthreads();
  if constexpr (static_logn(NT) > 0) {
    if (logn == static_logn(NT)) {   // the compile-time whole-limb schedule, in place from LDS
      u64* o = A.out + (size_t)g * n;
      ntt_inv_c<static_logn(NT), NT>(LdsIO{smem}, elem_out([o, m](int i, double x) { o[i] = d2u(canon(x, m)); }), smem, t.iv,
                                     t.ninv, m);
      return;
    }
  }
  lds_ntt_inv<NT>(smem, logn, t.iv, t.ninv, m);
  store_canon(A.out + (size_t)g * n, smem, n, m, NT);
}

// Plaintext for ct x pt: centered lift of the mod-t coefficients (c > (t-1)/2 -> c - t), NTT mod
// data prime `limb`.  grid = (L, n_plain).
HS_XF_KERNEL k_plain_ntt(const u64* __restrict__ coef, u64* out, int L, u64 t, const ModTab* __restrict__ tab, int logn, XF xf) {
  SMEM();
  const int n = 1 << logn;
  const int l = blockIdx.x, g = blockIdx.y;
  const ModTab tb = tab[l];
  const ModD m = mod_of(tb);
  const u64* c = coef + (size_t)g * n;
  u64* o = out + ((size_t)g * L + l) * n;
  auto in = [c, t](int i) {
    const u64 v = c[i];
    return v > (t - 1) / 2 ? (double)v - (double)t : (double)v;
  };
  auto sink = [o, m](int i, double x) { o[i] = d2u(canon(x, m)); };
  xf.fwd(in, sink, smem, tb.fw, tb.fwc, m);
}

// ------------------------------------------------------------------ encryption
// c0 = pk0 NTT(u) + NTT(e0 + floor(Q m / t + 1/2)),  c1 = pk1 NTT(u) + NTT(e1), per limb.
// floor(Q m / t + 1/2) = floor(Q/t) m + floor(((Q mod t) m + floor(t/2)) / t).
// samples: [n_ct][3][N] int32 (u, e0, e1).  grid = (L, n_ct).
template <int NT>
__global__ void __launch_bounds__(NT) k_encrypt(const u64* __restrict__ mcoef, const int* __restrict__ samples, const u64* __restrict__ pk,
                                                u64* out, int L, u64 t, u64 q_mod_t, const double2* __restrict__ qdt,
                                                const ModTab* __restrict__ tab, int logn) {
  SMEM();
  constexpr int PER = 16;  // n / NT <= 16 for every ring size
  const int n = 1 << logn;
  const int l = blockIdx.x, g = blockIdx.y;
  const ModTab tb = tab[l];
  const ModD m = mod_of(tb);
  const int* u = samples + (size_t)g * 3 * n;
  const int* e0 = u + n;
  const int* e1 = u + 2 * n;
  const u64* mc = mcoef + (size_t)g * n;
  u64* c0 = out + ((size_t)g * 2 * L + l) * n;
  u64* c1 = out + ((size_t)g * 2 * L + L + l) * n;
  const u64* p0 = pk + (size_t)l * n;
  const u64* p1 = pk + ((size_t)L + l) * n;
  double U[PER];
  // NTT(u)
  for (int i = threadIdx.x; i < n; i += NT) smem[lpad(i)] = (double)u[i];
  __syncthreads();
  lds_ntt_fwd<NT>(smem, logn, tb.fw, m);
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const int i = threadIdx.x + k * NT;
    if (i < n) U[k] = smem[lpad(i)];
  }
  __syncthreads();
  // c1
  for (int i = threadIdx.x; i < n; i += NT) smem[lpad(i)] = (double)e1[i];
  __syncthreads();
  lds_ntt_fwd<NT>(smem, logn, tb.fw, m);
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const int i = threadIdx.x + k * NT;
    if (i < n) c1[i] = d2u(canon(mulmod(reduce(U[k], m), u2d(p1[i]), m) + smem[lpad(i)], m));
  }
  __syncthreads();
  // c0
  const double2 qd = qdt[l];
  for (int i = threadIdx.x; i < n; i += NT) {
    const u64 mv = mc[i];
    const double d1 = mul_tw((double)mv, qd.x, qd.y, m);
    const double d2 = (double)((q_mod_t * mv + t / 2) / t);
    smem[lpad(i)] = reduce((double)e0[i] + d1 + d2, m);
  }
  __syncthreads();
  lds_ntt_fwd<NT>(smem, logn, tb.fw, m);
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const int i = threadIdx.x + k * NT;
    if (i < n) c0[i] = d2u(canon(mulmod(reduce(U[k], m), u2d(p0[i]), m) + smem[lpad(i)], m));
  }
}

// ------------------------------------------------------------------ slot-wise products
// out[g] = x[g] (.) pt[g], both polynomials; x, out: [n][2][L][N]; pt: [n][L][N].
// grid (N / (256 EW_EPT), rows): a block's row (g, w, l) is uniform; rows loop over gridDim.y.
static constexpr int EW_EPT = 4;
__global__ void k_mul_plain(const u64* __restrict__ x, const u64* __restrict__ pt, u64* out, i64 n_ct, int L,
                            int pt_stride_ct, const ModTab* __restrict__ tab, int logn) {
  const i64 n = 1 << logn;
  for (i64 row = blockIdx.y; row < n_ct * 2 * L; row += gridDim.y) {
    const int l = (int)(row % L);
    const i64 g = row / (2 * L);
    const ModD m = mod_of(tab[l]);
    const u64* xr = x + row * n;
    const u64* pr = pt + (g * pt_stride_ct + l) * n;
    u64* orow = out + row * n;
#pragma unroll
    for (int e = 0; e < EW_EPT; e++) {
      const i64 k = ((i64)blockIdx.x * EW_EPT + e) * blockDim.x + threadIdx.x;
      if (k < n) orow[k] = d2u(canon(mulmod(u2d(xr[k]), u2d(pr[k]), m), m));
    }
  }
}

// res[P] = sum over the chunks g of partition P of w[g] (.) mask[g]   (mask == nullptr: plain sum)
// grid (N / 256, 2 L, partitions): a block's row (w, l) is uniform; one element per thread, so that
// the chain over the partition's chunks (a pointer, then the words) runs in many threads at once.
__global__ void k_mask_acc(const u64* const* __restrict__ w, const u64* __restrict__ mask, const int* __restrict__ part_chunk0,
                           const int* __restrict__ part_nchunks, u64* res, int L, const ModTab* __restrict__ tab, int logn) {
  const int n = 1 << logn;
  const int P = blockIdx.z, row = blockIdx.y;   // row = w L + l
  const int l = row % L;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int g0 = part_chunk0[P], ng = part_nchunks[P];
  const ModD m = mod_of(tab[l]);
  double acc = 0.0;
  // four chunks at a time: their words (and masks) are all requested before the first is used
  constexpr int U = 4;
  for (int g = g0; g < g0 + ng; g += U) {
    u64 wv[U], mv[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int gg = g + u < g0 + ng ? g + u : g;
      const u64* wp = w[gg] + (size_t)row * n + k;
      wv[u] = gld(wp);
      mv[u] = gld(mask ? mask + ((size_t)gg * L + l) * n + k : wp);   // no branch around the load
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      if (g + u < g0 + ng) {
        double v = u2d(wv[u]);
        if (mask) v = mulmod(v, u2d(mv[u]), m);
        acc = reduce(acc + v, m);
      }
    }
  }
  res[((size_t)P * 2 * L + row) * n + k] = d2u(canon(acc, m));
}

// ------------------------------------------------------------------ rotation: key switching
// Batched power-of-two rotations.  Item b: out = (sigma_g(c0) + ks0, ks1) [+ addend], where
// (ks0, ks1) = KeySwitch(sigma_g(c1)) under the key for sigma_g(s) -> s.
//  1. k_rot_intt      sigma_g(c1) limbs (NTT-domain gather) -> coefficient form D[b][l] (u64)
//  2. k_modup_ip      per target modulus m and digit group: for each digit j,
//                     ext = (m in D_j) ? sigma_g(c1)_m : NTT_m(Conv_{D_j -> m}(D[b][D_j])),
//                     acc_w += ext (.) ksk_w[j][m]  -> ACC[b][dg][w][m] (balanced doubles)
//  3. k_moddown_intt  special limbs of sum_dg ACC -> coefficient form PC[b][w][k]
//  4. k_moddown_ntt   conv_i = NTT_i(Conv_{P -> q_i}(PC)), out_w,i = (acc_w,i - conv_i) P^-1
//                     (+ sigma_g(c0)_i for w = 0) (+ addend_w,i)
HS_XF_KERNEL k_rot_intt(const RotItem* __restrict__ items, u64* D, int L, const ModTab* __restrict__ tab, int logn, XF xf) {
  SMEM();
  const int n = 1 << logn;
  const int l = blockIdx.x, b = blockIdx.y;
  const RotItem it = items[b];
  const ModTab tb = tab[l];
  const ModD m = mod_of(tb);
  const u64* c1 = it.in + ((size_t)L + l) * n;
  const u32 gal = it.galois;
  u64* o = D + ((size_t)b * L + l) * n;
  auto in = [c1, gal, logn](int i) { return u2d(c1[galois_index((u32)i, gal, logn)]); };
  auto sink = [o, m](int i, double x) { o[i] = d2u(canon(x, m)); };
  xf.inv(in, sink, smem, tb.iv, tb.ninv, m);
}

// Accumulators live in the output rows ACC; a barrier separates the digits (element ownership
// differs between the transform's sink and the own-limb loop).  The accumulate step takes a
// thread's elements KB at a time with every load of the batch (key words, accumulators, the
// own limb's gathered words) issued before the first use, instead of one element's round trip
// after another.  The half-limb form holds the other half in registers during its first segment,
// so it batches fewer elements (within its 128 VGPRs).
template <class XF> struct KsBatch { static constexpr int value = 8; };
template <> struct KsBatch<XfSplit> { static constexpr int value = 2; };
HS_XF_KERNEL k_modup_ip(const RotItem* __restrict__ items, const u64* __restrict__ D, double* ACC, KsShape S,
                        const double2* __restrict__ up_inv, const double2* __restrict__ up_hat, const ModTab* __restrict__ tab,
                        int logn, XF xf) {
  SMEM();
  constexpr int NT = XF::NT;
  constexpr int KB = KsBatch<XF>::value;
  const int n = 1 << logn;
  const int mi = blockIdx.x, b = blockIdx.y, dg = blockIdx.z;
  const int LK = S.L + S.K;
  const RotItem it = items[b];
  const ModTab tb = tab[mi];
  const ModD m = mod_of(tb);
  const int j0 = dg * S.dpg, j1 = min(S.dnum, j0 + S.dpg);
  double* o0 = ACC + ((((size_t)b * S.ndg + dg) * 2 + 0) * LK + mi) * n;
  double* o1 = ACC + ((((size_t)b * S.ndg + dg) * 2 + 1) * LK + mi) * n;
  for (int j = j0; j < j1; j++) {
    // the transform's per-thread address arithmetic (and twiddle base) is recomputed per digit
    // instead of being hoisted out of the loop and held in registers across it
    int tid = threadIdx.x;
    const double2* tw = tb.fw;
    const double* twc = tb.fwc;
    asm volatile("" : "+v"(tid), "+s"(tw), "+s"(twc));
    const int lo = j * S.alpha, hi = min(S.L, lo + S.alpha);
    const bool own = (mi >= lo && mi < hi);
    const bool first = (j == j0);
    const u64* kb = it.key + (((size_t)0 * S.dnum + j) * LK + mi) * n;
    const u64* ka = it.key + (((size_t)1 * S.dnum + j) * LK + mi) * n;
    // elements base + e, e = e0 + c NT < cnt; value(c, e) reads the digit element (LDS or gathered)
    auto accumulate = [&](int base, int cnt, int e0, auto&& value) {
      u64 wb[KB], wa[KB];
      double a0[KB], a1[KB];
#pragma unroll
      for (int c = 0; c < KB; c++) {
        const int e = e0 + c * NT;
        const int i = base + (e < cnt ? e : e0);
        wb[c] = gld(kb + i);
        wa[c] = gld(ka + i);
        a0[c] = gld(o0 + i);  // read also for the first digit (ignored): no branch around the load
        a1[c] = gld(o1 + i);
      }
#pragma unroll
      for (int c = 0; c < KB; c++) {
        const int e = e0 + c * NT;
        if (e < cnt) {
          const double x = reduce(value(c, e), m);
          // the transform's outputs are within 2.9 q, so the products are exact but may reach
          // about 2.2 q: reduced before they are stored or summed
          double v0 = mulmod(x, u2d(wb[c]), m);
          double v1 = mulmod(x, u2d(wa[c]), m);
          v0 = reduce(first ? v0 : v0 + a0[c], m);
          v1 = reduce(first ? v1 : v1 + a1[c], m);
          gst(o0 + base + e, v0);
          gst(o1 + base + e, v1);
        }
      }
    };
    if (own) {
      const u64* c1 = it.in + ((size_t)S.L + mi) * n;
      for (int e0 = threadIdx.x; e0 < n; e0 += KB * NT) {
        u64 cw[KB];
#pragma unroll
        for (int c = 0; c < KB; c++) {
          const int e = e0 + c * NT;
          cw[c] = gld(c1 + galois_index((u32)(e < n ? e : e0), it.galois, logn));
        }
        accumulate(0, n, e0, [&](int c, int) { return u2d(cw[c]); });
      }
    } else {
      const u64* Dj = D + ((size_t)b * S.L + lo) * n;
      const int na = hi - lo;
      auto seg = [&](int base, int cnt) {
        for (int e0 = threadIdx.x; e0 < cnt; e0 += KB * NT) accumulate(base, cnt, e0, [&](int, int e) { return smem[lpad(e)]; });
      };
      if (na == 1) {
        // one source prime (alpha = 1): [x]_q as an integer, taken mod mi
        xf.fwd_seg([=](int i) { return reduce(u2d(Dj[i]), m); }, seg, smem, tw, twc, m, tid);
      } else {
        // fast basis conversion from the digit's primes to modulus mi
        const double2* cinv = up_inv + j * S.alpha;
        const double2* chat = up_hat + (size_t)j * S.alpha * LK + mi;
        auto src = [=](int i) {
          double acc = 0.0;
          for (int a = 0; a < na; a++) {
            const ModTab sa = tab[lo + a];
            const ModD ms = mod_of(sa);
            const double y = canon(mul_tw(u2d(Dj[(size_t)a * n + i]), cinv[a].x, cinv[a].y, ms), ms);
            const double2 hm = chat[(size_t)a * LK];
            acc = reduce(acc + mul_tw(y, hm.x, hm.y, m), m);
          }
          return acc;
        };
        xf.fwd_seg(src, seg, smem, tw, twc, m, tid);
      }
    }
    __syncthreads();
  }
}

// k_modup_ip at N = 2^14 with the accumulators in registers.  One workgroup per (part h of the
// output, target modulus mi), item b and digit group dg, PARTS = 2 (halves, 512 threads) or 1
// (the whole limb, 1024 threads); thread t owns the element pairs h P + 2t + 2 NT k + {0, 1}
// (k < 8, P = N / PARTS) of both accumulators through all digits of the group and writes them
// once, after the last digit, where k_modup_ip reads and writes them in memory for every digit.
// A digit's forward transform: stage 0 pairs e with e + 2^13 (with halves, each half's workgroup
// reads the whole digit and forms its own half, whose stages 1..13 are independent of the other
// half); stages 1..12 as radix-8 rounds through LDS, one task per thread and call; stage 13 pairs
// adjacent elements and runs in registers as the accumulation reads them.  The radix-8 rounds and
// the just-in-time twiddle loads keep the transform's registers beside the 64 that hold the
// accumulators.  LDS: one part (68 KiB, two workgroups per CU; or 136 KiB, one).  The
// accumulators start at zero and every digit's products are added and reduced, so they hold the
// residues of k_modup_ip's accumulators (the first digit's products reduced once more).
template <int PARTS>
__global__ void __launch_bounds__(1024 / PARTS) __attribute__((amdgpu_waves_per_eu(4)))
k_modup_ip_reg(const RotItem* __restrict__ items, const u64* __restrict__ D, double* ACC, KsShape S,
               const double2* __restrict__ up_inv, const double2* __restrict__ up_hat, const ModTab* __restrict__ tab) {
  SMEM();
  constexpr int LOGN = kSplitLogn, NT = 1024 / PARTS, H = 1 << (LOGN - 1), P = (1 << LOGN) / PARTS, EH = P / NT, NP = EH / 2;
  static_assert(EH == 16, "16 elements per thread");
  constexpr int n = 1 << LOGN;
  const int LK = S.L + S.K;
  // XCD-aware order: workgroup g of the grid runs on XCD g % 8, so each XCD takes a contiguous
  // range of the (item, digit group) tasks and the PARTS (L + K) workgroups of a task, which read
  // the same digits, share one L2
  int h, mi, b, dg;
  {
    const int per_task = PARTS * LK;   // == gridDim.x
    const int T = per_task * gridDim.y * gridDim.z;
    const int g = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const int x = g & 7, r = g >> 3, per = T >> 3, rem = T & 7;
    const int l = x < rem ? x * (per + 1) + r : rem * (per + 1) + (x - rem) * per + r;
    const int task = l / per_task, part = l % per_task;
    h = part % PARTS;
    mi = part / PARTS;
    b = task % gridDim.y;
    dg = task / gridDim.y;
  }
  const RotItem it = items[b];
  const ModTab tb = tab[mi];
  const ModD m = mod_of(tb);
  const int j0 = dg * S.dpg, j1 = min(S.dnum, j0 + S.dpg);
  const int hoff = h * P;
  using LT = typename std::conditional<PARTS == 2, LdsHalf<LOGN - 1>, LdsIO>::type;
  const LT Lh{smem};
  double acc0[EH], acc1[EH];   // element 2t + 2 NT k + c of the part at index 2k + c
#pragma unroll
  for (int k = 0; k < EH; k++) acc0[k] = acc1[k] = 0.0;
  for (int j = j0; j < j1; j++) {
    int tid = threadIdx.x;   // recomputed per digit (not held in registers across the loop)
    const double2* tw = tb.fw;
    const double* twc = tb.fwc;
    asm volatile("" : "+v"(tid), "+s"(tw), "+s"(twc));
    const int lo = j * S.alpha, hi = min(S.L, lo + S.alpha);
    const u64* kb = it.key + (((size_t)0 * S.dnum + j) * LK + mi) * n + hoff;
    const u64* ka = it.key + (((size_t)1 * S.dnum + j) * LK + mi) * n + hoff;
    // pair k of the thread: (x0, x1) at elements 2t + 2 NT k + {0, 1} of the part
    auto accumulate = [&](int k, double x0, double x1) {
      const int e = 2 * tid + k * 2 * NT;
      asm volatile("" : "+s"(kb), "+s"(ka));   // one pair's key words in flight at a time
      const u64 b0 = gld(kb + e), b1 = gld(kb + e + 1), a0 = gld(ka + e), a1 = gld(ka + e + 1);
      const double xs[2] = {reduce(x0, m), reduce(x1, m)};
      const u64 wb[2] = {b0, b1}, wa[2] = {a0, a1};
#pragma unroll
      for (int c = 0; c < 2; c++) {
        const double v0 = mulmod(xs[c], u2d(wb[c]), m);
        const double v1 = mulmod(xs[c], u2d(wa[c]), m);
        acc0[2 * k + c] = reduce(v0 + acc0[2 * k + c], m);
        acc1[2 * k + c] = reduce(v1 + acc1[2 * k + c], m);
      }
    };
    if (mi >= lo && mi < hi) {
      // the digit holds modulus mi: its extension is sigma_g(c1)_mi itself (NTT form, gathered)
      const u64* c1 = it.in + ((size_t)S.L + mi) * n;
#pragma unroll
      for (int k = 0; k < NP; k++) {
        const int e = hoff + 2 * tid + k * 2 * NT;
        const double x0 = u2d(gld(c1 + galois_index((u32)e, it.galois, LOGN)));
        const double x1 = u2d(gld(c1 + galois_index((u32)(e + 1), it.galois, LOGN)));
        accumulate(k, x0, x1);
      }
    } else {
      const u64* Dj = D + ((size_t)b * S.L + lo) * n;
      const int na = hi - lo;
      const double2* cinv = up_inv + j * S.alpha;
      const double2* chat = up_hat + (size_t)j * S.alpha * LK + mi;
      auto src = [=](int i) {
        if (na == 1) return reduce(u2d(gld(Dj + i)), m);   // one source prime: [x]_q taken mod mi
        double acc = 0.0;                                   // fast basis conversion D_j -> mi
        for (int a = 0; a < na; a++) {
          const ModTab sa = tab[lo + a];
          const ModD ms = mod_of(sa);
          const double y = canon(mul_tw(u2d(gld(Dj + (size_t)a * n + i)), cinv[a].x, cinv[a].y, ms), ms);
          const double2 hm = chat[(size_t)a * LK];
          acc = reduce(acc + mul_tw(y, hm.x, hm.y, m), m);
        }
        return acc;
      };
      // stage 0 (this part only), into LDS a few elements at a time
      const double2 w1 = ldtw(tw, 1);
      if constexpr (PARTS == 2) {
#pragma unroll 4
        for (int k = 0; k < EH; k++) {
          const int e = tid + k * NT;
          const double x0 = src(e), t = mul_tw(src(e + H), w1.x, w1.y, m);
          smem[lpad(e)] = h ? x0 - t : x0 + t;
        }
      } else {
#pragma unroll 4
        for (int k = 0; k < EH / 2; k++) {
          const int e = tid + k * NT;
          const double x0 = src(e), t = mul_tw(src(e + H), w1.x, w1.y, m);
          smem[lpad(e)] = x0 + t;
          smem[lpad(e + H)] = x0 - t;
        }
      }
      __syncthreads();
      // stages 1..12: four radix-8 rounds, the part's P / 8 tasks of each as two calls of one task
      // per thread; the opaque twiddle base keeps a call's twiddle loads from being hoisted into
      // the previous one
#define HS_R8(ST0)                                                                     \
  fwd_round_gc<LOGN, NT, ST0, 3, 1>(Lh, Lh, twc, m, h * (P / 8), tid);                  \
  asm volatile("" : "+s"(twc));                                                         \
  fwd_round_gc<LOGN, NT, ST0, 3, 1>(Lh, Lh, twc, m, h * (P / 8) + NT, tid);             \
  asm volatile("" : "+s"(twc));                                                         \
  __syncthreads();
      HS_R8(1) HS_R8(4) HS_R8(7) HS_R8(10)
#undef HS_R8
      // stage 13 (pairs e, e + 1; twiddle 2^13 + e / 2 of the whole limb) and the accumulation
#pragma unroll
      for (int k = 0; k < NP; k++) {
        const int e = 2 * tid + k * 2 * NT;
        const double w = gld(twc + (1 << 13) + ((hoff + e) >> 1));
        const double x0 = smem[lpad(e)], t = mul_twc(smem[lpad(e + 1)], w, m);
        accumulate(k, x0 + t, x0 - t);
      }
      __syncthreads();   // the next digit's stage 0 overwrites LDS
    }
  }
  double* o0 = ACC + ((((size_t)b * S.ndg + dg) * 2 + 0) * LK + mi) * n + hoff;
  double* o1 = ACC + ((((size_t)b * S.ndg + dg) * 2 + 1) * LK + mi) * n + hoff;
#pragma unroll
  for (int k = 0; k < NP; k++) {
    const int e = 2 * threadIdx.x + k * 2 * NT;
    gst(o0 + e, acc0[2 * k]);
    gst(o0 + e + 1, acc0[2 * k + 1]);
    gst(o1 + e, acc1[2 * k]);
    gst(o1 + e + 1, acc1[2 * k + 1]);
  }
}

HS_XF_KERNEL k_moddown_intt(const double* __restrict__ ACC, double* PC, KsShape S, const ModTab* __restrict__ tab, int logn, XF xf) {
  SMEM();
  const int n = 1 << logn;
  const int k = blockIdx.x, w = blockIdx.y, b = blockIdx.z;
  const int LK = S.L + S.K;
  const int mi = S.L + k;
  const ModTab tb = tab[mi];
  const ModD m = mod_of(tb);
  const int ndg = S.ndg;
  const double* a0 = ACC + (((size_t)b * ndg * 2 + w) * LK + mi) * n;
  const size_t dstride = (size_t)2 * LK * n;
  double* o = PC + (((size_t)b * 2 + w) * S.K + k) * n;
  auto in = [a0, dstride, ndg, m](int i) {
    double acc = 0.0;
    for (int dg = 0; dg < ndg; dg++) acc += a0[dg * dstride + i];
    return canon(acc, m);
  };
  auto sink = [o, m](int i, double x) { o[i] = canon(x, m); };
  xf.inv(in, sink, smem, tb.iv, tb.ninv, m);
}

HS_XF_KERNEL k_moddown_ntt(const RotItem* __restrict__ items, const double* __restrict__ ACC, const double* __restrict__ PC, KsShape S,
                           const double2* __restrict__ dn_inv, const double2* __restrict__ dn_hat, const double2* __restrict__ pinv,
                           const ModTab* __restrict__ tab, int logn, XF xf) {
  SMEM();
  const int n = 1 << logn;
  const int i_l = blockIdx.x, w = blockIdx.y, b = blockIdx.z;
  const int LK = S.L + S.K;
  const RotItem it = items[b];
  const ModTab tb = tab[i_l];
  const ModD m = mod_of(tb);
  const double* pc = PC + ((size_t)b * 2 + w) * S.K * n;
  const int K = S.K;
  auto src = [=](int i) {
    double acc = 0.0;
    for (int k = 0; k < K; k++) {
      const double x = pc[(size_t)k * n + i];
      if (K == 1) {
        acc = x;  // [x]_p as an integer in [0, p), taken mod q_i
      } else {
        const ModTab sp = tab[S.L + k];
        const ModD ms = mod_of(sp);
        const double2 ci = dn_inv[k];
        const double y = canon(mul_tw(x, ci.x, ci.y, ms), ms);
        const double2 hm = dn_hat[(size_t)k * S.L + i_l];
        acc = reduce(acc + mul_tw(y, hm.x, hm.y, m), m);
      }
    }
    return reduce(acc, m);
  };
  const double2 pv = pinv[i_l];
  const u64* c0 = it.in + (size_t)i_l * n;
  const u32 gal = it.galois;
  u64* out = it.out + ((size_t)w * S.L + i_l) * n;
  const u64* add = it.addend ? it.addend + ((size_t)w * S.L + i_l) * n : nullptr;
  const int ndg = S.ndg;
  const double* a0 = ACC + (((size_t)b * ndg * 2 + w) * LK + i_l) * n;
  const size_t dstride = (size_t)2 * LK * n;
  // the epilogue's loads (accumulators, sigma_g(c0), addend) KB elements at a time, all in
  // flight together, with branch-free addresses (unused words are read and ignored)
  constexpr int KB = KsBatch<XF>::value;
  auto seg = [&](int base, int cnt) {
    for (int e0 = threadIdx.x; e0 < cnt; e0 += KB * XF::NT) {
      double ac[KB];
      u64 cw[KB], aw[KB];
#pragma unroll
      for (int c = 0; c < KB; c++) {
        const int e = e0 + c * XF::NT;
        const int i = base + (e < cnt ? e : e0);
        double acc = 0.0;
        for (int dg = 0; dg < ndg; dg++) acc += gld(a0 + dg * dstride + i);
        ac[c] = acc;
        const u64* cp = c0 + galois_index((u32)i, gal, logn);
        cw[c] = gld(cp);
        aw[c] = gld(add ? add + i : cp);
      }
#pragma unroll
      for (int c = 0; c < KB; c++) {
        const int e = e0 + c * XF::NT;
        if (e < cnt) {
          double v = mul_tw(reduce(ac[c] - smem[lpad(e)], m), pv.x, pv.y, m);
          if (w == 0) v += u2d(cw[c]);
          if (add) v += u2d(aw[c]);
          gst(out + base + e, d2u(canon(v, m)));
        }
      }
    }
  };
  xf.fwd_seg(src, seg, smem, tb.fw, tb.fwc, m);
}

// ------------------------------------------------------------------ decryption
// phase x = c0 + c1 s in coefficient form, per limb: X[g][l][N] (u64).  grid = (L, n_ct).
HS_XF_KERNEL k_dec_phase(const u64* __restrict__ ct, const u64* __restrict__ sk, u64* X, int L, const ModTab* __restrict__ tab, int logn, XF xf) {
  SMEM();
  const int n = 1 << logn;
  const int l = blockIdx.x, g = blockIdx.y;
  const ModTab tb = tab[l];
  const ModD m = mod_of(tb);
  const u64* c0 = ct + ((size_t)g * 2 * L + l) * n;
  const u64* c1 = ct + ((size_t)g * 2 * L + L + l) * n;
  const u64* sl = sk + (size_t)l * n;
  u64* o = X + ((size_t)g * L + l) * n;
  auto in = [=](int i) { return canon(u2d(c0[i]) + mulmod(u2d(c1[i]), u2d(sl[i]), m), m); };
  auto sink = [o, m](int i, double x) { o[i] = d2u(canon(x, m)); };
  xf.inv(in, sink, smem, tb.iv, tb.ninv, m);
}

// m = round(t x / Q) mod t from the residues x_i (exact):  with y_i = [x_i Qhat_i^-1]_{q_i},
// t y_i = a_i q_i + r_i, round(t x / Q) = sum a_i + round(sum_i r_i Qhat_i / Q) (mod t).
// WT > 0: the word count of Q as a compile-time constant (the multiword arrays stay in registers
// and every word loop unrolls); WT = 0: runtime W <= 16.
template <int WT>
__global__ void k_dec_round(const u64* __restrict__ X, u64* M, int n_ct, int L, u64 t, const double2* __restrict__ dinv,
                            const u64* __restrict__ dhat, const u64* __restrict__ dq, int W_, const ModTab* __restrict__ tab, int logn) {
  constexpr int WA = WT > 0 ? WT : 16;
  const int W = WT > 0 ? WT : W_;
  const int n = 1 << logn;
  const int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n_ct * n) return;
  const int g = gid >> logn, k = gid & (n - 1);
  u64 S[WA];
  for (int w = 0; w < W; w++) S[w] = 0;
  u64 asum = 0;
  for (int i = 0; i < L; i++) {
    const ModTab tb = tab[i];
    const ModD m = mod_of(tb);
    const u64 q = (u64)tb.q;
    const double x = u2d(X[((size_t)g * L + i) * n + k]);
    const u64 y = d2u(canon(mul_tw(x, dinv[i].x, dinv[i].y, m), m));
    // t*y = a*q + r, 0 <= r < q: estimate a in floating point, fix with exact 64-bit wrap-around
    u64 a = (u64)((double)y * ((double)t / (double)q));
    i64 r = (i64)(t * y - a * q);
    while (r < 0) { r += (i64)q; a--; }
    while (r >= (i64)q) { r -= (i64)q; a++; }
    asum += a;
    // S += r * Qhat_i
    u64 carry = 0;
    for (int w = 0; w < W; w++) {
      const u64 h = dhat[(size_t)i * W + w];
      const u64 lo = h * (u64)r;
      const u64 hi = __umul64hi(h, (u64)r);
      u64 s1 = S[w] + lo;
      u64 c1 = s1 < lo;
      u64 s2 = s1 + carry;
      u64 c2 = s2 < carry;
      S[w] = s2;
      carry = hi + c1 + c2;
    }
  }
  // T = 2 S + Q; kq = floor(T / 2Q) by repeated subtraction (kq <= L)
  u64 T[WA], twoq[WA];
  {
    u64 sh = 0, cadd = 0, shq = 0;
    for (int w = 0; w < W; w++) {
      const u64 s2 = (S[w] << 1) | sh;
      sh = S[w] >> 63;
      const u64 v = s2 + dq[w];
      const u64 c1 = v < s2;
      const u64 v2 = v + cadd;
      const u64 c2 = v2 < cadd;
      T[w] = v2;
      cadd = c1 + c2;
      twoq[w] = (dq[w] << 1) | shq;
      shq = dq[w] >> 63;
    }
  }
  u64 kq = 0;
  for (int guard = 0; guard <= L + 1; guard++) {
    bool ge = true;
    for (int w = W - 1; w >= 0; w--) {
      if (T[w] != twoq[w]) { ge = T[w] > twoq[w]; break; }
    }
    if (!ge) break;
    u64 br = 0;
    for (int w = 0; w < W; w++) {
      const u64 a = T[w], bq = twoq[w];
      const u64 d = a - bq;
      const u64 b1 = a < bq;
      const u64 d2 = d - br;
      const u64 b2 = d < br;
      T[w] = d2;
      br = b1 | b2;
    }
    kq++;
  }
  // asum + kq < (L + 2) t: a 32-bit remainder when that stays below 2^32 (t < 2^26, L < 62)
  M[gid] = (t < (1ull << 26) && L < 62) ? (u64)((u32)(asum + kq) % (u32)t) : (asum + kq) % t;
}

// Decode (forward mod-t NTT), take slot p for the sorted rows of partition P, scatter with the row
// map.  One workgroup per partition.
template <int NT>
__global__ void __launch_bounds__(NT) k_decode_scatter(const u64* __restrict__ M, const u32* __restrict__ slot_pos, const int* __restrict__ rm,
                                                       const i64* __restrict__ pinfo, i64* y, int tmod, const ModTab* __restrict__ tab, int logn) {
  SMEM();
  const int n = 1 << logn;
  const int P = blockIdx.x;
  const ModTab tb = tab[tmod];
  const ModD m = mod_of(tb);
  const i64 t = (i64)tb.q;
  // pinfo per partition: (row0, rows, nonzero rows, row-map offset, group, slot offset)
  const i64* pi = pinfo + 6 * P;
  const i64 row0 = pi[0], rows = pi[1], nz = pi[2], rm0 = pi[3], grp = pi[4], off = pi[5];
  const u64* mc = M + (size_t)grp * n;
  for (int i = threadIdx.x; i < n; i += NT) smem[lpad(i)] = u2d(mc[i]);
  __syncthreads();
  lds_ntt_fwd<NT>(smem, logn, tb.fw, m);
  for (i64 p = threadIdx.x; p < rows; p += NT) {
    i64 v = 0;
    if (p < nz) {
      v = (i64)d2u(canon(smem[lpad(slot_pos[off + p])], m));
      if (v > t / 2) v -= t;
    }
    y[row0 + rm[rm0 + p]] = v;
  }
}

// ------------------------------------------------------------------ CSSC scatter (App. B)
// Row r (global) of partition P = r / s goes to sorted position rank[r]; its j-th nonzero lands at
// CSSC entry cp[P][j] + rank[r] of that partition.
__global__ void k_cssc_scatter(const i64* __restrict__ row_ptr, const int* __restrict__ col, const i64* __restrict__ val,
                               const int* __restrict__ rank, const i64* __restrict__ cp, const i64* __restrict__ part_cp_off,
                               const i64* __restrict__ part_nnz_off, i64 R, i64 s, i64* va, int* ci) {
  const i64 r = blockIdx.x * (i64)blockDim.x + threadIdx.x;
  if (r >= R) return;
  const i64 P = r / s;
  const i64 k0 = row_ptr[r], k1 = row_ptr[r + 1];
  const i64 cpo = part_cp_off[P], nzo = part_nnz_off[P];
  for (i64 k = k0; k < k1; k++) {
    const i64 pos = nzo + cp[cpo + (k - k0)] + rank[r];
    va[pos] = val[k];
    ci[pos] = col[k];
  }
}

// CSR validation: col in [0, C) and strictly ascending within each row; sets *bad on violation.
__global__ void k_csr_check(const i64* __restrict__ row_ptr, const int* __restrict__ col, i64 R, i64 C, int* bad) {
  const i64 r = blockIdx.x * (i64)blockDim.x + threadIdx.x;
  if (r >= R) return;
  const i64 k0 = row_ptr[r], k1 = row_ptr[r + 1];
  int prev = -1;
  for (i64 k = k0; k < k1; k++) {
    const int c = col[k];
    if (c < 0 || c >= C || c <= prev) { atomicOr(bad, 1); return; }
    prev = c;
  }
}

// ------------------------------------------------------------------ host launchers
static int nt_for(int logn) { return logn >= 14 ? 1024 : (logn <= 10 ? 64 : (1 << (logn - 4))); }
static size_t lds_bytes(int logn) { return (size_t)lds_doubles(1 << logn) * sizeof(double); }

// Dynamic LDS above the default limit needs the attribute once per kernel instantiation.
static std::mutex g_attr_mu;
static std::map<const void*, size_t> g_attr_set;
static void ensure_lds(const void* f, size_t bytes) {
  std::lock_guard<std::mutex> g(g_attr_mu);
  auto it = g_attr_set.find(f);
  if (it != g_attr_set.end() && it->second >= bytes) return;
  HS_CHECK_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  g_attr_set[f] = bytes;
}

#define HS_LAUNCH_NT(NTV, KERNEL, GRID, STREAM, ...)                                               \
  case NTV:                                                                                         \
    ensure_lds((const void*)KERNEL<NTV>, _lds);                                                     \
    hipLaunchKernelGGL(KERNEL<NTV>, GRID, dim3(NTV), _lds, STREAM, __VA_ARGS__);                    \
    break;
#define HS_DISPATCH_NT(logn, KERNEL, GRID, STREAM, ...)                                             \
  do {                                                                                              \
    ProfScope _prof(#KERNEL, STREAM);                                                               \
    const size_t _lds = lds_bytes(logn);                                                            \
    if (_lds > 160 * 1024) throw Error{HS_EPARAM, "ring too large for the LDS-resident transform"}; \
    switch (nt_for(logn)) {                                                                         \
      HS_LAUNCH_NT(1024, KERNEL, GRID, STREAM, __VA_ARGS__)                                         \
      HS_LAUNCH_NT(512, KERNEL, GRID, STREAM, __VA_ARGS__)                                          \
      HS_LAUNCH_NT(256, KERNEL, GRID, STREAM, __VA_ARGS__)                                          \
      HS_LAUNCH_NT(128, KERNEL, GRID, STREAM, __VA_ARGS__)                                          \
      HS_LAUNCH_NT(64, KERNEL, GRID, STREAM, __VA_ARGS__)                                           \
      default: throw Error{HS_EPARAM, "unsupported ring size"};                                     \
    }                                                                                               \
    HS_CHECK_HIP(hipGetLastError());                                                                \
  } while (0)

static size_t split_lds_bytes() { return (size_t)split_lds_doubles() * sizeof(double); }

#define HS_LAUNCH_XF(XFT, XFV, LDSB, KERNEL, GRID, STREAM, ...)                              \
  do {                                                                                         \
    ensure_lds((const void*)KERNEL<XFT>, LDSB);                                                \
    hipLaunchKernelGGL(KERNEL<XFT>, GRID, dim3(XFT::NT), LDSB, STREAM, __VA_ARGS__, XFV);     \
  } while (0)
// Ring size (and the context's tuned variant) -> transform policy: 2^14 half-limb or whole-limb,
// 2^11..2^13 compile-time (radix 16) or runtime (radix 8), smaller rings runtime with 64 threads.
#define HS_DISPATCH_XF(VARIANT, C, KERNEL, GRID, STREAM, ...)                                            \
  do {                                                                                                   \
    ProfScope _prof(#KERNEL, STREAM);                                                                    \
    const int _logn = (C)->logn;                                                                         \
    const bool _alt = (VARIANT) == 1;                                                                    \
    switch (_logn) {                                                                                     \
      case 14:                                                                                           \
        if (_alt) HS_LAUNCH_XF(XfStatic<1024>, XfStatic<1024>{}, lds_bytes(14), KERNEL, GRID, STREAM, __VA_ARGS__); \
        else HS_LAUNCH_XF(XfSplit, XfSplit{}, split_lds_bytes(), KERNEL, GRID, STREAM, __VA_ARGS__);    \
        break;                                                                                           \
      case 13:                                                                                           \
        if (_alt) HS_LAUNCH_XF(XfRuntime<512>, XfRuntime<512>{13}, lds_bytes(13), KERNEL, GRID, STREAM, __VA_ARGS__); \
        else HS_LAUNCH_XF(XfStatic<512>, XfStatic<512>{}, lds_bytes(13), KERNEL, GRID, STREAM, __VA_ARGS__); \
        break;                                                                                           \
      case 12:                                                                                           \
        if (_alt) HS_LAUNCH_XF(XfRuntime<256>, XfRuntime<256>{12}, lds_bytes(12), KERNEL, GRID, STREAM, __VA_ARGS__); \
        else HS_LAUNCH_XF(XfStatic<256>, XfStatic<256>{}, lds_bytes(12), KERNEL, GRID, STREAM, __VA_ARGS__); \
        break;                                                                                           \
      case 11:                                                                                           \
        if (_alt) HS_LAUNCH_XF(XfRuntime<128>, XfRuntime<128>{11}, lds_bytes(11), KERNEL, GRID, STREAM, __VA_ARGS__); \
        else HS_LAUNCH_XF(XfStatic<128>, XfStatic<128>{}, lds_bytes(11), KERNEL, GRID, STREAM, __VA_ARGS__); \
        break;                                                                                           \
      default:                                                                                           \
        if (_logn < 1 || _logn > 10) throw Error{HS_EPARAM, "ring too large for the LDS-resident transform"}; \
        HS_LAUNCH_XF(XfRuntime<64>, XfRuntime<64>{_logn}, lds_bytes(_logn), KERNEL, GRID, STREAM, __VA_ARGS__); \
    }                                                                                                    \
    HS_CHECK_HIP(hipGetLastError());                                                                     \
  } while (0)

void upload_cdt(const u64* tab20) { HS_CHECK_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_cdt), tab20, 20 * sizeof(u64))); }


static int cu_count(int device) {
  static std::atomic<int> cache[64];
  if (device < 0 || device >= 64) return 256;
  int v = cache[device].load();
  if (!v) {
    HS_CHECK_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, device));
    cache[device] = v;
  }
  return v;
}

void launch_ntt15_rows(const hs_ctx* c, u64* data, i64 nblocks, int nl, int mod0, int inverse, const NttRows& rows, hipStream_t st) {
  if (nblocks <= 0) return;
  HS_REQUIRE(c->logn == kN15Logn, HS_EPARAM, "one-workgroup N = 2^15 transform on another ring");
  HS_REQUIRE(rows.mode == 0 || (rows.per > 0 && (nblocks + rows.per - 1) / rows.per <= kNttRowItems), HS_EPARAM, "row map too large");
  const size_t lds = (size_t)n15_lds_doubles() * sizeof(double);
  ProfUnits units(nblocks);   // limbs per launch, for the profile's roofline
  ProfScope _prof("k_ntt15", st);
  ensure_lds((const void*)k_ntt15, lds);
  hipLaunchKernelGGL(k_ntt15, dim3((unsigned)nblocks), dim3(kN15NT), lds, st, data, nl, mod0, inverse, (const ModTab*)c->d_tab, rows);
  HS_CHECK_HIP(hipGetLastError());
}

void launch_ntt(const hs_ctx* c, u64* data, i64 nblocks, int nl, int mod0, int inverse, hipStream_t st) {
  if (nblocks <= 0) return;
  if (c->logn == kN15Logn) {
    launch_ntt15_rows(c, data, nblocks, nl, mod0, inverse, NttRows{}, st);
    return;
  }
  const i64 grid = 2 * (i64)cu_count(c->device);
  if (c->logn == kSplitLogn && c->xf_variant_ntt == 0 && !inverse && nblocks >= 2 * grid && option(c, HS_OPT_NTT_PIPE) == 0) {
    // enough limbs for every workgroup of the grid to loop over at least two
    ProfScope _prof("k_ntt_fwd_pipe", st);
    ensure_lds((const void*)k_ntt_fwd_pipe, split_lds_bytes());
    hipLaunchKernelGGL(k_ntt_fwd_pipe, dim3((unsigned)grid), dim3(kSplitNT), split_lds_bytes(), st, data, nblocks, nl, mod0,
                       (const ModTab*)c->d_tab);
    HS_CHECK_HIP(hipGetLastError());
    return;
  }
  HS_DISPATCH_XF(c->xf_variant_ntt, c, k_ntt, dim3((unsigned)nblocks), st, data, nl, mod0, inverse, (const ModTab*)c->d_tab, c->logn);
}

void launch_sample_small(const hs_ctx* c, int* out, int nobj, i64 obj_stride, u64 seed, u32 purpose, u64 index0, u64 index_step,
                         int kind, hipStream_t st) {
  if (nobj <= 0) return;
  const int per = kind == 0 ? 16 : 8;
  const i64 threads = (i64)nobj * (c->N / per);
  ProfScope _prof("k_sample_small", st);
  hipLaunchKernelGGL(k_sample_small, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, out, nobj, obj_stride, seed, purpose, index0, index_step, kind, c->logn);
  HS_CHECK_HIP(hipGetLastError());
}

void launch_sample_enc(const hs_ctx* c, int* out, int nobj, u64 seed, u32 pu, u32 pe0, u32 pe1, hipStream_t st) {
  if (nobj <= 0) return;
  const i64 threads = (i64)nobj * (c->N / 8);   // the Gaussian polynomials' blocks (the ternary one has half)
  ProfScope _prof("k_sample_enc", st);
  hipLaunchKernelGGL(k_sample_enc, dim3((unsigned)((threads + 255) / 256), 3), dim3(256), 0, st, out, nobj, seed, pu, pe0, pe1, c->logn);
  HS_CHECK_HIP(hipGetLastError());
}

void launch_enc_ntt(const hs_ctx* c, const u64* mcoef, const int* samples, int n_ct, u64* prep, hipStream_t st) {
  if (n_ct <= 0) return;
  HS_DISPATCH_XF(c->xf_variant_ntt, c, k_enc_ntt, dim3((unsigned)(n_ct * 3 * c->L)), st, mcoef, samples, prep, c->L, c->t, c->q_mod_t,
                 (const double2*)c->d_qdt, (const ModTab*)c->d_tab, c->logn);
}

void launch_sk_ntt(const hs_ctx* c, u64* sk, const int* s_coef, hipStream_t st) {
  HS_DISPATCH_NT(c->logn, k_sk_ntt, dim3(c->n_mod), st, sk, s_coef, (const ModTab*)c->d_tab, c->logn);
}

void launch_ksk_limbs(const hs_ctx* c, const KskArgs* d_args, int count, hipStream_t st) {
  if (count <= 0) return;
  HS_DISPATCH_NT(c->logn, k_ksk_limb, dim3(count), st, d_args, (const ModTab*)c->d_tab, c->logn);
}

void launch_pack_encode(const hs_ctx* c, const PackArgs& a, int nchunks, hipStream_t st) {
  if (nchunks <= 0) return;
  HS_DISPATCH_NT(c->logn, k_pack_encode, dim3(nchunks), st, a, (const u32*)c->d_slot_pos, (const ModTab*)c->d_tab, c->n_mod, c->logn);
}

void launch_plain_ntt(const hs_ctx* c, const u64* coef, u64* out, int n_plain, hipStream_t st) {
  if (n_plain <= 0) return;
  HS_DISPATCH_XF(c->xf_variant_ntt, c, k_plain_ntt, dim3(c->L, n_plain), st, coef, out, c->L, c->t, (const ModTab*)c->d_tab, c->logn);
}

void launch_encrypt(const hs_ctx* c, const u64* mcoef, const int* samples, const u64* pk, u64* out, int n_ct, hipStream_t st) {
  if (n_ct <= 0) return;
  HS_DISPATCH_NT(c->logn, k_encrypt, dim3(c->L, n_ct), st, mcoef, samples, pk, out, c->L, c->t, c->q_mod_t,
                 (const double2*)c->d_qdt, (const ModTab*)c->d_tab, c->logn);
}

void launch_mul_plain(const hs_ctx* c, const u64* x, const u64* pt, u64* out, i64 n_ct, int pt_stride_ct, hipStream_t st) {
  if (n_ct <= 0) return;
  const i64 rows = n_ct * 2 * c->L;
  const dim3 grid((unsigned)std::max<i64>(1, ((i64)c->N + 256 * EW_EPT - 1) / (256 * EW_EPT)), (unsigned)std::min<i64>(rows, 65535));
  ProfScope _prof("k_mul_plain", st);
  hipLaunchKernelGGL(k_mul_plain, grid, dim3(256), 0, st, x, pt, out, n_ct, c->L, pt_stride_ct, (const ModTab*)c->d_tab, c->logn);
  HS_CHECK_HIP(hipGetLastError());
}

void launch_mask_acc(const hs_ctx* c, const u64* const* w, const u64* mask, const int* part_chunk0, const int* part_nchunks,
                     u64* res, int nparts, hipStream_t st) {
  if (nparts <= 0) return;
  const dim3 grid((unsigned)std::max<i64>(1, ((i64)c->N + 255) / 256), (unsigned)(2 * c->L), (unsigned)nparts);
  ProfScope _prof("k_mask_acc", st);
  hipLaunchKernelGGL(k_mask_acc, grid, dim3(256), 0, st, w, mask, part_chunk0, part_nchunks, res, c->L, (const ModTab*)c->d_tab, c->logn);
  HS_CHECK_HIP(hipGetLastError());
}

void launch_rotate_batch(const hs_ctx* c, const RotItem* d_items, int B, const KsShape& S, u64* D, double* ACC, double* PC, hipStream_t st) {
  if (B <= 0) return;
  ProfUnits units(B);
  const ModTab* tab = (const ModTab*)c->d_tab;
  HS_DISPATCH_XF(c->xf_variant, c, k_rot_intt, dim3(c->L, B), st, d_items, D, c->L, tab, c->logn);
  // register accumulators: whole limbs (one workgroup per CU) from 64 items per level on, halves
  // (two per CU) below: measured 0.66 vs 0.68 ms at 128 items, 1.21 vs 1.29 at 256, 0.19 vs
  // 0.18 at 32
  const int acc_opt = option(c, HS_OPT_MODUP_ACC);
  if (c->logn == kSplitLogn && (acc_opt == 3 || (acc_opt == 0 && B >= 64))) {
    ProfScope _prof("k_modup_ip_reg", st);
    ensure_lds((const void*)k_modup_ip_reg<1>, lds_bytes(14));
    hipLaunchKernelGGL(k_modup_ip_reg<1>, dim3(c->L + c->K, B, S.ndg), dim3(1024), lds_bytes(14), st, d_items, (const u64*)D, ACC, S,
                       (const double2*)c->d_up_inv, (const double2*)c->d_up_hat, tab);
    HS_CHECK_HIP(hipGetLastError());
  } else if (c->logn == kSplitLogn && acc_opt != 1) {
    ProfScope _prof("k_modup_ip_reg", st);
    ensure_lds((const void*)k_modup_ip_reg<2>, split_lds_bytes());
    hipLaunchKernelGGL(k_modup_ip_reg<2>, dim3(2 * (c->L + c->K), B, S.ndg), dim3(kSplitNT), split_lds_bytes(), st, d_items, (const u64*)D,
                       ACC, S, (const double2*)c->d_up_inv, (const double2*)c->d_up_hat, tab);
    HS_CHECK_HIP(hipGetLastError());
  } else {
    HS_DISPATCH_XF(c->xf_variant, c, k_modup_ip, dim3(c->L + c->K, B, S.ndg), st, d_items, (const u64*)D, ACC, S,
                   (const double2*)c->d_up_inv, (const double2*)c->d_up_hat, tab, c->logn);
  }
  HS_DISPATCH_XF(c->xf_variant, c, k_moddown_intt, dim3(c->K, 2, B), st, (const double*)ACC, PC, S, tab, c->logn);
  HS_DISPATCH_XF(c->xf_variant, c, k_moddown_ntt, dim3(c->L, 2, B), st, d_items, (const double*)ACC, (const double*)PC, S,
                 (const double2*)c->d_dn_inv, (const double2*)c->d_dn_hat, (const double2*)c->d_pinv, tab, c->logn);
}

void launch_dec_phase(const hs_ctx* c, const u64* ct, const u64* sk, u64* X, int n_ct, hipStream_t st) {
  if (n_ct <= 0) return;
  HS_DISPATCH_XF(c->xf_variant_ntt, c, k_dec_phase, dim3(c->L, n_ct), st, ct, sk, X, c->L, (const ModTab*)c->d_tab, c->logn);
}

void launch_dec_round(const hs_ctx* c, const u64* X, u64* M, int n_ct, hipStream_t st) {
  if (n_ct <= 0) return;
  const i64 total = (i64)n_ct * c->N;
  ProfScope _prof("k_dec_round", st);
  const dim3 grid((unsigned)((total + 255) / 256));
#define HS_DEC_ROUND(WT)                                                                                          \
  hipLaunchKernelGGL(k_dec_round<WT>, grid, dim3(256), 0, st, X, M, n_ct, c->L, c->t, (const double2*)c->d_dec_inv, \
                     (const u64*)c->d_dec_hat, (const u64*)c->d_dec_q, c->dec_words, (const ModTab*)c->d_tab, c->logn)
  switch (c->dec_words) {
    case 2: HS_DEC_ROUND(2); break;
    case 3: HS_DEC_ROUND(3); break;
    case 4: HS_DEC_ROUND(4); break;
    case 5: HS_DEC_ROUND(5); break;
    case 6: HS_DEC_ROUND(6); break;
    case 7: HS_DEC_ROUND(7); break;
    case 8: HS_DEC_ROUND(8); break;
    case 9: HS_DEC_ROUND(9); break;
    case 10: HS_DEC_ROUND(10); break;
    case 11: HS_DEC_ROUND(11); break;
    default:
      HS_REQUIRE(c->dec_words <= 16, HS_EPARAM, "ciphertext modulus too wide for decryption");
      HS_DEC_ROUND(0);
  }
#undef HS_DEC_ROUND
  HS_CHECK_HIP(hipGetLastError());
}

void launch_decode_scatter(const hs_ctx* c, const u64* M, const int* rm, const i64* pinfo, i64* y, int nparts, hipStream_t st) {
  if (nparts <= 0) return;
  HS_DISPATCH_NT(c->logn, k_decode_scatter, dim3(nparts), st, M, (const u32*)c->d_slot_pos, rm, pinfo, y, c->n_mod,
                 (const ModTab*)c->d_tab, c->logn);
}

void launch_cssc_scatter(const i64* row_ptr, const int* col, const i64* val, const int* rank, const i64* cp, const i64* part_cp_off,
                         const i64* part_nnz_off, i64 R, i64 s, i64* va, int* ci, hipStream_t st) {
  if (R <= 0) return;
  ProfScope _prof("k_cssc_scatter", st);
  hipLaunchKernelGGL(k_cssc_scatter, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, st, row_ptr, col, val, rank, cp, part_cp_off,
                     part_nnz_off, R, s, va, ci);
  HS_CHECK_HIP(hipGetLastError());
}

void launch_csr_check(const i64* row_ptr, const int* col, i64 R, i64 C, int* bad, hipStream_t st) {
  if (R <= 0) return;
  ProfScope _prof("k_csr_check", st);
  hipLaunchKernelGGL(k_csr_check, dim3((unsigned)((R + 255) / 256)), dim3(256), 0, st, row_ptr, col, R, C, bad);
  HS_CHECK_HIP(hipGetLastError());
}

}  // namespace hs
