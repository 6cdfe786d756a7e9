// Two-pass key switching and two-pass NTT kernels (multi-workgroup transforms, hs_pass.hpp).
//
// One batched power-of-two rotation level runs as five kernels; every workgroup owns one block of
// BE elements of one limb, so a level has (limbs x blocks x items) workgroups:
//  K1 k2_rot_intt_low   sigma_g(c1) (NTT-domain gather), inverse low pass            -> T1
//  K2 k2_modup_high     inverse high pass (coefficients), ModUp conversion of the digit to every
//                       other modulus, forward high pass                              -> E
//  K3 k2_ip_low         forward low pass of each digit's extension (own limb: sigma_g(c1)), key
//                       inner product over the digits; special limbs also get the inverse low pass
//                                                                                     -> ACC, T2
//  K4 k2_moddown_high   inverse high pass of the special limbs, conversion P -> q_i, forward high
//                       pass                                                          -> F
//  K5 k2_final_low      forward low pass, out = (ACC - F) P^-1 + sigma_g(c0) (+ addend); where the
//                       output is the next level's input, also the next level's K1 for it
//                       (the Galois permutation of NTT slots maps every contiguous block onto
//                       one block, so the block this workgroup holds is exactly the source of
//                       one block of the next gather)
// Intermediates are balanced doubles in HBM (mostly served from the 256 MB Infinity Cache).
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <type_traits>

#include "hs_pass.hpp"
#include "kernels.hpp"

namespace hs {

#define SMEM() extern __shared__ double smem_raw[]
// LDS layout of every two-pass kernel: [staged twiddles: BE double2][data buffers of lds_doubles(BE)]
#define SMEM2_N(G, TWN)                           \
  SMEM();                                         \
  double2* twl = (double2*)smem_raw;              \
  double* smem = smem_raw + 2 * (TWN)
#define SMEM2(G) SMEM2_N(G, (G).BE)

__device__ __forceinline__ ModD mod_of2(const ModTab& t) { return ModD{t.q, t.qinv}; }

__device__ __forceinline__ u32 galois_index2(u32 k, u32 g, int logn) {
  const u32 n2m = (2u << logn) - 1;
  const u32 e = 2 * brev_bits(k, logn) + 1;
  const u32 e2 = (u32)(((u64)g * e) & n2m);
  return brev_bits((e2 - 1) >> 1, logn);
}

// ------------------------------------------------------------------ standalone two-pass NTT
// One pass over `nl`-limb polynomials: grid (nblk, n_polys * nl).  in/out either u64 canonical
// residues or balanced doubles (in place allowed).
template <int NT, bool HIGH, bool FWD, class GT>
__device__ __forceinline__ void ntt_pass_body(double* smem, double2* twl, const void* in, int in_u64, void* out, int out_u64, int nl, int mod0,
                                              int scale, const ModTab* __restrict__ tab, GT G) {
  constexpr int PER = (GT::kMaxBE + NT - 1) / NT;
  const int n = 1 << G.logn;
  const int blk = blockIdx.x, row = blockIdx.y;
  const ModTab tb = tab[mod0 + row % nl];
  const ModD m = mod_of2(tb);
  const size_t base = (size_t)row * n;
  // every global load first (twiddles and the block), then the LDS stores
  TwPre<NT, HIGH, FWD, GT> tw;
  tw.load(G, blk, FWD ? tb.fw : tb.iv);
  double x[PER];
#pragma unroll
  for (int r = 0; r < PER; r++) {
    const int e = threadIdx.x + r * NT;
    if (e < G.BE) {
      const int gi = gidx_of_lds<HIGH>(G, blk, e);
      x[r] = in_u64 ? u2d(gld((const u64*)in + base + gi)) : gld((const double*)in + base + gi);
    }
  }
  tw.store(twl, G);
#pragma unroll
  for (int r = 0; r < PER; r++) {
    const int e = threadIdx.x + r * NT;
    if (e < G.BE) smem[lpadx<HIGH>(e)] = x[r];
  }
  __syncthreads();
  if (FWD) pass_fwd<NT, HIGH>(smem, twl, G, blk, tb.fw, m, false);
  else pass_inv<NT, HIGH>(smem, twl, G, blk, scale != 0, tb.iv, tb.ninv, m, false);
  for (int e = threadIdx.x; e < G.BE; e += NT) {
    const int gi = gidx_of_lds<HIGH>(G, blk, e);
    if (out_u64) gst((u64*)out + base + gi, d2u(canon(smem[lpadx<HIGH>(e)], m)));
    else gst((double*)out + base + gi, smem[lpadx<HIGH>(e)]);
  }
}

#define HS2_PASS_KERNEL(NAME, HIGH, FWD)                                                                      \
  template <int NT, class GT>                                                                                         \
  __global__ void __launch_bounds__(NT) NAME(const void* in, int in_u64, void* out, int out_u64, int nl,      \
                                             int mod0, int scale, const ModTab* __restrict__ tab, GT G) { \
    SMEM2(G);                                                                                                 \
    ntt_pass_body<NT, HIGH, FWD, GT>(smem, twl, in, in_u64, out, out_u64, nl, mod0, scale, tab, G);               \
  }
HS2_PASS_KERNEL(k2_ntt_pass_hf, true, true)
HS2_PASS_KERNEL(k2_ntt_pass_lf, false, true)
HS2_PASS_KERNEL(k2_ntt_pass_li, false, false)
HS2_PASS_KERNEL(k2_ntt_pass_hi, true, false)

// ------------------------------------------------------------------ key switching, K1..K5
template <int NT, class GT>
__global__ void __launch_bounds__(NT) k2_rot_intt_low(const RotItem* __restrict__ items, double* T1, int L, const ModTab* __restrict__ tab, GT G) {
  SMEM2(G);
  constexpr int PER = (GT::kMaxBE + NT - 1) / NT;
  const int n = 1 << G.logn;
  const int blk = blockIdx.x, l = blockIdx.y, b = blockIdx.z;
  const RotItem it = items[b];
  const ModTab tb = tab[l];
  const ModD m = mod_of2(tb);
  // every global load first (twiddles and the gathered block), then the LDS stores
  TwPre<NT, false, false, GT> tw;
  tw.load(G, blk, tb.iv);
  const u64* c1 = it.in + ((size_t)L + l) * n;
  u64 x[PER];
#pragma unroll
  for (int r = 0; r < PER; r++) {
    const int e = threadIdx.x + r * NT;
    if (e < G.BE) x[r] = gld(c1 + galois_index2((u32)gidx_of_lds<false>(G, blk, e), it.galois, G.logn));
  }
  tw.store(twl, G);
#pragma unroll
  for (int r = 0; r < PER; r++) {
    const int e = threadIdx.x + r * NT;
    if (e < G.BE) smem[lpad(e)] = u2d(x[r]);
  }
  __syncthreads();
  pass_inv<NT, false>(smem, twl, G, blk, false, tb.iv, tb.ninv, m, false);
  double* o = T1 + ((size_t)b * L + l) * n;
  for (int e = threadIdx.x; e < G.BE; e += NT) gst(o + gidx_of_lds<false>(G, blk, e), smem[lpad(e)]);
}

// grid (nblk, dnum * (L + K), B): digit j = y / (L+K), target modulus mi = y % (L+K) (own limbs of
// the digit exit at once).  The digit's inverse high pass is recomputed by each target's
// workgroup: two passes per workgroup instead of a chain of L + K.
template <int NT, class GT>
__global__ void __launch_bounds__(NT) k2_modup_high(const double* __restrict__ T1, double* E, KsShape S, const double2* __restrict__ up_inv,
                                                    const double2* __restrict__ up_hat, const ModTab* __restrict__ tab, GT G) {
  SMEM();
  constexpr int AMAX = 4;  // source primes per digit whose twiddles are prefetched (more: staged late)
  constexpr int PER = (GT::kMaxBE + NT - 1) / NT;
  const int n = 1 << G.logn;
  const int LK = S.L + S.K;
  const int blk = blockIdx.x, j = blockIdx.y / LK, mi = blockIdx.y % LK, b = blockIdx.z;
  const int lo = j * S.alpha, hi = min(S.L, lo + S.alpha), na = hi - lo;
  if (mi >= lo && mi < hi) return;
  // LDS: [alpha + 1 twiddle tables of 2^S][alpha + 1 blocks]: table a < na inverts source a, table
  // alpha is the target's forward pass; block a holds source a, block alpha the target
  const int TWH = 1 << G.S;
  double2* twl = (double2*)smem_raw;
  double* smem = smem_raw + 2 * (size_t)(S.alpha + 1) * TWH;
  const int LB = lds_doubles(G.BE);
  double* work = smem + (size_t)S.alpha * LB;
  const ModTab tm = tab[mi];
  const ModD mm = mod_of2(tm);
  TwPre<NT, true, true, GT> twf;
  twf.load(G, blk, tm.fw);
  TwPre<NT, true, false, GT> twi[AMAX];
#pragma unroll
  for (int a = 0; a < AMAX; a++)
    if (a < na) twi[a].load(G, blk, tab[lo + a].iv);
  for (int a = 0; a < na; a++) {
    const double* src = T1 + ((size_t)b * S.L + lo + a) * n;
    double x[PER];
#pragma unroll
    for (int r = 0; r < PER; r++) {
      const int e = threadIdx.x + r * NT;
      if (e < G.BE) x[r] = gld(src + gidx_of_lds<true>(G, blk, e));
    }
    double* buf = smem + (size_t)a * LB;
#pragma unroll
    for (int r = 0; r < PER; r++) {
      const int e = threadIdx.x + r * NT;
      if (e < G.BE) buf[lpadx<true>(e)] = x[r];
    }
  }
  twf.store(twl + (size_t)S.alpha * TWH, G);
#pragma unroll
  for (int a = 0; a < AMAX; a++)
    if (a < na) twi[a].store(twl + (size_t)a * TWH, G);
  for (int a = AMAX; a < na; a++) stage_twiddles<NT, true, false>(twl + (size_t)a * TWH, G, blk, tab[lo + a].iv);
  __syncthreads();
  for (int a = 0; a < na; a++) {
    const ModTab ta = tab[lo + a];
    const ModD ma = mod_of2(ta);
    double* buf = smem + (size_t)a * LB;
    pass_inv<NT, true>(buf, twl + (size_t)a * TWH, G, blk, true, ta.iv, ta.ninv, ma, false);
    for (int e = threadIdx.x; e < G.BE; e += NT) {
      double x = canon(buf[lpadx<true>(e)], ma);
      if (na > 1) {
        const double2 ci = up_inv[j * S.alpha + a];
        x = canon(mul_tw(x, ci.x, ci.y, ma), ma);   // [x (Q_j/q_a)^-1]_{q_a}
      }
      buf[lpadx<true>(e)] = x;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < G.BE; e += NT) {
    double acc = 0.0;
    for (int a = 0; a < na; a++) {
      const double y = smem[(size_t)a * LB + lpadx<true>(e)];
      if (na > 1) {
        const double2 hm = up_hat[((size_t)j * S.alpha + a) * LK + mi];
        acc = reduce(acc + mul_tw(y, hm.x, hm.y, mm), mm);
      } else {
        acc = reduce(y, mm);   // one source prime: [x]_q as an integer, taken mod mi
      }
    }
    work[lpadx<true>(e)] = acc;
  }
  __syncthreads();
  pass_fwd<NT, true>(work, twl + (size_t)S.alpha * TWH, G, blk, tm.fw, mm, false);
  double* o = E + (((size_t)b * S.dnum + j) * LK + mi) * n;
  for (int e = threadIdx.x; e < G.BE; e += NT) gst(o + gidx_of_lds<true>(G, blk, e), work[lpadx<true>(e)]);
}

// K2 with TG targets per workgroup: the digit's inverse high pass runs once for TG targets, whose
// forward high passes then run concurrently (one modulus and twiddle table per block).  grid
// (nblk, dnum * ngrp, B), ngrp = ceil((L + K - na_min) / TG) with na_min the primes of the last
// (smallest) digit; target t of digit j is modulus t (t < lo) or t + na, skipping the digit's own
// primes; groups past a digit's targets exit.
template <int NT, int TG, class GT>
__global__ void __launch_bounds__(NT) k2_modup_grp(const double* __restrict__ T1, double* E, KsShape S, int ngrp,
                                                   const double2* __restrict__ up_inv, const double2* __restrict__ up_hat,
                                                   const ModTab* __restrict__ tab, GT G) {
  SMEM();
  constexpr int AMAX = 4;
  constexpr int PER = (GT::kMaxBE + NT - 1) / NT;
  const int n = 1 << G.logn;
  const int LK = S.L + S.K;
  const int blk = blockIdx.x, j = blockIdx.y / ngrp, g = blockIdx.y % ngrp, b = blockIdx.z;
  const int lo = j * S.alpha, hi = min(S.L, lo + S.alpha), na = hi - lo;
  const int t0 = g * TG, nt = min(TG, LK - na - t0);
  if (nt <= 0) return;
  // LDS: [alpha + TG twiddle tables of 2^S][TG moduli (q, 1/q)][alpha + TG blocks]
  const int TWH = 1 << G.S;
  double2* twl = (double2*)smem_raw;
  double2* mods = twl + (size_t)(S.alpha + TG) * TWH;
  double* smem = (double*)(mods + TG);
  const int LB = lds_doubles(G.BE);
  double* work = smem + (size_t)S.alpha * LB;
  int mis[TG];
#pragma unroll
  for (int tt = 0; tt < TG; tt++) {
    const int t = t0 + (tt < nt ? tt : 0);
    mis[tt] = t < lo ? t : t + na;
  }
  TwPre<NT, true, true, GT> twf[TG];
#pragma unroll
  for (int tt = 0; tt < TG; tt++) twf[tt].load(G, blk, tab[mis[tt]].fw);
  TwPre<NT, true, false, GT> twi[AMAX];
#pragma unroll
  for (int a = 0; a < AMAX; a++)
    if (a < na) twi[a].load(G, blk, tab[lo + a].iv);
  for (int a = 0; a < na; a++) {
    const double* src = T1 + ((size_t)b * S.L + lo + a) * n;
    double x[PER];
#pragma unroll
    for (int r = 0; r < PER; r++) {
      const int e = threadIdx.x + r * NT;
      if (e < G.BE) x[r] = gld(src + gidx_of_lds<true>(G, blk, e));
    }
    double* buf = smem + (size_t)a * LB;
#pragma unroll
    for (int r = 0; r < PER; r++) {
      const int e = threadIdx.x + r * NT;
      if (e < G.BE) buf[lpadx<true>(e)] = x[r];
    }
  }
#pragma unroll
  for (int tt = 0; tt < TG; tt++) twf[tt].store(twl + (size_t)(S.alpha + tt) * TWH, G);
  if (threadIdx.x < TG) {
    const ModTab tq = tab[mis[threadIdx.x]];
    mods[threadIdx.x] = double2{tq.q, tq.qinv};
  }
#pragma unroll
  for (int a = 0; a < AMAX; a++)
    if (a < na) twi[a].store(twl + (size_t)a * TWH, G);
  for (int a = AMAX; a < na; a++) stage_twiddles<NT, true, false>(twl + (size_t)a * TWH, G, blk, tab[lo + a].iv);
  __syncthreads();
  for (int a = 0; a < na; a++) {
    const ModTab ta = tab[lo + a];
    const ModD ma = mod_of2(ta);
    double* buf = smem + (size_t)a * LB;
    pass_inv<NT, true>(buf, twl + (size_t)a * TWH, G, blk, true, ta.iv, ta.ninv, ma, false);
    for (int e = threadIdx.x; e < G.BE; e += NT) {
      double x = canon(buf[lpadx<true>(e)], ma);
      if (na > 1) {
        const double2 ci = up_inv[j * S.alpha + a];
        x = canon(mul_tw(x, ci.x, ci.y, ma), ma);   // [x (Q_j/q_a)^-1]_{q_a}
      }
      buf[lpadx<true>(e)] = x;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < (nt << G.lbe); t += NT) {
    const int tt = t >> G.lbe, e = t & (G.BE - 1);
    const ModD mm{mods[tt].x, mods[tt].y};
    double acc = 0.0;
    for (int a = 0; a < na; a++) {
      const double y = smem[(size_t)a * LB + lpadx<true>(e)];
      if (na > 1) {
        const int t_mod = (t0 + tt) < lo ? (t0 + tt) : (t0 + tt + na);
        const double2 hm = up_hat[((size_t)j * S.alpha + a) * LK + t_mod];
        acc = reduce(acc + mul_tw(y, hm.x, hm.y, mm), mm);
      } else {
        acc = reduce(y, mm);   // one source prime: [x]_q as an integer, taken mod the target
      }
    }
    work[(size_t)tt * LB + lpadx<true>(e)] = acc;
  }
  __syncthreads();
  pass_fwd_multi_mod<NT, true>(work, LB, nt, twl + (size_t)S.alpha * TWH, TWH, mods, G, blk);
  for (int t = threadIdx.x; t < (nt << G.lbe); t += NT) {
    const int tt = t >> G.lbe, e = t & (G.BE - 1);
    const int t_mod = (t0 + tt) < lo ? (t0 + tt) : (t0 + tt + na);
    double* o = E + (((size_t)b * S.dnum + j) * LK + t_mod) * n;
    gst(o + gidx_of_lds<true>(G, blk, e), work[(size_t)tt * LB + lpadx<true>(e)]);
  }
}

// grid (nblk, L + K, B).  The next digit's block is loaded into registers while the current one
// is transformed (its twiddles are staged once: every digit uses modulus mi).
template <int NT, class GT>
__global__ void __launch_bounds__(NT) k2_ip_low(const RotItem* __restrict__ items, const double* __restrict__ E, double* ACC, double* T2, KsShape S,
                                                const ModTab* __restrict__ tab, GT G) {
  SMEM2(G);
  constexpr int PER = kBlockElems / NT > 0 ? kBlockElems / NT : 1;
  const int n = 1 << G.logn;
  const int blk = blockIdx.x, mi = blockIdx.y, b = blockIdx.z;
  const int LK = S.L + S.K;
  const RotItem it = items[b];
  const ModTab tm = tab[mi];
  const ModD m = mod_of2(tm);
  double a0[PER], a1[PER], nx[PER];
#pragma unroll
  for (int k = 0; k < PER; k++) { a0[k] = 0.0; a1[k] = 0.0; }
  auto load_digit = [&](int j) {
    const int lo = j * S.alpha, hi = min(S.L, lo + S.alpha);
    if (mi >= lo && mi < hi) {
      const u64* c1 = it.in + ((size_t)S.L + mi) * n;
#pragma unroll
      for (int k = 0; k < PER; k++) {
        const int e = threadIdx.x + k * NT;
        if (e < G.BE) nx[k] = u2d(c1[galois_index2((u32)gidx_of_lds<false>(G, blk, e), it.galois, G.logn)]);
      }
    } else {
      const double* src = E + (((size_t)b * S.dnum + j) * LK + mi) * n;
#pragma unroll
      for (int k = 0; k < PER; k++) {
        const int e = threadIdx.x + k * NT;
        if (e < G.BE) nx[k] = src[gidx_of_lds<false>(G, blk, e)];
      }
    }
  };
  stage_twiddles<NT, false, true>(twl, G, blk, tm.fw);
  load_digit(0);
  for (int j = 0; j < S.dnum; j++) {
    const int lo = j * S.alpha, hi = min(S.L, lo + S.alpha);
    const bool own = (mi >= lo && mi < hi);
#pragma unroll
    for (int k = 0; k < PER; k++) {
      const int e = threadIdx.x + k * NT;
      if (e < G.BE) smem[lpad(e)] = nx[k];
    }
    if (j + 1 < S.dnum) load_digit(j + 1);
    __syncthreads();
    if (!own) pass_fwd<NT, false>(smem, twl, G, blk, tm.fw, m, false);
    const u64* kb = it.key + (((size_t)0 * S.dnum + j) * LK + mi) * n;
    const u64* ka = it.key + (((size_t)1 * S.dnum + j) * LK + mi) * n;
#pragma unroll
    for (int k = 0; k < PER; k++) {
      const int e = threadIdx.x + k * NT;
      if (e < G.BE) {
        const int gi = gidx_of_lds<false>(G, blk, e);
        const double x = smem[lpad(e)];
        a0[k] += mulmod(x, u2d(kb[gi]), m);
        a1[k] += mulmod(x, u2d(ka[gi]), m);
      }
    }
    if ((j & 3) == 3) {
#pragma unroll
      for (int k = 0; k < PER; k++) { a0[k] = reduce(a0[k], m); a1[k] = reduce(a1[k], m); }
    }
    __syncthreads();
  }
  if (mi < S.L) {
    double* o0 = ACC + (((size_t)b * 2 + 0) * S.L + mi) * n;
    double* o1 = ACC + (((size_t)b * 2 + 1) * S.L + mi) * n;
#pragma unroll
    for (int k = 0; k < PER; k++) {
      const int e = threadIdx.x + k * NT;
      if (e < G.BE) {
        const int gi = gidx_of_lds<false>(G, blk, e);
        o0[gi] = reduce(a0[k], m);
        o1[gi] = reduce(a1[k], m);
      }
    }
  } else {
    stage_twiddles<NT, false, false>(twl, G, blk, tm.iv);
    for (int w = 0; w < 2; w++) {
#pragma unroll
      for (int k = 0; k < PER; k++) {
        const int e = threadIdx.x + k * NT;
        if (e < G.BE) smem[lpad(e)] = canon(w == 0 ? a0[k] : a1[k], m);
      }
      __syncthreads();
      pass_inv<NT, false>(smem, twl, G, blk, false, tm.iv, tm.ninv, m, false);
      double* o = T2 + (((size_t)b * 2 + w) * S.K + (mi - S.L)) * n;
      for (int e = threadIdx.x; e < G.BE; e += NT) o[gidx_of_lds<false>(G, blk, e)] = smem[lpad(e)];
      __syncthreads();
    }
  }
}

// K3 with every digit resident at once: the digit blocks (own limb: sigma_g(c1)) sit side by side
// in LDS and one workgroup of NT threads transforms all of them concurrently, then forms the inner
// product per element.  LDS [staged twiddles: BE double2][dnum blocks of lds_doubles(BE)].
// grid (nblk, L + 2K, B): y < L is data prime y (both accumulators); y >= L is special prime
// L + (y - L) / 2 and accumulator (y - L) % 2 only, whose workgroup also runs that accumulator's
// inverse low pass (splitting the special limbs this way keeps every workgroup's work close to
// that of a data-prime workgroup, which sets the kernel's duration).
template <int NT, int DMAX, class GT>
__global__ void __launch_bounds__(NT) k2_ip_par(const RotItem* __restrict__ items, const double* __restrict__ E, double* ACC, double* T2, KsShape S,
                                                const ModTab* __restrict__ tab, GT G) {
  SMEM2(G);
  constexpr int PER = GT::kMaxBE / NT > 0 ? GT::kMaxBE / NT : 1;
  const int n = 1 << G.logn;
  const int blk = blockIdx.x, y = blockIdx.y, b = blockIdx.z;
  const bool special = y >= S.L;
  const int mi = special ? S.L + ((y - S.L) >> 1) : y;
  const int wsel = special ? ((y - S.L) & 1) : 0;
  const int LK = S.L + S.K;
  const int LB = lds_doubles(G.BE);
  const RotItem it = items[b];
  const ModTab tm = tab[mi];
  const ModD m = mod_of2(tm);
  const int jown = special ? -1 : mi / S.alpha;
  // Every global load is issued before the first wait, without branches: the key words (a
  // special-prime workgroup reads its one key part into both sets), the digit blocks and the
  // twiddles of the forward (and, for the special primes, inverse) low pass.  Digits beyond dnum
  // and elements beyond the block (runtime geometry) read valid words that are ignored.
  const int p0 = special ? wsel : 0, p1 = special ? wsel : 1;
  TwPre<NT, false, true, GT> twf;
  twf.load(G, blk, tm.fw);
  u64 kbv[PER][DMAX], kav[PER][DMAX], xv[PER][DMAX];  // raw words: converted after the loads
  const u64* c1 = it.in + ((size_t)S.L + mi) * n;
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const int e = threadIdx.x + k * NT;
    const int gi = gidx_of_lds<false>(G, blk, e < G.BE ? e : 0);
#pragma unroll
    for (int j = 0; j < DMAX; j++) {
      const int jj = j < S.dnum ? j : 0;
      kbv[k][j] = gld(it.key + (((size_t)p0 * S.dnum + jj) * LK + mi) * n + gi);
      kav[k][j] = gld(it.key + (((size_t)p1 * S.dnum + jj) * LK + mi) * n + gi);
      const u64* src = (jj == jown) ? c1 + galois_index2((u32)gi, it.galois, G.logn)
                                    : (const u64*)(E + (((size_t)b * S.dnum + jj) * LK + mi) * n + gi);
      xv[k][j] = gld(src);
    }
  }
  TwPre<NT, false, false, GT> twi;
  if (special) twi.load(G, blk, tm.iv);
  twf.store(twl, G);
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const int e = threadIdx.x + k * NT;
#pragma unroll
    for (int j = 0; j < DMAX; j++)
      if (j < S.dnum && e < G.BE) smem[(size_t)j * LB + lpad(e)] = (j == jown) ? u2d(xv[k][j]) : __longlong_as_double((long long)xv[k][j]);
  }
  __syncthreads();
  pass_fwd_multi<NT, false>(smem, LB, S.dnum, jown >= 0 ? (1u << jown) : 0u, twl, G, blk, m);
  double r0[PER], r1[PER];
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const int e = threadIdx.x + k * NT;
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int j = 0; j < DMAX; j++) {
      if (j < S.dnum && e < G.BE) {
        const double x = smem[(size_t)j * LB + lpad(e)];
        a0 += mulmod(x, u2d(kbv[k][j]), m);
        a1 += mulmod(x, u2d(kav[k][j]), m);
        if ((j & 3) == 3) { a0 = reduce(a0, m); a1 = reduce(a1, m); }
      }
    }
    r0[k] = reduce(a0, m);
    r1[k] = reduce(a1, m);
    if (!special && e < G.BE) {
      const int gi = gidx_of_lds<false>(G, blk, e);
      gst(ACC + (((size_t)b * 2 + 0) * S.L + mi) * n + gi, r0[k]);
      gst(ACC + (((size_t)b * 2 + 1) * S.L + mi) * n + gi, r1[k]);
    }
  }
  if (!special) return;
  // special prime: inverse low pass of the selected accumulator (r0 = r1 here)
  __syncthreads();
  twi.store(twl, G);
#pragma unroll
  for (int k = 0; k < PER; k++)
    if (threadIdx.x + k * NT < G.BE) smem[lpad(threadIdx.x + k * NT)] = canon(r0[k], m);
  __syncthreads();
  pass_inv_multi<NT, false>(smem, LB, 1, false, twl, tm.ninv, G, blk, m);
  double* o = T2 + (((size_t)b * 2 + wsel) * S.K + (mi - S.L)) * n;
  for (int e = threadIdx.x; e < G.BE; e += NT) gst(o + gidx_of_lds<false>(G, blk, e), smem[lpad(e)]);
}

// grid (nblk, 2 L, B): polynomial w = y / L, data prime i = y % L.  The special limbs' inverse
// high pass is recomputed per target.
template <int NT, class GT>
__global__ void __launch_bounds__(NT) k2_moddown_high(const double* __restrict__ T2, double* F, KsShape S, const double2* __restrict__ dn_inv,
                                                      const double2* __restrict__ dn_hat, const ModTab* __restrict__ tab, GT G) {
  SMEM();
  constexpr int KMAX = 4;  // special primes whose twiddles are prefetched (more: staged late)
  constexpr int PER = (GT::kMaxBE + NT - 1) / NT;
  const int n = 1 << G.logn;
  const int blk = blockIdx.x, w = blockIdx.y / S.L, i = blockIdx.y % S.L, b = blockIdx.z;
  // LDS: [K + 1 twiddle tables of 2^S][K + 1 blocks]: table k < K inverts special prime k, table K
  // is the target's forward pass; block k holds special limb k, block K the target
  const int TWH = 1 << G.S;
  double2* twl = (double2*)smem_raw;
  double* smem = smem_raw + 2 * (size_t)(S.K + 1) * TWH;
  const int LB = lds_doubles(G.BE);
  double* work = smem + (size_t)S.K * LB;
  const ModTab tq = tab[i];
  const ModD mq = mod_of2(tq);
  TwPre<NT, true, true, GT> twf;
  twf.load(G, blk, tq.fw);
  TwPre<NT, true, false, GT> twi[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; k++)
    if (k < S.K) twi[k].load(G, blk, tab[S.L + k].iv);
  for (int k = 0; k < S.K; k++) {
    const double* src = T2 + (((size_t)b * 2 + w) * S.K + k) * n;
    double x[PER];
#pragma unroll
    for (int r = 0; r < PER; r++) {
      const int e = threadIdx.x + r * NT;
      if (e < G.BE) x[r] = gld(src + gidx_of_lds<true>(G, blk, e));
    }
    double* buf = smem + (size_t)k * LB;
#pragma unroll
    for (int r = 0; r < PER; r++) {
      const int e = threadIdx.x + r * NT;
      if (e < G.BE) buf[lpadx<true>(e)] = x[r];
    }
  }
  twf.store(twl + (size_t)S.K * TWH, G);
#pragma unroll
  for (int k = 0; k < KMAX; k++)
    if (k < S.K) twi[k].store(twl + (size_t)k * TWH, G);
  for (int k = KMAX; k < S.K; k++) stage_twiddles<NT, true, false>(twl + (size_t)k * TWH, G, blk, tab[S.L + k].iv);
  __syncthreads();
  for (int k = 0; k < S.K; k++) {
    const ModTab tp = tab[S.L + k];
    const ModD mp = mod_of2(tp);
    double* buf = smem + (size_t)k * LB;
    pass_inv<NT, true>(buf, twl + (size_t)k * TWH, G, blk, true, tp.iv, tp.ninv, mp, false);
    for (int e = threadIdx.x; e < G.BE; e += NT) {
      double x = canon(buf[lpadx<true>(e)], mp);
      if (S.K > 1) {
        const double2 ci = dn_inv[k];
        x = canon(mul_tw(x, ci.x, ci.y, mp), mp);
      }
      buf[lpadx<true>(e)] = x;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < G.BE; e += NT) {
    double acc = 0.0;
    for (int k = 0; k < S.K; k++) {
      const double y = smem[(size_t)k * LB + lpadx<true>(e)];
      if (S.K > 1) {
        const double2 hm = dn_hat[(size_t)k * S.L + i];
        acc = reduce(acc + mul_tw(y, hm.x, hm.y, mq), mq);
      } else {
        acc = reduce(y, mq);
      }
    }
    work[lpadx<true>(e)] = acc;
  }
  __syncthreads();
  pass_fwd<NT, true>(work, twl + (size_t)S.K * TWH, G, blk, tq.fw, mq, false);
  double* o = F + (((size_t)b * 2 + w) * S.L + i) * n;
  for (int e = threadIdx.x; e < G.BE; e += NT) gst(o + gidx_of_lds<true>(G, blk, e), work[lpadx<true>(e)]);
}

// The epilogue's operands (accumulator, sigma_g(c0), addend) are loaded with the block, before
// the pass, so their latency hides behind it.
template <int NT, class GT>
__global__ void __launch_bounds__(NT) k2_final_low(const RotItem* __restrict__ items, const double* __restrict__ F, const double* __restrict__ ACC,
                                                   const double2* __restrict__ pinv, KsShape S, const ModTab* __restrict__ tab, GT G,
                                                   const RotItem* __restrict__ next_items, double* T1) {
  SMEM2(G);
  __shared__ int s_dst;
  constexpr int PER = (GT::kMaxBE + NT - 1) / NT;
  const int n = 1 << G.logn;
  const int blk = blockIdx.x, wi = blockIdx.y, b = blockIdx.z;
  const int w = wi / S.L, i = wi % S.L;
  const RotItem it = items[b];
  const ModTab tq = tab[i];
  const ModD m = mod_of2(tq);
  // fused next-level K1 (see below): the gather block it fills, found before the first barrier
  const bool fuse = w == 1 && next_items != nullptr && it.next != 0;   // uniform per workgroup
  const int bn = fuse ? (int)it.next - 1 : 0;
  const u32 g2 = (fuse ? next_items + bn : items + b)->galois;          // a valid item either way
  for (int t = threadIdx.x; t < G.nblk; t += NT)
    if ((galois_index2((u32)(t << G.lbe), g2, G.logn) >> G.lbe) == (u32)blk) s_dst = t;
  TwPre<NT, false, true, GT> tw;
  tw.load(G, blk, tq.fw);
  const double* src = F + (((size_t)b * 2 + w) * S.L + i) * n;
  const double* acc = ACC + (((size_t)b * 2 + w) * S.L + i) * n;
  const u64* c0 = it.in + (size_t)i * n;
  const u64* add = it.addend ? it.addend + ((size_t)w * S.L + i) * n : nullptr;
  double x[PER], av[PER];
  u64 c0w[PER], adw[PER];  // raw words, converted after the pass (branch-free loads)
#pragma unroll
  for (int r = 0; r < PER; r++) {
    const int e = threadIdx.x + r * NT;
    const int gi = gidx_of_lds<false>(G, blk, e < G.BE ? e : 0);
    x[r] = gld(src + gi);
    av[r] = gld(acc + gi);
    const u64* c0p = c0 + galois_index2((u32)gi, it.galois, G.logn);
    c0w[r] = gld(c0p);
    adw[r] = gld(add ? add + gi : c0p);
  }
  tw.store(twl, G);
#pragma unroll
  for (int r = 0; r < PER; r++) {
    const int e = threadIdx.x + r * NT;
    if (e < G.BE) smem[lpad(e)] = x[r];
  }
  __syncthreads();
  // the fused step's inverse twiddles, in flight during the forward pass (loaded by every
  // workgroup: no branch around the loads)
  const int dst = s_dst;
  TwPre<NT, false, false, GT> twi;
  twi.load(G, dst, tq.iv);
  pass_fwd<NT, false>(smem, twl, G, blk, tq.fw, m, false);
  const double2 pv = pinv[i];
  u64* out = it.out + ((size_t)w * S.L + i) * n;
#pragma unroll
  for (int r = 0; r < PER; r++) {
    const int e = threadIdx.x + r * NT;
    if (e < G.BE) {
      const int gi = gidx_of_lds<false>(G, blk, e);
      const double cv = (w == 0 ? u2d(c0w[r]) : 0.0) + (add ? u2d(adw[r]) : 0.0);
      const double v = canon(mul_tw(reduce(av[r] - smem[lpad(e)], m), pv.x, pv.y, m) + cv, m);
      gst(out + gi, d2u(v));
      if (fuse) smem[lpad(e)] = v;   // the element this thread has just read
    }
  }
  if (!fuse) return;
  // The next level's K1 for this output: sigma_g'(c1') gathered block by block, inverse low pass.
  // Block dst of the gather reads only this block (the permutation maps blocks onto blocks).
  __syncthreads();   // the output block is in LDS; the forward pass's twiddles are no longer read
  twi.store(twl, G);
#pragma unroll
  for (int r = 0; r < PER; r++) {
    const int e = threadIdx.x + r * NT;
    if (e < G.BE) {
      const u32 sidx = galois_index2((u32)gidx_of_lds<false>(G, dst, e), g2, G.logn);
      x[r] = smem[lpad((int)sidx - (blk << G.lbe))];
    }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < PER; r++) {
    const int e = threadIdx.x + r * NT;
    if (e < G.BE) smem[lpad(e)] = x[r];
  }
  __syncthreads();
  pass_inv<NT, false>(smem, twl, G, dst, false, tq.iv, tq.ninv, m, false);
  double* o = T1 + ((size_t)bn * S.L + i) * n;
  for (int e = threadIdx.x; e < G.BE; e += NT) gst(o + gidx_of_lds<false>(G, dst, e), smem[lpad(e)]);
}

// ------------------------------------------------------------------ launchers
// ModUp targets per workgroup of K2: 1 = k2_modup_high, 2 or 3 = k2_modup_grp, 0 = automatic
// (three on the small-level geometry of N = 16384, whose ModUp blocks are smaller than the
// level's; otherwise two below 5 items and three from 5 on: the shared inverse pass saves work
// while fewer, longer workgroups cost latency).
static std::mutex g2_mu;
static std::map<const void*, size_t> g2_set;
static void ensure_lds2(const void* f, size_t bytes) {
  std::lock_guard<std::mutex> g(g2_mu);
  auto it = g2_set.find(f);
  if (it != g2_set.end() && it->second >= bytes) return;
  HS_CHECK_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  g2_set[f] = bytes;
}

template <class GT>
static int nt2(const GT& G) { return (G.BE >= 2048 || (G.BE >= 512 && G.logn >= 14)) ? 256 : 64; }
// geometry of the all-digit inner product (K3): half-size blocks of the level's geometry, and never
// below 1024 elements
template <class GT> struct IpGeom { using type = typename HalfBlocks<GT>::type; };
template <> struct IpGeom<PassGeomC<14, 9>> { using type = PassGeomC<14, 10>; };
// geometry of the ModUp kernel (K2): the level's, never below 1024 elements, and 1024 at N = 2^15
// (with two-prime digits its LDS, (digit primes + targets) x (block + twiddles), allows one
// workgroup per CU on 2048-element blocks and three on 1024: 0.57 -> 0.47 ms for a level of 20
// relinearisations; at N = 2^14 the 2048-element levels measured faster as they are)
template <class GT> struct ModupGeom { using type = GT; };
// geometry of the ModDown kernel (K4): the level's, 1024 elements at N = 2^15
template <class GT> struct ModdownGeom { using type = GT; };
template <> struct ModdownGeom<PassGeomC<15, 11>> { using type = PassGeomC<15, 10>; };
template <> struct ModupGeom<PassGeomC<14, 9>> { using type = PassGeomC<14, 10>; };
template <> struct ModupGeom<PassGeomC<15, 11>> { using type = PassGeomC<15, 10>; };

// Launch KERNEL<NT, GT> (GT = the geometry type in scope) with 256 or 64 threads.
#define HS2_LAUNCH(KERNEL, GRID, LDS, STREAM, ...)                                                  \
  do {                                                                                              \
    ProfScope _prof(#KERNEL, STREAM);                                                               \
    if (nt2(G) == 256) {                                                                            \
      ensure_lds2((const void*)KERNEL<256, GT>, LDS);                                               \
      hipLaunchKernelGGL((KERNEL<256, GT>), GRID, dim3(256), LDS, STREAM, __VA_ARGS__);             \
    } else {                                                                                        \
      ensure_lds2((const void*)KERNEL<64, GT>, LDS);                                                \
      hipLaunchKernelGGL((KERNEL<64, GT>), GRID, dim3(64), LDS, STREAM, __VA_ARGS__);               \
    }                                                                                               \
    HS_CHECK_HIP(hipGetLastError());                                                                \
  } while (0)

// Calls f(geometry): compile-time for the ring sizes this path serves, runtime otherwise.
template <class F>
static void with_geom(int logn, F&& f) {
  switch (logn) {
    case 12: f(PassGeomC<12>{}); break;
    case 13: f(PassGeomC<13>{}); break;
    case 14: f(PassGeomC<14>{}); break;
    case 15: f(PassGeomC<15>{}); break;
    default: f(make_geom(logn)); break;
  }
}

// A few limbs of N = 2^14 (the clients' transforms) run on 512-element blocks: four times the
// workgroups of the 2048-element geometry, each with a quarter of the serial work (measured in
// decryption: 63 -> 54 us).
void launch_ntt2(const hs_ctx* c, u64* data, double* scratch, i64 rows, int nl, int mod0, int inverse, hipStream_t st) {
  if (rows <= 0) return;
  auto body = [&](auto G) {
    using GT = decltype(G);
    const size_t lds = (size_t)(lds_doubles(G.BE) + 2 * G.BE) * sizeof(double);
    const ModTab* tab = (const ModTab*)c->d_tab;
    const dim3 grid(G.nblk, (unsigned)rows);
    if (!inverse) {
      HS2_LAUNCH(k2_ntt_pass_hf, grid, lds, st, data, 1, scratch, 0, nl, mod0, 0, tab, G);
      HS2_LAUNCH(k2_ntt_pass_lf, grid, lds, st, scratch, 0, data, 1, nl, mod0, 0, tab, G);
    } else {
      HS2_LAUNCH(k2_ntt_pass_li, grid, lds, st, data, 1, scratch, 0, nl, mod0, 0, tab, G);
      HS2_LAUNCH(k2_ntt_pass_hi, grid, lds, st, scratch, 0, data, 1, nl, mod0, 1, tab, G);
    }
  };
  if (c->logn == 14 && rows <= 64) body(PassGeomC<14, 9>{});
  else with_geom(c->logn, body);
}

// Block size of the two-pass key switch at N = 2^14: 3 = 512-element blocks for the single-pass
// kernels (K1, K4, K5) with ModUp and the inner product on 1024 (more, shorter workgroups: the
// kernels are latency-bound at a few items per level), 1 = 2048-element blocks throughout (K3 on
// 1024), 2 = 1024-element blocks throughout, 0 = automatic: 3 up to kSmallLevel items, else 1.

void launch_rotate_batch2(const hs_ctx* c, const RotItem* d_items, int B, const KsShape& S, double* T1, double* E, double* ACC, double* T2,
                          double* F, hipStream_t st, int B1, const RotItem* d_next) {
  if (B <= 0) return;
  if (B1 < 0 || B1 > B) B1 = B;
  ProfUnits units(B);
  auto body = [&](auto G) {
    using GT = decltype(G);
    const size_t LB = (size_t)lds_doubles(G.BE) * sizeof(double);
    const size_t TW = (size_t)2 * G.BE * sizeof(double);
    const size_t TWH = (size_t)2 * (1 << G.S) * sizeof(double);
    const ModTab* tab = (const ModTab*)c->d_tab;
    const int LK = c->L + c->K;
    if (B1 > 0) HS2_LAUNCH(k2_rot_intt_low, dim3(G.nblk, c->L, B1), TW + LB, st, d_items, T1, c->L, tab, G);
    using G2T = typename ModupGeom<GT>::type;
    // targets per ModUp workgroup: three on 1024-element blocks (the small-level geometry at
    // N = 2^14, where it measured fastest at every level size), else two below 5 items
    const int tg_opt = option(c, HS_OPT_MODUP_GROUP);
    const int tg = tg_opt > 0 ? tg_opt : ((B >= 5 || !std::is_same<G2T, GT>::value) ? 3 : 2);
    G2T G2{};
    if constexpr (std::is_same<G2T, GT>::value) G2 = G;   // a runtime geometry carries its fields
    const size_t LB2 = (size_t)lds_doubles(G2.BE) * sizeof(double);
    if (tg <= 1) {
      HS2_LAUNCH(k2_modup_high, dim3(G.nblk, c->dnum * LK, B), (TWH + LB) * (c->alpha + 1), st, (const double*)T1, E, S,
                 (const double2*)c->d_up_inv, (const double2*)c->d_up_hat, tab, G);
    } else {
      // enough groups for the digit with the fewest primes (the last one), which has the most targets
      const int na_min = c->L - (c->dnum - 1) * c->alpha;
      const int ngrp = (LK - na_min + tg - 1) / tg;
      const size_t lds = (TWH + LB2) * (c->alpha + tg) + 16 * (size_t)tg;
      ProfScope _prof("k2_modup_grp", st);
      if (tg == 2) {
        ensure_lds2((const void*)k2_modup_grp<512, 2, G2T>, lds);
        hipLaunchKernelGGL((k2_modup_grp<512, 2, G2T>), dim3(G2.nblk, c->dnum * ngrp, B), dim3(512), lds, st, (const double*)T1, E, S, ngrp,
                           (const double2*)c->d_up_inv, (const double2*)c->d_up_hat, tab, G2);
      } else {
        ensure_lds2((const void*)k2_modup_grp<512, 3, G2T>, lds);
        hipLaunchKernelGGL((k2_modup_grp<512, 3, G2T>), dim3(G2.nblk, c->dnum * ngrp, B), dim3(512), lds, st, (const double*)T1, E, S, ngrp,
                           (const double2*)c->d_up_inv, (const double2*)c->d_up_hat, tab, G2);
      }
      HS_CHECK_HIP(hipGetLastError());
    }
    // the all-digit inner product on half-size blocks where the geometry is compile-time (twice
    // the workgroups, each with half the serial work; two fit a CU)
    using G3T = typename IpGeom<GT>::type;
    const G3T G3{};
    constexpr int NT3 = G3T::kMaxBE >= 2048 ? 1024 : 512;
    const size_t LB3 = (size_t)lds_doubles(G3.BE) * sizeof(double), TW3 = (size_t)2 * G3.BE * sizeof(double);
    if (TW3 + LB3 * c->dnum <= (size_t)160 * 1024 && G3.BE >= 1024 && c->dnum <= 6) {
      ProfScope _prof("k2_ip_par", st);
      ensure_lds2((const void*)k2_ip_par<NT3, 6, G3T>, TW3 + LB3 * c->dnum);
      hipLaunchKernelGGL((k2_ip_par<NT3, 6, G3T>), dim3(G3.nblk, c->L + 2 * c->K, B), dim3(NT3), TW3 + LB3 * c->dnum, st, d_items, (const double*)E,
                         ACC, T2, S, tab, G3);
      HS_CHECK_HIP(hipGetLastError());
    } else {
      HS2_LAUNCH(k2_ip_low, dim3(G.nblk, LK, B), TW + LB, st, d_items, (const double*)E, ACC, T2, S, tab, G);
    }
    using G4T = typename ModdownGeom<GT>::type;
    if constexpr (std::is_same<G4T, GT>::value) {
      HS2_LAUNCH(k2_moddown_high, dim3(G.nblk, 2 * c->L, B), (TWH + LB) * (c->K + 1), st, (const double*)T2, F, S,
                 (const double2*)c->d_dn_inv, (const double2*)c->d_dn_hat, tab, G);
    } else {
      auto k4 = [&](auto G) {   // the macro launches on this geometry
        using GT = decltype(G);
        const size_t LB4 = (size_t)lds_doubles(G.BE) * sizeof(double);
        HS2_LAUNCH(k2_moddown_high, dim3(G.nblk, 2 * c->L, B), (TWH + LB4) * (c->K + 1), st, (const double*)T2, F, S,
                   (const double2*)c->d_dn_inv, (const double2*)c->d_dn_hat, tab, G);
      };
      k4(G4T{});
    }
    HS2_LAUNCH(k2_final_low, dim3(G.nblk, 2 * c->L, B), TW + LB, st, d_items, (const double*)F, (const double*)ACC,
               (const double2*)c->d_pinv, S, tab, G, d_next, T1);
  };
  constexpr int kSmallLevel = 8;
  const int blk_opt = option(c, HS_OPT_KS_BLOCK);
  const int blk = blk_opt == 0 ? (B <= kSmallLevel ? 3 : 1) : blk_opt;
  if (c->logn == 14 && blk == 3) body(PassGeomC<14, 9>{});
  else if (c->logn == 14 && blk == 2) body(PassGeomC<14, 10>{});
  else with_geom(c->logn, body);
}

}  // namespace hs
