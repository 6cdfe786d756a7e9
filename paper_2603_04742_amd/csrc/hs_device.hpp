// Device-side modular arithmetic and the LDS-resident negacyclic NTT for gfx950.
//
// Residues live in HBM as u64 in [0, q).  Inside kernels they are held as IEEE doubles carrying
// exact integers ("balanced" form: any integer congruent to the residue, |x| < 2^52).  For
// moduli q < 2^50 a modular product needs six full-rate FP64 operations (van der Hoeven, Lecerf &
// Quintin, "Modular SIMD arithmetic in Mathemagix", ACM TOMS 2016): the exact product is split as
// h + l with h = fl(a b), l = fma(a, b, -h); a quotient estimate qt is rounded to an integer with
// the 1.5*2^52 constant; r = fma(-qt, q, h) + l is then exact and small.  On MI355X this runs at
// ~5.9 T modmul/s against ~1.8 T/s for a 64-bit integer Shoup product.
//
// Bounds used below (q < 2^50, w in [0, q), wq = fl(w / q)):
//   mul_tw(a, w, wq), |a| <= 2^51 : result r = a w mod q exactly, |r| <= 0.625 q
//   mulmod(a, b),  |a b| <= 2^100 : |r| <= 0.75 q
//   reduce(x),        |x| <  2^52 : |r| <= q/2 + 1
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef HS_NTT_RADIX_BITS
#define HS_NTT_RADIX_BITS 3  // register rounds of radix 2^3: keeps the NTT under 128 VGPRs at 1024 threads
#endif

namespace hs {

typedef uint64_t u64;
typedef uint32_t u32;

struct ModD {
  double q;     // modulus
  double qinv;  // fl(1/q)
};

static constexpr double kRound = 6755399441055744.0;  // 1.5 * 2^52

__device__ __forceinline__ double rint_small(double x) {  // |x| < 2^51
  return __builtin_fma(x, 1.0, kRound) - kRound;
}

// x mod q into [-q/2 - 1, q/2 + 1]; |x| < 2^52.
__device__ __forceinline__ double reduce(double x, ModD m) {
  double k = __builtin_rint(x * m.qinv);
  return __builtin_fma(-k, m.q, x);
}

// a * w mod q for a twiddle or constant w in [0, q) with precomputed wq = fl(w/q); |a| <= 2^51.
__device__ __forceinline__ double mul_tw(double a, double w, double wq, ModD m) {
  double h = a * w;
  double l = __builtin_fma(a, w, -h);
  double k = __builtin_fma(a, wq, kRound) - kRound;
  double r = __builtin_fma(-k, m.q, h);
  return r + l;
}

// a * b mod q for arbitrary balanced operands with |a b| <= 2^100.
__device__ __forceinline__ double mulmod(double a, double b, ModD m) {
  double h = a * b;
  double l = __builtin_fma(a, b, -h);
  double k = __builtin_fma(h, m.qinv, kRound) - kRound;
  double r = __builtin_fma(-k, m.q, h);
  return r + l;
}

// a * w mod q for a twiddle |w| < q given alone (no precomputed quotient): the quotient is
// estimated from the rounded product, fl(a w) fl(1/q), which errs from a w / q by at most
// 2^-52 |a w| / q < 2^-52 |a|.  For |a| <= 1.91 * 2^50 that keeps the estimate below 2^51 (exact
// rounding by kRound) and the result r = a w - k q exact with |r| <= q (1/2 + 2^-52 |a|), i.e.
// <= 0.625 q, 0.79 q, 0.98 q for |a| <= q/2 + 1, 1.125 q, 1.91 q.  It is mulmod's arithmetic
// (as many operations as mul_tw) under these bounds.
__device__ __forceinline__ double mul_twc(double a, double w, ModD m) { return mulmod(a, w, m); }

// Balanced value (|x| < 2^52) -> canonical residue in [0, q).
__device__ __forceinline__ double canon(double x, ModD m) {
  double r = reduce(x, m);
  return r < 0.0 ? r + m.q : r;
}

// Residue <-> double for integers in [0, 2^52): the integer is the mantissa of 2^52 + x, so
// each direction is one integer and one floating-point operation.
__device__ __forceinline__ double u2d(u64 x) {
  return __longlong_as_double((long long)(x | 0x4330000000000000ULL)) - 4503599627370496.0;
}
__device__ __forceinline__ u64 d2u(double x) {
  return (u64)__double_as_longlong(x + 4503599627370496.0) ^ 0x4330000000000000ULL;
}

// Twiddle tables are global memory; loading through an address-space-1 pointer gives global
// (not flat) loads, which do not hold up the LDS wait counter.
typedef const double __attribute__((address_space(1)))* gdbl_ptr;
__device__ __forceinline__ double2 ldtw(const double2* p, int i) {
  const gdbl_ptr g = (gdbl_ptr)(const double*)(p + i);
  return double2{g[0], g[1]};
}

// Global memory through address-space-1 pointers: such a load cannot alias LDS, so the compiler
// issues a workgroup's loads together ahead of the LDS stores that consume them instead of
// waiting for each one in turn (a flat pointer could point into LDS), and it does not hold up the
// LDS wait counter.
template <class T>
__device__ __forceinline__ T gld(const T* p) { return *(const T __attribute__((address_space(1)))*)p; }
template <class T>
__device__ __forceinline__ void gst(T* p, T v) { *(T __attribute__((address_space(1)))*)p = v; }

__device__ __forceinline__ u32 brev_bits(u32 x, int bits) { return __brev(x) >> (32 - bits); }

// LDS layout with one pad double every 16, so that power-of-two strides spread over the banks.
__device__ __forceinline__ int lpad(int i) { return i + (i >> 4); }
__host__ __device__ constexpr int lds_doubles(int n) { return n + (n >> 4); }

// Twiddle tables per modulus: tw[i] = (w_i, fl(w_i / q)) with
//   forward  w_i = psi^bitrev(i)          (Cooley-Tukey, merged psi twisting),
//   inverse  w_i = psi^-bitrev(i)         (Gentleman-Sande).
// NTT order: A[k] = a(psi^(2 bitrev(k) + 1)), evaluations at odd powers in bit-reversed order.

// One forward round: stages [stage, stage + R) on sub-groups of 2^R elements held in registers.
// The sub-group of thread-slot sg is base | (u << lo), u < 2^R.  At round stage k the twiddle index
// is 2^st + (hb << k) + (u >> (R - k)) with hb = base >> (lo + R): 2^k contiguous twiddles.
// `lazy` counts stages since the last full reduction (uniform across the workgroup).
template <int R, int NT>
__device__ __forceinline__ void fwd_round(double* s, int logn, int stage, int lazy,
                                          const double2* __restrict__ tw, ModD m) {
  const int n = 1 << logn;
  const int lo = logn - stage - R;  // lowest index bit touched by this round
  for (int sg = threadIdx.x; sg < (n >> R); sg += NT) {
    const int base = ((sg >> lo) << (lo + R)) | (sg & ((1 << lo) - 1));
    const int hb = base >> (lo + R);
    double x[1 << R];
#pragma unroll
    for (int u = 0; u < (1 << R); u++) x[u] = s[lpad(base + (u << lo))];
    int lz = lazy;
#pragma unroll
    for (int k = 0; k < R; k++) {
      if (lz >= 2) {
#pragma unroll
        for (int u = 0; u < (1 << R); u++) x[u] = reduce(x[u], m);
        lz = 0;
      }
      const double2* twk = tw + (1 << (stage + k)) + (hb << k);
#pragma unroll
      for (int j = 0; j < (1 << k); j++) {
        const double2 w = twk[j];
#pragma unroll
        for (int v = 0; v < (1 << (R - 1 - k)); v++) {
          const int u = (j << (R - k)) | v;          // bit R-1-k of u is 0
          const int u2 = u | (1 << (R - 1 - k));
          const double t = mul_tw(x[u2], w.x, w.y, m);
          x[u2] = x[u] - t;
          x[u] = x[u] + t;
        }
      }
      lz++;
    }
#pragma unroll
    for (int u = 0; u < (1 << R); u++) s[lpad(base + (u << lo))] = x[u];
  }
}

// Forward negacyclic NTT of one limb resident in LDS: inputs |x| <= q, outputs |x| <= 2.25 q.
// Radix-16 rounds in registers; stage s pairs indices differing in bit logn-1-s.  A stage adds
// at most 0.625 q, so two stages run between full reductions and every twiddle operand stays
// below 1.625 q < 2^51.  The caller synchronises before (data in LDS) and the function ends with
// a barrier.
template <int NT>
__device__ __forceinline__ void lds_ntt_fwd(double* s, int logn, const double2* __restrict__ tw, ModD m) {
  int stage = 0, lazy = 0;
  while (stage < logn) {
    const int R = min(HS_NTT_RADIX_BITS, logn - stage);
    switch (R) {
      case 4: fwd_round<4, NT>(s, logn, stage, lazy, tw, m); break;
      case 3: fwd_round<3, NT>(s, logn, stage, lazy, tw, m); break;
      case 2: fwd_round<2, NT>(s, logn, stage, lazy, tw, m); break;
      default: fwd_round<1, NT>(s, logn, stage, lazy, tw, m); break;
    }
    for (int k = 0; k < R; k++) { if (lazy >= 2) lazy = 0; lazy++; }
    stage += R;
    __syncthreads();
  }
}

// One inverse round: stages [stage, stage + R), lo = stage.  At round stage k the twiddle index is
// (n >> (st + 1)) + (hb << (R - 1 - k)) + (u >> (k + 1)): 2^(R-1-k) contiguous twiddles.
template <int R, int NT>
__device__ __forceinline__ void inv_round(double* s, int logn, int stage, bool last,
                                          const double2* __restrict__ tw, double2 ninv, ModD m) {
  const int n = 1 << logn;
  const int lo = stage;
  for (int sg = threadIdx.x; sg < (n >> R); sg += NT) {
    const int base = ((sg >> lo) << (lo + R)) | (sg & ((1 << lo) - 1));
    const int hb = base >> (lo + R);
    double x[1 << R];
#pragma unroll
    for (int u = 0; u < (1 << R); u++) x[u] = s[lpad(base + (u << lo))];
#pragma unroll
    for (int k = 0; k < R; k++) {
      const int st = stage + k;
      const double2* twk = tw + (n >> (st + 1)) + (hb << (R - 1 - k));
#pragma unroll
      for (int j = 0; j < (1 << (R - 1 - k)); j++) {
        const double2 w = twk[j];
#pragma unroll
        for (int v = 0; v < (1 << k); v++) {
          const int u = (j << (k + 1)) | v;          // bit k of u is 0
          const int u2 = u | (1 << k);
          const double a = x[u], b = x[u2];
          x[u] = reduce(a + b, m);
          x[u2] = mul_tw(a - b, w.x, w.y, m);
        }
      }
    }
    if (last) {
#pragma unroll
      for (int u = 0; u < (1 << R); u++) x[u] = mul_tw(x[u], ninv.x, ninv.y, m);
    }
#pragma unroll
    for (int u = 0; u < (1 << R); u++) s[lpad(base + (u << lo))] = x[u];
  }
}

// Inverse negacyclic NTT of one limb in LDS, including the 1/N scaling: inputs |x| <= q, outputs
// |x| <= 0.625 q.  Stage s pairs indices differing in bit s; X' = reduce(X + Y), Y' = (X - Y) w.
template <int NT>
__device__ __forceinline__ void lds_ntt_inv(double* s, int logn, const double2* __restrict__ tw, double2 ninv, ModD m) {
  int stage = 0;
  while (stage < logn) {
    const int R = min(HS_NTT_RADIX_BITS, logn - stage);
    const bool last = (stage + R == logn);
    switch (R) {
      case 4: inv_round<4, NT>(s, logn, stage, last, tw, ninv, m); break;
      case 3: inv_round<3, NT>(s, logn, stage, last, tw, ninv, m); break;
      case 2: inv_round<2, NT>(s, logn, stage, last, tw, ninv, m); break;
      default: inv_round<1, NT>(s, logn, stage, last, tw, ninv, m); break;
    }
    stage += R;
    __syncthreads();
  }
}

// ---------------------------------------------------------------- compile-time transforms
// For the ring sizes that fill a workgroup (N = 16 NT) every round parameter is a constant:
// element offsets become immediates, the loops unroll fully and the data source of the first round
// and the sink of the last round can be global memory, saving two LDS passes.  Rounds split LOGN
// into ceil(LOGN / 4) near-equal parts (14 -> 4,4,3,3).
//
// Forward reductions run before global stages 2, 5, 8, 11 (inputs |x| <= q): a stage adds at most
// 0.625 q, so twiddle operands stay <= 1.75 q < 2^51 and outputs are |x| <= 2.375 q + 1.

__host__ __device__ constexpr int ilog2c(int x) { return x <= 1 ? 0 : 1 + ilog2c(x >> 1); }
__host__ __device__ constexpr int st_rounds(int logn) { return (logn + 3) / 4; }
__host__ __device__ constexpr int st_rbits(int logn, int r) {  // bits of round r
  return logn / st_rounds(logn) + (r < logn % st_rounds(logn) ? 1 : 0);
}
__host__ __device__ constexpr int st_first(int logn, int r) {  // first stage of round r (forward)
  return r == 0 ? 0 : st_first(logn, r - 1) + st_rbits(logn, r - 1);
}
__host__ __device__ constexpr bool fwd_reduces_before(int st) { return st >= 2 && (st - 2) % 3 == 0; }

// Element access of a round: element base | (u << LO) for u < 2^R, base with zero bits [LO, LO+R).
// In LDS with one pad per 16 doubles the offset of u is the constant X + (X >> 4), X = u << LO.
struct LdsIO {
  double* s;
  template <int R, int LO>
  __device__ __forceinline__ void get(double (&x)[1 << R], int base) const {
    const double* p = s + lpad(base);
#pragma unroll
    for (int u = 0; u < (1 << R); u++) x[u] = p[(u << LO) + ((u << LO) >> 4)];
  }
  template <int R, int LO>
  __device__ __forceinline__ void put(const double (&x)[1 << R], int base) const {
    double* p = s + lpad(base);
#pragma unroll
    for (int u = 0; u < (1 << R); u++) p[(u << LO) + ((u << LO) >> 4)] = x[u];
  }
};
// Canonical u64 residues in global memory.
struct U64In {
  const u64* g;
  template <int R, int LO>
  __device__ __forceinline__ void get(double (&x)[1 << R], int base) const {
#pragma unroll
    for (int u = 0; u < (1 << R); u++) x[u] = u2d(g[base + (u << LO)]);
  }
};
struct U64Out {
  u64* g;
  ModD m;
  template <int R, int LO>
  __device__ __forceinline__ void put(const double (&x)[1 << R], int base) const {
#pragma unroll
    for (int u = 0; u < (1 << R); u++) g[base + (u << LO)] = d2u(canon(x[u], m));
  }
};

// Stages [ST0, ST0 + R) of the forward transform on one register group (hb = base >> (LO + R)).
template <int R, int ST0>
__device__ __forceinline__ void ct_group(double (&x)[1 << R], int hb, const double2* __restrict__ tw, ModD m) {
#pragma unroll
  for (int k = 0; k < R; k++) {
    if (fwd_reduces_before(ST0 + k)) {
#pragma unroll
      for (int u = 0; u < (1 << R); u++) x[u] = reduce(x[u], m);
    }
    const double2* twk = tw + (1 << (ST0 + k)) + (hb << k);
#pragma unroll
    for (int j = 0; j < (1 << k); j++) {
      const double2 w = ldtw(twk, j);
#pragma unroll
      for (int v = 0; v < (1 << (R - 1 - k)); v++) {
        const int u = (j << (R - k)) | v;
        const int u2 = u | (1 << (R - 1 - k));
        const double t = mul_tw(x[u2], w.x, w.y, m);
        x[u2] = x[u] - t;
        x[u] = x[u] + t;
      }
    }
  }
}

// ct_group over the 8-byte twiddle table (w alone, mul_twc): half the twiddle bytes of ct_group,
// with the same reductions (before stages 2, 5, 8, ...).  After a reduction the inputs of the
// next three stages are within q/2 + 1, 1.125 q and 1.91 q (products within 0.625 q, 0.79 q,
// 0.98 q by the bounds of mul_twc) and the third stage's outputs within 2.9 q < 2^52; stages 0
// and 1 take inputs within q and 1.75 q (canonical inputs; stage 0 by either table).  So every
// stage input stays within 1.91 q, whichever stage a round starts at, and a round that ends
// between reductions leaves its outputs within 1.91 q (one stage after one) or 2.9 q.
template <int R, int ST0>
__device__ __forceinline__ void ct_group_c(double (&x)[1 << R], int hb, const double* __restrict__ twc, ModD m) {
#pragma unroll
  for (int k = 0; k < R; k++) {
    if (fwd_reduces_before(ST0 + k)) {
#pragma unroll
      for (int u = 0; u < (1 << R); u++) x[u] = reduce(x[u], m);
    }
    const double __attribute__((address_space(1)))* twk =
        (const double __attribute__((address_space(1)))*)(twc + (1 << (ST0 + k)) + (hb << k));
#pragma unroll
    for (int j = 0; j < (1 << k); j++) {
      const double w = twk[j];
#pragma unroll
      for (int v = 0; v < (1 << (R - 1 - k)); v++) {
        const int u = (j << (R - k)) | v;
        const int u2 = u | (1 << (R - 1 - k));
        const double t = mul_twc(x[u2], w, m);
        x[u2] = x[u] - t;
        x[u] = x[u] + t;
      }
    }
  }
}

// Stages [ST0, ST0 + R) of the inverse transform (Gentleman-Sande, stage s pairs bit s).
template <int R, int ST0, int LOGN, bool LAST>
__device__ __forceinline__ void gs_group(double (&x)[1 << R], int hb, const double2* __restrict__ tw, double2 ninv, ModD m) {
#pragma unroll
  for (int k = 0; k < R; k++) {
    const double2* twk = tw + ((1 << LOGN) >> (ST0 + k + 1)) + (hb << (R - 1 - k));
#pragma unroll
    for (int j = 0; j < (1 << (R - 1 - k)); j++) {
      const double2 w = ldtw(twk, j);
#pragma unroll
      for (int v = 0; v < (1 << k); v++) {
        const int u = (j << (k + 1)) | v;
        const int u2 = u | (1 << k);
        const double a = x[u], b = x[u2];
        x[u] = reduce(a + b, m);
        x[u2] = mul_tw(a - b, w.x, w.y, m);
      }
    }
  }
  if (LAST) {
#pragma unroll
    for (int u = 0; u < (1 << R); u++) x[u] = mul_tw(x[u], ninv.x, ninv.y, m);
  }
}

// Forward stages [ST0, ST0 + R) over TPT tasks per thread starting at task sg0 (a task is the
// register group of element base | (u << LO), LO = LOGN - ST0 - R).
template <int LOGN, int NT, int ST0, int R, int TPT, class In, class Out>
__device__ __forceinline__ void fwd_round_g(const In& in, const Out& out, const double2* __restrict__ tw, ModD m, int sg0, int tid) {
  constexpr int LO = LOGN - ST0 - R;
#pragma unroll
  for (int it = 0; it < TPT; it++) {
    const int sg = sg0 + tid + it * NT;
    const int base = ((sg >> LO) << (LO + R)) | (sg & ((1 << LO) - 1));
    double x[1 << R];
    in.template get<R, LO>(x, base);
    ct_group<R, ST0>(x, sg >> LO, tw, m);
    out.template put<R, LO>(x, base);
  }
}

// fwd_round_g with ct_group_c (8-byte twiddles).
template <int LOGN, int NT, int ST0, int R, int TPT, class In, class Out>
__device__ __forceinline__ void fwd_round_gc(const In& in, const Out& out, const double* __restrict__ twc, ModD m, int sg0, int tid) {
  constexpr int LO = LOGN - ST0 - R;
#pragma unroll
  for (int it = 0; it < TPT; it++) {
    const int sg = sg0 + tid + it * NT;
    const int base = ((sg >> LO) << (LO + R)) | (sg & ((1 << LO) - 1));
    double x[1 << R];
    in.template get<R, LO>(x, base);
    ct_group_c<R, ST0>(x, sg >> LO, twc, m);
    out.template put<R, LO>(x, base);
  }
}

// Inverse stages [ST0, ST0 + R) (stage s pairs bit s, so LO = ST0), same task scheme.
template <int LOGN, int NT, int ST0, int R, int TPT, bool LAST, class In, class Out>
__device__ __forceinline__ void inv_round_g(const In& in, const Out& out, const double2* __restrict__ tw, double2 ninv, ModD m, int sg0, int tid) {
  constexpr int LO = ST0;
#pragma unroll
  for (int it = 0; it < TPT; it++) {
    const int sg = sg0 + tid + it * NT;
    const int base = ((sg >> LO) << (LO + R)) | (sg & ((1 << LO) - 1));
    double x[1 << R];
    in.template get<R, LO>(x, base);
    gs_group<R, LO, LOGN, LAST>(x, sg >> LO, tw, ninv, m);
    out.template put<R, LO>(x, base);
  }
}

// Round r of the whole-limb schedule.
template <int LOGN, int NT, int RD, class In, class Out>
__device__ __forceinline__ void fwd_round_c(const In& in, const Out& out, const double2* __restrict__ tw, ModD m, int tid) {
  constexpr int R = st_rbits(LOGN, RD);
  static_assert((1 << (LOGN - R)) % NT == 0, "round does not tile the workgroup");
  fwd_round_g<LOGN, NT, st_first(LOGN, RD), R, (1 << (LOGN - R)) / NT>(in, out, tw, m, 0, tid);
}
template <int LOGN, int NT, int RD, class In, class Out>
__device__ __forceinline__ void inv_round_c(const In& in, const Out& out, const double2* __restrict__ tw, double2 ninv, ModD m, int tid) {
  constexpr int R = st_rbits(LOGN, RD);
  static_assert((1 << (LOGN - R)) % NT == 0, "round does not tile the workgroup");
  inv_round_g<LOGN, NT, st_first(LOGN, RD), R, (1 << (LOGN - R)) / NT, RD == st_rounds(LOGN) - 1>(in, out, tw, ninv, m, 0, tid);
}

template <int LOGN, int NT, int RD, class In, class Out>
__device__ __forceinline__ void fwd_rounds_from(const In& in, const Out& out, double* s, const double2* __restrict__ tw, ModD m, int tid) {
  constexpr int NR = st_rounds(LOGN);
  if constexpr (NR == 1) {
    fwd_round_c<LOGN, NT, 0>(in, out, tw, m, tid);
  } else if constexpr (RD == 0) {
    fwd_round_c<LOGN, NT, 0>(in, LdsIO{s}, tw, m, tid);
    __syncthreads();
    fwd_rounds_from<LOGN, NT, 1>(in, out, s, tw, m, tid);
  } else if constexpr (RD == NR - 1) {
    fwd_round_c<LOGN, NT, RD>(LdsIO{s}, out, tw, m, tid);
  } else {
    fwd_round_c<LOGN, NT, RD>(LdsIO{s}, LdsIO{s}, tw, m, tid);
    __syncthreads();
    fwd_rounds_from<LOGN, NT, RD + 1>(in, out, s, tw, m, tid);
  }
}

template <int LOGN, int NT, int RD, class In, class Out>
__device__ __forceinline__ void inv_rounds_from(const In& in, const Out& out, double* s, const double2* __restrict__ tw, double2 ninv,
                                                ModD m, int tid) {
  constexpr int NR = st_rounds(LOGN);
  if constexpr (NR == 1) {
    inv_round_c<LOGN, NT, 0>(in, out, tw, ninv, m, tid);
  } else if constexpr (RD == 0) {
    inv_round_c<LOGN, NT, 0>(in, LdsIO{s}, tw, ninv, m, tid);
    __syncthreads();
    inv_rounds_from<LOGN, NT, 1>(in, out, s, tw, ninv, m, tid);
  } else if constexpr (RD == NR - 1) {
    inv_round_c<LOGN, NT, RD>(LdsIO{s}, out, tw, ninv, m, tid);
  } else {
    inv_round_c<LOGN, NT, RD>(LdsIO{s}, LdsIO{s}, tw, ninv, m, tid);
    __syncthreads();
    inv_rounds_from<LOGN, NT, RD + 1>(in, out, s, tw, ninv, m, tid);
  }
}

// Whole transforms, s = LDS of lds_doubles(2^LOGN) doubles.  `tid` is the thread index; a kernel
// running several transforms in a loop passes a copy it has made opaque to the optimiser, so that
// per-thread address arithmetic is recomputed per transform rather than hoisted and held in
// registers across the loop.  The first round reads `in`, the last writes `out` (either may be LdsIO{s}: then the caller synchronises before / after as with the
// runtime-size functions).  No barrier at the end: `out` of the last round is written by the
// thread that computed it.
template <int LOGN, int NT, class In, class Out>
__device__ __forceinline__ void ntt_fwd_c(const In& in, const Out& out, double* s, const double2* __restrict__ tw, ModD m,
                                          int tid = threadIdx.x) {
  fwd_rounds_from<LOGN, NT, 0>(in, out, s, tw, m, tid);
}
template <int LOGN, int NT, class In, class Out>
__device__ __forceinline__ void ntt_inv_c(const In& in, const Out& out, double* s, const double2* __restrict__ tw, double2 ninv, ModD m,
                                          int tid = threadIdx.x) {
  inv_rounds_from<LOGN, NT, 0>(in, out, s, tw, ninv, m, tid);
}

// Element-wise sources and sinks: f(e) -> double (|x| <= q), g(e, x).
template <class F>
struct ElemIn {
  F f;
  template <int R, int LO>
  __device__ __forceinline__ void get(double (&x)[1 << R], int base) const {
#pragma unroll
    for (int u = 0; u < (1 << R); u++) x[u] = f(base + (u << LO));
  }
};
template <class G>
struct ElemOut {
  G g;
  template <int R, int LO>
  __device__ __forceinline__ void put(const double (&x)[1 << R], int base) const {
#pragma unroll
    for (int u = 0; u < (1 << R); u++) g(base + (u << LO), x[u]);
  }
};
template <class F> __device__ __forceinline__ ElemIn<F> elem_in(F f) { return ElemIn<F>{f}; }
template <class G> __device__ __forceinline__ ElemOut<G> elem_out(G g) { return ElemOut<G>{g}; }

// LDS holding one half of a limb (elements with a fixed top index bit, HB = log2 of the half).
template <int HB>
struct LdsHalf {
  double* s;
  template <int R, int LO>
  __device__ __forceinline__ void get(double (&x)[1 << R], int base) const { LdsIO{s}.template get<R, LO>(x, base & ((1 << HB) - 1)); }
  template <int R, int LO>
  __device__ __forceinline__ void put(const double (&x)[1 << R], int base) const { LdsIO{s}.template put<R, LO>(x, base & ((1 << HB) - 1)); }
};

// ---- N = 2^14 with half-limb LDS (68 KiB, two workgroups per CU, NT = 512)
// Forward: stage 0 pairs e with e + 2^13 and is done in registers as the limb is read; the two
// halves are then independent 13-stage problems.  Each thread owns elements tid + 512 k of both
// halves, which is exactly its register group of stages 1..4 (LO = 9), so that round needs no LDS.
// The second half waits in registers while the first runs stages 5..13 through LDS
// (rounds 3,3,3 with two tasks per thread, reading the 8-byte twiddles: ct_group_c, outputs
// within 2.9 q).  Inverse: the mirror image (stages 0..12 per half, stage 13 and the 1/N scaling
// in registers at the end).
static constexpr int kSplitLogn = 14, kSplitNT = 512;
__host__ __device__ constexpr int split_lds_doubles() { return lds_doubles(1 << (kSplitLogn - 1)); }

template <class In, class Out>
__device__ __forceinline__ void ntt_fwd_split(const In& in, const Out& out, double* s, const double2* __restrict__ tw,
                                              const double* __restrict__ twc, ModD m,
                                              int tid = threadIdx.x) {
  constexpr int LOGN = kSplitLogn, NT = kSplitNT, H = 1 << (LOGN - 1), EH = H / NT;
  static_assert(EH == 16, "split layout assumes 16 elements per thread and half");
  double a[EH], b[EH];
  const double2 w1 = ldtw(tw, 1);
#pragma unroll
  for (int k = 0; k < EH; k++) {
    const int e = tid + k * NT;
    a[k] = in(e);
    b[k] = in(e + H);
  }
#pragma unroll
  for (int k = 0; k < EH; k++) {
    const double t = mul_tw(b[k], w1.x, w1.y, m);
    b[k] = a[k] - t;
    a[k] = a[k] + t;
  }
  ct_group<4, 1>(a, 0, tw, m);
  LdsHalf<LOGN - 1>{s}.template put<4, 9>(a, tid);
  __syncthreads();
  fwd_round_gc<LOGN, NT, 5, 3, 2>(LdsHalf<LOGN - 1>{s}, LdsHalf<LOGN - 1>{s}, twc, m, 0, tid);
  __syncthreads();
  fwd_round_gc<LOGN, NT, 8, 3, 2>(LdsHalf<LOGN - 1>{s}, LdsHalf<LOGN - 1>{s}, twc, m, 0, tid);
  __syncthreads();
  fwd_round_gc<LOGN, NT, 11, 3, 2>(LdsHalf<LOGN - 1>{s}, elem_out(out), twc, m, 0, tid);
  __syncthreads();
  ct_group<4, 1>(b, 1, tw, m);
  LdsHalf<LOGN - 1>{s}.template put<4, 9>(b, H + tid);
  __syncthreads();
  fwd_round_gc<LOGN, NT, 5, 3, 2>(LdsHalf<LOGN - 1>{s}, LdsHalf<LOGN - 1>{s}, twc, m, 1 << 10, tid);
  __syncthreads();
  fwd_round_gc<LOGN, NT, 8, 3, 2>(LdsHalf<LOGN - 1>{s}, LdsHalf<LOGN - 1>{s}, twc, m, 1 << 10, tid);
  __syncthreads();
  fwd_round_gc<LOGN, NT, 11, 3, 2>(LdsHalf<LOGN - 1>{s}, elem_out(out), twc, m, 1 << 10, tid);
}

// As ntt_fwd_split, but each half's result stays in LDS and seg(base, count) is called (after a
// barrier) to consume elements base .. base + count - 1, element base + e at s[lpad(e)]; for
// epilogues too heavy to inline into the last round.  Ends with a barrier.
template <class In, class Seg>
__device__ __forceinline__ void ntt_fwd_split_seg(const In& in, const Seg& seg, double* s, const double2* __restrict__ tw,
                                                  const double* __restrict__ twc, ModD m,
                                                  int tid = threadIdx.x) {
  constexpr int LOGN = kSplitLogn, NT = kSplitNT, H = 1 << (LOGN - 1), EH = H / NT;
  double a[EH], b[EH];
  const double2 w1 = ldtw(tw, 1);
#pragma unroll
  for (int k = 0; k < EH; k++) {
    const int e = tid + k * NT;
    a[k] = in(e);
    b[k] = in(e + H);
  }
#pragma unroll
  for (int k = 0; k < EH; k++) {
    const double t = mul_tw(b[k], w1.x, w1.y, m);
    b[k] = a[k] - t;
    a[k] = a[k] + t;
  }
  const LdsHalf<LOGN - 1> L{s};
  ct_group<4, 1>(a, 0, tw, m);
  L.template put<4, 9>(a, tid);
  __syncthreads();
  fwd_round_gc<LOGN, NT, 5, 3, 2>(L, L, twc, m, 0, tid);
  __syncthreads();
  fwd_round_gc<LOGN, NT, 8, 3, 2>(L, L, twc, m, 0, tid);
  __syncthreads();
  fwd_round_gc<LOGN, NT, 11, 3, 2>(L, L, twc, m, 0, tid);
  __syncthreads();
  seg(0, H);
  __syncthreads();
  ct_group<4, 1>(b, 1, tw, m);
  L.template put<4, 9>(b, H + tid);
  __syncthreads();
  fwd_round_gc<LOGN, NT, 5, 3, 2>(L, L, twc, m, 1 << 10, tid);
  __syncthreads();
  fwd_round_gc<LOGN, NT, 8, 3, 2>(L, L, twc, m, 1 << 10, tid);
  __syncthreads();
  fwd_round_gc<LOGN, NT, 11, 3, 2>(L, L, twc, m, 1 << 10, tid);
  __syncthreads();
  seg(H, H);
  __syncthreads();
}

template <class In, class Out>
__device__ __forceinline__ void ntt_inv_split(const In& in, const Out& out, double* s, const double2* __restrict__ tw, double2 ninv, ModD m,
                                              int tid = threadIdx.x) {
  constexpr int LOGN = kSplitLogn, NT = kSplitNT, H = 1 << (LOGN - 1), EH = H / NT;
  static_assert(EH == 16, "split layout assumes 16 elements per thread and half");
  double a[EH], b[EH];
  inv_round_g<LOGN, NT, 0, 3, 2, false>(elem_in(in), LdsHalf<LOGN - 1>{s}, tw, ninv, m, 0, tid);
  __syncthreads();
  inv_round_g<LOGN, NT, 3, 3, 2, false>(LdsHalf<LOGN - 1>{s}, LdsHalf<LOGN - 1>{s}, tw, ninv, m, 0, tid);
  __syncthreads();
  inv_round_g<LOGN, NT, 6, 3, 2, false>(LdsHalf<LOGN - 1>{s}, LdsHalf<LOGN - 1>{s}, tw, ninv, m, 0, tid);
  __syncthreads();
  LdsHalf<LOGN - 1>{s}.template get<4, 9>(a, tid);
  gs_group<4, 9, LOGN, false>(a, 0, tw, ninv, m);
  __syncthreads();
  inv_round_g<LOGN, NT, 0, 3, 2, false>(elem_in(in), LdsHalf<LOGN - 1>{s}, tw, ninv, m, 1 << 10, tid);
  __syncthreads();
  inv_round_g<LOGN, NT, 3, 3, 2, false>(LdsHalf<LOGN - 1>{s}, LdsHalf<LOGN - 1>{s}, tw, ninv, m, 1 << 10, tid);
  __syncthreads();
  inv_round_g<LOGN, NT, 6, 3, 2, false>(LdsHalf<LOGN - 1>{s}, LdsHalf<LOGN - 1>{s}, tw, ninv, m, 1 << 10, tid);
  __syncthreads();
  LdsHalf<LOGN - 1>{s}.template get<4, 9>(b, H + tid);
  gs_group<4, 9, LOGN, false>(b, 1, tw, ninv, m);
  // stage 13 with the scaling merged into its twiddle: w' = w / N mod q
  const double2 w = ldtw(tw, 1);
  const double wn = canon(mul_tw(w.x, ninv.x, ninv.y, m), m);
  const double wnq = wn / m.q;
#pragma unroll
  for (int k = 0; k < EH; k++) {
    const int e = tid + k * NT;
    const double x = a[k], y = b[k];
    out(e, mul_tw(x + y, ninv.x, ninv.y, m));
    out(e + H, mul_tw(x - y, wn, wnq, m));
  }
}

// Ring size handled by the compile-time path for a workgroup of NT threads (0: runtime path).
__host__ __device__ constexpr int static_logn(int nt) { return nt >= 128 ? ilog2c(nt) + 4 : 0; }

// ---------------------------------------------------------------- ChaCha20 (RFC 8439)
__device__ __forceinline__ u32 rotl32(u32 v, int c) { return (v << c) | (v >> (32 - c)); }

// One 64-byte block: key = (seed lo, seed hi, 0 x 6), counter = block, nonce = (purpose,
// index lo, index hi).
__device__ inline void chacha_block(u64 seed, u32 purpose, u64 index, u32 block, u32 out[16]) {
  const u32 init[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u,
                        (u32)seed, (u32)(seed >> 32), 0u, 0u, 0u, 0u, 0u, 0u,
                        block, purpose, (u32)index, (u32)(index >> 32)};
  u32 x[16];
#pragma unroll
  for (int i = 0; i < 16; i++) x[i] = init[i];
#define HS_QR(a, b, c, d)                         \
  x[a] += x[b]; x[d] = rotl32(x[d] ^ x[a], 16);   \
  x[c] += x[d]; x[b] = rotl32(x[b] ^ x[c], 12);   \
  x[a] += x[b]; x[d] = rotl32(x[d] ^ x[a], 8);    \
  x[c] += x[d]; x[b] = rotl32(x[b] ^ x[c], 7);
#pragma unroll
  for (int r = 0; r < 10; r++) {
    HS_QR(0, 4, 8, 12) HS_QR(1, 5, 9, 13) HS_QR(2, 6, 10, 14) HS_QR(3, 7, 11, 15)
    HS_QR(0, 5, 10, 15) HS_QR(1, 6, 11, 12) HS_QR(2, 7, 8, 13) HS_QR(3, 4, 9, 14)
  }
#undef HS_QR
#pragma unroll
  for (int i = 0; i < 16; i++) out[i] = x[i] + init[i];
}

}  // namespace hs
