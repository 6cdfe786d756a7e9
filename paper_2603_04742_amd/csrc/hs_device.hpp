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

// Balanced value (|x| < 2^52) -> canonical residue in [0, q).
__device__ __forceinline__ double canon(double x, ModD m) {
  double r = reduce(x, m);
  return r < 0.0 ? r + m.q : r;
}

__device__ __forceinline__ double u2d(u64 x) { return (double)x; }           // x < 2^53
__device__ __forceinline__ u64 d2u(double x) { return (u64)x; }              // 0 <= x < 2^53

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
__device__ void lds_ntt_fwd(double* s, int logn, const double2* __restrict__ tw, ModD m) {
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
__device__ void lds_ntt_inv(double* s, int logn, const double2* __restrict__ tw, double2 ninv, ModD m) {
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
