// Exact BFV ciphertext product (both operands encrypted): the scaled tensor
//   (d0, d1, d2) = round(t/Q * (a0 b0, a0 b1 + a1 b0, a1 b1))  mod Q
// of the centered lifts a_i, b_j in (-Q/2, Q/2), with the products taken exactly: the lifts are
// reduced to a tensor basis of T primes (data, special and extra primes, product M > 4 N Q^2), the
// negacyclic products are formed in NTT form there, and each coefficient is reconstructed by CRT
// as an integer in (-M/2, M/2) before the exact rounding.  Per-coefficient multiword arithmetic in
// 64-bit words; the division by 2Q uses a Barrett reciprocal.
//
// The kernels are instantiated for a word capacity KW (8, 16 or 24) chosen by the context: every
// multiword loop is unrolled to KW and predicated on the value's runtime width, so each word has a
// compile-time index and the values stay in registers (with runtime indices they would live in
// private scratch memory, whose traffic dominated these kernels).  The Barrett reciprocal is
// floor(2^(64 KW) / 2Q), which puts the quotient at the fixed word offset KW of the product.
#include <utility>

#include "hs_device.hpp"
#include "kernels.hpp"

namespace hs {

__device__ __forceinline__ ModD mody(const ModTab& t) { return ModD{t.q, t.qinv}; }

// f(std::integral_constant<int, I>) for I = 0 .. N-1, expanded at compile time (the nested word
// loops below are too long for the loop unroller to flatten on its own)
template <class F, int... I>
__device__ __forceinline__ void static_for_seq(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// the 128-bit product a b from four 32 x 32 -> 64 multiply-adds (no partial sum exceeds 2^64 - 1)
__device__ __forceinline__ void mul128(u64 a, u64 b, u64& lo, u64& hi) {
  const u64 a0 = (u32)a, a1 = a >> 32, b0 = (u32)b, b1 = b >> 32;
  const u64 p0 = a0 * b0;
  const u64 p1 = a0 * b1 + (p0 >> 32);
  const u64 p2 = a1 * b0 + (u32)p1;
  hi = a1 * b1 + (p1 >> 32) + (p2 >> 32);
  lo = (p2 << 32) | (u32)p0;
}

// acc += a[0..W) * v, the carry running through the words of acc above W
template <int KW>
__device__ __forceinline__ void mw_mac(u64 (&acc)[KW], const u64* a, int W, u64 v) {
  u64 carry = 0;
#pragma unroll
  for (int w = 0; w < KW; w++) {
    if (w < W) {
      u64 lo, hi;
      mul128(a[w], v, lo, hi);
      const u64 s1 = acc[w] + lo;
      const u64 c1 = s1 < lo;
      const u64 s2 = s1 + carry;
      const u64 c2 = s2 < carry;
      acc[w] = s2;
      carry = hi + c1 + c2;
    } else {
      const u64 s = acc[w] + carry;
      carry = s < carry;
      acc[w] = s;
    }
  }
}
// sign of a - b over the low W words (b: device words)
template <int KW>
__device__ __forceinline__ int mw_cmp(const u64 (&a)[KW], const u64* b, int W) {
  int r = 0;
#pragma unroll
  for (int w = KW - 1; w >= 0; w--)
    if (w < W && r == 0) {
      const u64 y = b[w];
      if (a[w] != y) r = a[w] < y ? -1 : 1;
    }
  return r;
}
// a -= b over the low W words (a >= b)
template <int KW>
__device__ __forceinline__ void mw_sub(u64 (&a)[KW], const u64* b, int W) {
  u64 br = 0;
#pragma unroll
  for (int w = 0; w < KW; w++)
    if (w < W) {
      const u64 x = a[w], y = b[w];
      const u64 d = x - y;
      const u64 b1 = x < y;
      const u64 d2 = d - br;
      const u64 b2 = d < br;
      a[w] = d2;
      br = b1 | b2;
    }
}
// a = b - a over the low W words (b >= a)
template <int KW>
__device__ __forceinline__ void mw_rsub(u64 (&a)[KW], const u64* b, int W) {
  u64 br = 0;
#pragma unroll
  for (int w = 0; w < KW; w++)
    if (w < W) {
      const u64 x = b[w], y = a[w];
      const u64 d = x - y;
      const u64 b1 = x < y;
      const u64 d2 = d - br;
      const u64 b2 = d < br;
      a[w] = d2;
      br = b1 | b2;
    }
}
// value of the low W words mod q: Horner over 32-bit digits from the top, r = r 2^32 + digit
// with r32 = 2^32 mod q, no integer division (|r| stays below 0.625 q + 2^32 < 2^51)
template <int KW>
__device__ __forceinline__ u64 mw_mod(const u64 (&a)[KW], int W, double2 r32, ModD m) {
  double r = 0.0;
#pragma unroll
  for (int w = KW - 1; w >= 0; w--)
    if (w < W) {
      r = mul_tw(r, r32.x, r32.y, m) + (double)(u32)(a[w] >> 32);
      r = mul_tw(r, r32.x, r32.y, m) + (double)(u32)a[w];
    }
  return d2u(canon(r, m));
}
// (c0, c1, c2) += x * y
__device__ __forceinline__ void acc3(u64& c0, u64& c1, u64& c2, u64 x, u64 y) {
  u64 lo, hi;
  mul128(x, y, lo, hi);
  c0 += lo;
  const u64 k0 = c0 < lo;
  c1 += hi;
  const u64 k1 = c1 < hi;
  c1 += k0;
  const u64 k2 = c1 < k0;
  c2 += k1 + k2;
}

// Centered lift of data-prime residues to the T tensor moduli.  x: [rows][L][N] coefficient form;
// out: [rows][T][N].  grid-stride over rows * N coefficients.  The constant tables sit in LDS; a
// nonzero WQc fixes the word width at compile time.
template <int KW, int WQc = 0>
__global__ void __launch_bounds__(256) k_crt_lift(const u64* __restrict__ x, u64* out, int rows, TensorConst C,
                                                  const ModTab* __restrict__ tab, int logn) {
  const i64 n = 1 << logn;
  const i64 total = (i64)rows * n;
  extern __shared__ __align__(16) u64 cl_lds[];
  const int L = C.L, T = C.T, WQ = WQc ? WQc : C.WQ;
  u64* l_qhat = cl_lds;                  // [L][WQ]
  u64* l_Q = l_qhat + (size_t)L * WQ;    // [WQ]
  u64* l_halfQ = l_Q + WQ;               // [WQ]
  const int nu = L * WQ + 2 * WQ;        // u64 words above, padded to 16 bytes
  double2* l_qm = (double2*)(cl_lds + nu + (nu & 1));  // (q, 1/q) [T]
  double2* l_qinv = l_qm + T;            // (Q/q_i)^-1 mod q_i [L]
  double2* l_r32 = l_qinv + L;           // [T]
  for (int i = threadIdx.x; i < L * WQ; i += blockDim.x) l_qhat[i] = C.qhat[i];
  for (int i = threadIdx.x; i < WQ; i += blockDim.x) { l_Q[i] = C.Q[i]; l_halfQ[i] = C.halfQ[i]; }
  for (int i = threadIdx.x; i < T; i += blockDim.x) {
    l_qm[i] = double2{tab[i].q, tab[i].qinv};
    l_r32[i] = C.r32[i];
    if (i < L) l_qinv[i] = C.qhat_inv[i];
  }
  __syncthreads();
  for (i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x; idx < total; idx += (i64)gridDim.x * blockDim.x) {
    const i64 row = idx >> logn, k = idx & (n - 1);
    const u64* xr = x + (size_t)row * L * n;
    // S = sum_i [x_i (Q/q_i)^-1]_{q_i} Q/q_i  (< L Q), then S mod Q
    u64 S[KW];
#pragma unroll
    for (int w = 0; w < KW; w++) S[w] = 0;
    for (int i = 0; i < L; i++) {
      const double2 qm = l_qm[i], qi = l_qinv[i];
      const ModD m{qm.x, qm.y};
      const u64 y = d2u(canon(mul_tw(u2d(xr[(size_t)i * n + k]), qi.x, qi.y, m), m));
      mw_mac<KW>(S, l_qhat + (size_t)i * WQ, WQ, y);
    }
    for (int guard = 0; guard <= L; guard++) {
      if (mw_cmp<KW>(S, l_Q, WQ) < 0) break;
      mw_sub<KW>(S, l_Q, WQ);
    }
    const bool neg = mw_cmp<KW>(S, l_halfQ, WQ) > 0;
    if (neg) mw_rsub<KW>(S, l_Q, WQ);  // magnitude Q - S
    u64* o = out + (size_t)row * T * n;
    for (int mi = 0; mi < T; mi++) {
      if (mi < L) { o[(size_t)mi * n + k] = xr[(size_t)mi * n + k]; continue; }
      const double2 qm = l_qm[mi];
      const ModD m{qm.x, qm.y};
      const u64 q = (u64)qm.x;
      const u64 r = mw_mod<KW>(S, WQ, l_r32[mi], m);
      o[(size_t)mi * n + k] = neg ? (r ? q - r : 0) : r;
    }
  }
}

// NTT-domain products: lifted [item][4][T][N] (a0, a1, b0, b1) -> [item][3][T][N].
__global__ void k_tensor(const u64* __restrict__ lift, u64* prod, int items, int T, const ModTab* __restrict__ tab, int logn) {
  const i64 n = 1 << logn;
  const i64 total = (i64)items * T * n;
  for (i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x; idx < total; idx += (i64)gridDim.x * blockDim.x) {
    const i64 k = idx & (n - 1);
    const i64 r = idx >> logn;
    const int mi = (int)(r % T), it = (int)(r / T);
    const ModD m = mody(tab[mi]);
    const u64* L4 = lift + (size_t)it * 4 * T * n;
    const double a0 = u2d(L4[((size_t)0 * T + mi) * n + k]), a1 = u2d(L4[((size_t)1 * T + mi) * n + k]);
    const double b0 = u2d(L4[((size_t)2 * T + mi) * n + k]), b1 = u2d(L4[((size_t)3 * T + mi) * n + k]);
    u64* P = prod + (size_t)it * 3 * T * n;
    P[((size_t)0 * T + mi) * n + k] = d2u(canon(mulmod(a0, b0, m), m));
    P[((size_t)1 * T + mi) * n + k] = d2u(canon(mulmod(a0, b1, m) + mulmod(a1, b0, m), m));
    P[((size_t)2 * T + mi) * n + k] = d2u(canon(mulmod(a1, b1, m), m));
  }
}

// Scale and round: prod [item][3][T][N] coefficient form -> out [item][4][L][N] coefficient form
// laid out (d0, d2, 0, d1) so that (d0, d2) is the ciphertext to relinearise and (0, d1) its addend.
// (registers over occupancy: the widest instantiation holds about 60 live words per lane)
// Optional compile-time word widths (0: the context's runtime values) fold the width predicates.
template <int KW, int WMc = 0, int WAc = 0, int WDc = 0, int WMUc = 0, int WQc = 0>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) k_scale_round(const u64* __restrict__ prod, u64* out, int items, TensorConst C,
                                                     const ModTab* __restrict__ tab, int logn) {
  const i64 n = 1 << logn;
  const i64 total = (i64)items * 3 * n;
  // the constant tables in LDS, once per workgroup (read word by word in the loops below)
  extern __shared__ __align__(16) u64 tc_lds[];
  const int T = C.T;
  const int WM = WMc ? WMc : C.WM, WA = WAc ? WAc : C.WA, WD = WDc ? WDc : C.WD;
  const int WMU = WMUc ? WMUc : C.WMU, WQ = WQc ? WQc : C.WQ;
  u64* l_mhat = tc_lds;                  // [T][WM]
  u64* l_M = l_mhat + (size_t)T * WM;    // [WM + 1]
  u64* l_halfM = l_M + (WM + 1);         // [WM]
  u64* l_mu = l_halfM + WM;              // [WMU + 1]
  u64* l_D = l_mu + (WMU + 1);         // [WD]
  u64* l_Q = l_D + WD;                 // [WQ]
  const int nu = T * WM + 2 * WM + 2 + WMU + WD + WQ;   // u64 words above, padded to 16 bytes
  double2* l_qm = (double2*)(tc_lds + nu + (nu & 1));            // (q, 1/q) [T]
  double2* l_minv = l_qm + T;            // [T]
  double2* l_r32 = l_minv + T;           // [T]
  for (int i = threadIdx.x; i < T * WM; i += blockDim.x) l_mhat[i] = C.mhat[i];
  for (int i = threadIdx.x; i < WM + 1; i += blockDim.x) l_M[i] = C.M[i];
  for (int i = threadIdx.x; i < WM; i += blockDim.x) l_halfM[i] = C.halfM[i];
  for (int i = threadIdx.x; i < WMU + 1; i += blockDim.x) l_mu[i] = C.mu[i];
  for (int i = threadIdx.x; i < WD; i += blockDim.x) l_D[i] = C.D[i];
  for (int i = threadIdx.x; i < WQ; i += blockDim.x) l_Q[i] = C.Q[i];
  for (int i = threadIdx.x; i < T; i += blockDim.x) {
    l_qm[i] = double2{tab[i].q, tab[i].qinv};
    l_minv[i] = C.mhat_inv[i];
    l_r32[i] = C.r32[i];
  }
  __syncthreads();
  for (i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x; idx < total; idx += (i64)gridDim.x * blockDim.x) {
    const i64 k = idx & (n - 1);
    const i64 r = idx >> logn;
    const int w = (int)(r % 3), it = (int)(r / 3);
    const u64* P = prod + ((size_t)it * 3 + w) * C.T * n;
    // X = sum_m [x_m Mhat_m^-1]_m Mhat_m  - floor(sum_m y_m / m) M
    u64 S[KW];
#pragma unroll
    for (int i = 0; i < KW; i++) S[i] = 0;
    double est = 0.0;
    for (int mi = 0; mi < T; mi++) {
      const double2 qm = l_qm[mi], mv = l_minv[mi];
      const ModD m{qm.x, qm.y};
      const u64 y = d2u(canon(mul_tw(u2d(P[(size_t)mi * n + k]), mv.x, mv.y, m), m));
      mw_mac<KW>(S, l_mhat + (size_t)mi * WM, WM, y);
      est += (double)y * qm.y;  // error ~1e-13: the estimate minus one stays a lower bound
    }
    u64 kq = (u64)est;
    if (kq > 0) kq -= 1;  // never above the true quotient; the loop below finishes it
    if (kq) {             // S -= kq M over WM + 1 words (M is stored with WM + 1)
      u64 carry = 0, br = 0;
#pragma unroll
      for (int i = 0; i < KW; i++)
        if (i < WM + 1) {
          u64 lo, hi;
          mul128(l_M[i], kq, lo, hi);
          const u64 p = lo + carry;
          carry = hi + (p < lo);
          const u64 d = S[i] - p;
          const u64 b1 = S[i] < p;
          const u64 d2 = d - br;
          const u64 b2 = d < br;
          S[i] = d2;
          br = b1 | b2;
        }
    }
#pragma unroll
    for (int guard = 0; guard < 4; guard++)
      if (mw_cmp<KW>(S, l_M, WM + 1) >= 0) mw_sub<KW>(S, l_M, WM + 1);
    const bool neg = mw_cmp<KW>(S, l_halfM, WM) > 0;
    if (neg) mw_rsub<KW>(S, l_M, WM);  // |X| = M - S
    // A = 2 t |X| + Q  (WA words, below 2^(64 KW))
    u64 A[KW];
#pragma unroll
    for (int i = 0; i < KW; i++) A[i] = 0;
    {
      u64 carry = 0;
      const u64 v = 2 * C.t;
#pragma unroll
      for (int i = 0; i < KW; i++)
        if (i < WM) {
          u64 lo, hi;
          mul128(S[i], v, lo, hi);
          const u64 s = lo + carry;
          carry = hi + (s < lo);
          A[i] = s;
        } else if (i == WM) {
          A[i] = carry;
        }
      carry = 0;
#pragma unroll
      for (int i = 0; i < KW; i++)
        if (i < WA) {
          const u64 qv = i < WQ ? l_Q[i] : 0;
          const u64 s1 = A[i] + qv;
          const u64 c1 = s1 < qv;
          const u64 s2 = s1 + carry;
          const u64 c2 = s2 < carry;
          A[i] = s2;
          carry = c1 + c2;
        }
    }
    // quotient estimate floor(A mu / 2^(64 KW)): words KW .. 2 KW of the product, by columns
    u64 qe[KW + 1];
    {
      u64 c0 = 0, c1 = 0, c2 = 0;
      static_for<2 * KW>([&](auto cc) {
        constexpr int col = decltype(cc)::value;
        static_for<KW>([&](auto ic) {
          constexpr int i = decltype(ic)::value;
          constexpr int j = col - i;
          if constexpr (j >= 0 && j < KW) {
            if (i < WA && j < WMU) acc3(c0, c1, c2, A[i], l_mu[j]);
          }
        });
        if constexpr (col >= KW) qe[col - KW] = c0;
        c0 = c1; c1 = c2; c2 = 0;
      });
      qe[KW] = c0;
    }
    // R = A - qe * 2Q, kept in the low WD + 1 words of A (0 <= R < 3 (2Q)); then fix the quotient
    {
      u64 c0 = 0, c1 = 0, c2 = 0, br = 0;
      static_for<KW>([&](auto cc) {
        constexpr int col = decltype(cc)::value;
        if (col <= WD) {
          static_for<col + 1>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            constexpr int i = col - j;
            if (i < WD && j <= WMU) acc3(c0, c1, c2, qe[j], l_D[i]);
          });
          const u64 x = A[col];
          const u64 d = x - c0;
          const u64 b1 = x < c0;
          const u64 d2 = d - br;
          const u64 b2 = d < br;
          A[col] = d2;
          br = b1 | b2;
          c0 = c1; c1 = c2; c2 = 0;
        }
      });
#pragma unroll
      for (int guard = 0; guard < 4; guard++) {
        // R >= 2Q over WD + 1 words (the word of 2Q above WD is zero)
        int cmp = 0;
#pragma unroll
        for (int i = KW - 1; i >= 0; i--)
          if (i <= WD && cmp == 0) {
            const u64 y = i < WD ? l_D[i] : 0;
            if (A[i] != y) cmp = A[i] < y ? -1 : 1;
          }
        if (cmp < 0) break;
        u64 bb = 0;
#pragma unroll
        for (int i = 0; i < KW; i++)
          if (i <= WD) {
            const u64 x = A[i], y = i < WD ? l_D[i] : 0;
            const u64 d = x - y;
            const u64 b1 = x < y;
            const u64 d2 = d - bb;
            const u64 b2 = d < bb;
            A[i] = d2;
            bb = b1 | b2;
          }
        u64 inc = 1;
#pragma unroll
        for (int i = 0; i <= KW; i++) {  // qe += 1
          const u64 s = qe[i] + inc;
          inc = s < inc;
          qe[i] = s;
        }
      }
    }
    // residues of the rounded quotient (negated for a negative X)
    const int slot = (w == 0) ? 0 : (w == 1 ? 3 : 1);  // (d0, d2, 0, d1)
    u64* o = out + ((size_t)it * 4 + slot) * C.L * n;
    u64* z = out + ((size_t)it * 4 + 2) * C.L * n;
    for (int i = 0; i < C.L; i++) {
      const double2 qm = l_qm[i];
      const ModD m{qm.x, qm.y};
      const u64 q = (u64)qm.x;
      const u64 rr = mw_mod<KW + 1>(qe, WMU + 1, l_r32[i], m);
      o[(size_t)i * n + k] = neg ? (rr ? q - rr : 0) : rr;
      if (w == 0) z[(size_t)i * n + k] = 0;
    }
  }
}

// ------------------------------------------------------------------ launchers
static dim3 grid_t(i64 total) { return dim3((unsigned)std::min<i64>((total + 255) / 256, 256 * 32)); }

void launch_crt_lift(const hs_ctx* c, const TensorConst& C, const u64* x, u64* out, int rows, hipStream_t st) {
  if (rows <= 0) return;
  ProfScope _prof("k_crt_lift", st);
  const size_t u64s = (size_t)C.L * C.WQ + 2 * C.WQ;
  const size_t lds = 8 * (u64s + (u64s & 1)) + 16 * (2 * (size_t)C.T + C.L);   // the tables staged by k_crt_lift
  const dim3 grid = grid_t((i64)rows * c->N);
  const ModTab* tab = (const ModTab*)c->d_tab;
  if (C.kw == 24 && C.WQ == 11) hipLaunchKernelGGL((k_crt_lift<24, 11>), grid, dim3(256), lds, st, x, out, rows, C, tab, c->logn);
  else if (C.kw == 8) hipLaunchKernelGGL(k_crt_lift<8>, grid, dim3(256), lds, st, x, out, rows, C, tab, c->logn);
  else if (C.kw == 16) hipLaunchKernelGGL(k_crt_lift<16>, grid, dim3(256), lds, st, x, out, rows, C, tab, c->logn);
  else if (C.kw == 24) hipLaunchKernelGGL(k_crt_lift<24>, grid, dim3(256), lds, st, x, out, rows, C, tab, c->logn);
  else throw ::hs::Error{HS_EPARAM, "no tensor kernel for this word capacity"};
  HS_CHECK_HIP(hipGetLastError());
}
void launch_tensor(const hs_ctx* c, const u64* lift, u64* prod, int items, int T, hipStream_t st) {
  if (items <= 0) return;
  ProfScope _prof("k_tensor", st);
  hipLaunchKernelGGL(k_tensor, grid_t((i64)items * T * c->N), dim3(256), 0, st, lift, prod, items, T, (const ModTab*)c->d_tab, c->logn);
  HS_CHECK_HIP(hipGetLastError());
}
void launch_scale_round(const hs_ctx* c, const TensorConst& C, const u64* prod, u64* out, int items, hipStream_t st) {
  if (items <= 0) return;
  ProfScope _prof("k_scale_round", st);
  const size_t u64s = (size_t)C.T * C.WM + 2 * C.WM + 2 + C.WMU + C.WD + C.WQ;
  const size_t lds = 8 * (u64s + (u64s & 1)) + 3 * 16 * (size_t)C.T;   // the tables staged by k_scale_round
  const dim3 grid = grid_t((i64)items * 3 * c->N);
  // 12 x 50-bit data primes (N = 1024 ... 32768, 2 special primes): the widths at compile time
  if (C.kw == 24 && C.WM == 21 && C.WA == 21 && C.WD == 10 && C.WMU == 15 && C.WQ == 11)
    hipLaunchKernelGGL((k_scale_round<24, 21, 21, 10, 15, 11>), grid, dim3(256), lds, st, prod, out, items, C, (const ModTab*)c->d_tab, c->logn);
  else if (C.kw == 8) hipLaunchKernelGGL(k_scale_round<8>, grid, dim3(256), lds, st, prod, out, items, C, (const ModTab*)c->d_tab, c->logn);
  else if (C.kw == 16) hipLaunchKernelGGL(k_scale_round<16>, grid, dim3(256), lds, st, prod, out, items, C, (const ModTab*)c->d_tab, c->logn);
  else if (C.kw == 24) hipLaunchKernelGGL(k_scale_round<24>, grid, dim3(256), lds, st, prod, out, items, C, (const ModTab*)c->d_tab, c->logn);
  else throw ::hs::Error{HS_EPARAM, "no tensor kernel for this word capacity"};
  HS_CHECK_HIP(hipGetLastError());
}

}  // namespace hs
