// Exact BFV ciphertext product (both operands encrypted): the scaled tensor
//   (d0, d1, d2) = round(t/Q * (a0 b0, a0 b1 + a1 b0, a1 b1))  mod Q
// of the centered lifts a_i, b_j in (-Q/2, Q/2), with the products taken exactly: the lifts are
// reduced to a tensor basis of T primes (data, special and extra primes, product M > 4 N Q^2), the
// negacyclic products are formed in NTT form there, and each coefficient is reconstructed by CRT
// as an integer in (-M/2, M/2) before the exact rounding.  Per-coefficient multiword arithmetic in
// 64-bit words; the division by 2Q uses a Barrett reciprocal.
#include "hs_device.hpp"
#include "kernels.hpp"

namespace hs {

static constexpr int kMaxW = 24;  // words of the largest multiword value (A = 2 t |X| + Q)

__device__ __forceinline__ ModD mody(const ModTab& t) { return ModD{t.q, t.qinv}; }

// acc[0..W) += a[0..W) * v  (returns nothing; acc must have room for the carry)
__device__ __forceinline__ void mw_mac(u64* acc, const u64* a, int W, u64 v) {
  u64 carry = 0;
  for (int w = 0; w < W; w++) {
    const u64 lo = a[w] * v, hi = __umul64hi(a[w], v);
    const u64 s1 = acc[w] + lo;
    const u64 c1 = s1 < lo;
    const u64 s2 = s1 + carry;
    const u64 c2 = s2 < carry;
    acc[w] = s2;
    carry = hi + c1 + c2;
  }
  for (int w = W; carry && w < kMaxW; w++) {
    const u64 s = acc[w] + carry;
    carry = s < carry;
    acc[w] = s;
  }
}
__device__ __forceinline__ int mw_cmp(const u64* a, const u64* b, int W) {
  for (int w = W - 1; w >= 0; w--)
    if (a[w] != b[w]) return a[w] < b[w] ? -1 : 1;
  return 0;
}
__device__ __forceinline__ void mw_sub(u64* a, const u64* b, int W) {  // a -= b, a >= b
  u64 br = 0;
  for (int w = 0; w < W; w++) {
    const u64 x = a[w], y = b[w];
    const u64 d = x - y;
    const u64 b1 = x < y;
    const u64 d2 = d - br;
    const u64 b2 = d < br;
    a[w] = d2;
    br = b1 | b2;
  }
}
// value mod q for a multiword value (Horner from the top word)
__device__ __forceinline__ u64 mw_mod(const u64* a, int W, u64 q, double2 r64, ModD m) {
  double r = 0.0;
  for (int w = W - 1; w >= 0; w--) r = canon(mul_tw(r, r64.x, r64.y, m) + u2d(a[w] % q), m);
  return d2u(r);
}

// Centered lift of data-prime residues to the T tensor moduli.  x: [rows][L][N] coefficient form;
// out: [rows][T][N].  grid-stride over rows * N coefficients.
__global__ void k_crt_lift(const u64* __restrict__ x, u64* out, int rows, TensorConst C, const ModTab* __restrict__ tab, int logn) {
  const i64 n = 1 << logn;
  const i64 total = (i64)rows * n;
  for (i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x; idx < total; idx += (i64)gridDim.x * blockDim.x) {
    const i64 row = idx >> logn, k = idx & (n - 1);
    const u64* xr = x + (size_t)row * C.L * n;
    u64 S[kMaxW];
    for (int w = 0; w < C.WQ + 1; w++) S[w] = 0;
    for (int i = 0; i < C.L; i++) {
      const ModTab tb = tab[i];
      const ModD m = mody(tb);
      const u64 y = d2u(canon(mul_tw(u2d(xr[(size_t)i * n + k]), C.qhat_inv[i].x, C.qhat_inv[i].y, m), m));
      mw_mac(S, C.qhat + (size_t)i * C.WQ, C.WQ, y);
    }
    for (int guard = 0; guard <= C.L && mw_cmp(S, C.Q, C.WQ) >= 0; guard++) mw_sub(S, C.Q, C.WQ);
    const bool neg = mw_cmp(S, C.halfQ, C.WQ) > 0;
    if (neg) {  // mag = Q - S
      u64 t[kMaxW];
      for (int w = 0; w < C.WQ; w++) t[w] = C.Q[w];
      mw_sub(t, S, C.WQ);
      for (int w = 0; w < C.WQ; w++) S[w] = t[w];
    }
    u64* o = out + (size_t)row * C.T * n;
    for (int mi = 0; mi < C.T; mi++) {
      if (mi < C.L) { o[(size_t)mi * n + k] = xr[(size_t)mi * n + k]; continue; }
      const ModTab tb = tab[mi];
      const ModD m = mody(tb);
      const u64 q = (u64)tb.q;
      const u64 r = mw_mod(S, C.WQ, q, C.r64[mi], m);
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
__global__ void k_scale_round(const u64* __restrict__ prod, u64* out, int items, TensorConst C, const ModTab* __restrict__ tab, int logn) {
  const i64 n = 1 << logn;
  const i64 total = (i64)items * 3 * n;
  for (i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x; idx < total; idx += (i64)gridDim.x * blockDim.x) {
    const i64 k = idx & (n - 1);
    const i64 r = idx >> logn;
    const int w = (int)(r % 3), it = (int)(r / 3);
    const u64* P = prod + ((size_t)it * 3 + w) * C.T * n;
    // X = sum_m [x_m Mhat_m^-1]_m Mhat_m  - floor(sum_m y_m / m) M
    u64 S[kMaxW];
    for (int i = 0; i < kMaxW; i++) S[i] = 0;
    double est = 0.0;
    for (int mi = 0; mi < C.T; mi++) {
      const ModTab tb = tab[mi];
      const ModD m = mody(tb);
      const u64 y = d2u(canon(mul_tw(u2d(P[(size_t)mi * n + k]), C.mhat_inv[mi].x, C.mhat_inv[mi].y, m), m));
      mw_mac(S, C.mhat + (size_t)mi * C.WM, C.WM, y);
      est += (double)y / tb.q;
    }
    u64 kq = (u64)est;
    if (kq > 0) kq -= 1;  // never above the true quotient; the loop below finishes it
    if (kq) {
      u64 t[kMaxW];
      for (int i = 0; i < kMaxW; i++) t[i] = 0;
      mw_mac(t, C.M, C.WM, kq);
      mw_sub(S, t, C.WM + 1);
    }
    for (int guard = 0; guard < 4 && mw_cmp(S, C.M, C.WM + 1) >= 0; guard++) mw_sub(S, C.M, C.WM + 1);
    const bool neg = mw_cmp(S, C.halfM, C.WM) > 0;
    if (neg) {
      u64 t[kMaxW];
      for (int i = 0; i < C.WM; i++) t[i] = C.M[i];
      mw_sub(t, S, C.WM);
      for (int i = 0; i < C.WM; i++) S[i] = t[i];
    }
    // A = 2 t |X| + Q
    u64 A[kMaxW];
    for (int i = 0; i < kMaxW; i++) A[i] = 0;
    mw_mac(A, S, C.WM, 2 * C.t);
    {
      u64 q2[kMaxW];
      for (int i = 0; i < kMaxW; i++) q2[i] = i < C.WQ ? C.Q[i] : 0;
      u64 carry = 0;
      for (int i = 0; i < C.WA; i++) {
        const u64 s1 = A[i] + q2[i];
        const u64 c1 = s1 < q2[i];
        const u64 s2 = s1 + carry;
        const u64 c2 = s2 < carry;
        A[i] = s2;
        carry = c1 + c2;
      }
    }
    // quotient estimate floor(A mu / 2^(64 WA)), then fix with remainders (at most 2 steps)
    u64 qe[kMaxW];
    for (int i = 0; i < kMaxW; i++) qe[i] = 0;
    {
      // top words of A * mu: word WA + j of the product, j = 0 .. WMU
      u64 prodw[2 * kMaxW + 2];
      for (int i = 0; i < C.WA + C.WMU + 1; i++) prodw[i] = 0;
      for (int i = 0; i < C.WA; i++) {
        u64 carry = 0;
        for (int j = 0; j < C.WMU; j++) {
          const u64 lo = A[i] * C.mu[j], hi = __umul64hi(A[i], C.mu[j]);
          const u64 s1 = prodw[i + j] + lo;
          const u64 c1 = s1 < lo;
          const u64 s2 = s1 + carry;
          const u64 c2 = s2 < carry;
          prodw[i + j] = s2;
          carry = hi + c1 + c2;
        }
        prodw[i + C.WMU] += carry;
      }
      for (int j = 0; j < kMaxW && C.WA + j < C.WA + C.WMU + 1; j++) qe[j] = prodw[C.WA + j];
    }
    {
      u64 R[kMaxW], QD[kMaxW];
      for (int i = 0; i < kMaxW; i++) { R[i] = A[i]; QD[i] = 0; }
      for (int j = 0; j <= C.WMU; j++)
        if (qe[j]) {
          u64 carry = 0;
          for (int i = 0; i < C.WD && i + j < kMaxW; i++) {
            const u64 lo = qe[j] * C.D[i], hi = __umul64hi(qe[j], C.D[i]);
            const u64 s1 = QD[i + j] + lo;
            const u64 c1 = s1 < lo;
            const u64 s2 = s1 + carry;
            const u64 c2 = s2 < carry;
            QD[i + j] = s2;
            carry = hi + c1 + c2;
          }
          for (int i = j + C.WD; carry && i < kMaxW; i++) {
            const u64 s = QD[i] + carry;
            carry = s < carry;
            QD[i] = s;
          }
        }
      mw_sub(R, QD, C.WA);
      u64 Dw[kMaxW];
      for (int i = 0; i < kMaxW; i++) Dw[i] = i < C.WD ? C.D[i] : 0;
      for (int guard = 0; guard < 4 && mw_cmp(R, Dw, C.WA) >= 0; guard++) {
        mw_sub(R, Dw, C.WA);
        for (int i = 0; i < kMaxW; i++) {  // qe += 1
          qe[i] += 1;
          if (qe[i] != 0) break;
        }
      }
    }
    // residues of the rounded quotient (negated for a negative X)
    const int slot = (w == 0) ? 0 : (w == 1 ? 3 : 1);  // (d0, d2, 0, d1)
    u64* o = out + ((size_t)it * 4 + slot) * C.L * n;
    u64* z = out + ((size_t)it * 4 + 2) * C.L * n;
    for (int i = 0; i < C.L; i++) {
      const ModTab tb = tab[i];
      const ModD m = mody(tb);
      const u64 q = (u64)tb.q;
      const u64 rr = mw_mod(qe, C.WMU + 1, q, C.r64[i], m);
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
  hipLaunchKernelGGL(k_crt_lift, grid_t((i64)rows * c->N), dim3(256), 0, st, x, out, rows, C, (const ModTab*)c->d_tab, c->logn);
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
  hipLaunchKernelGGL(k_scale_round, grid_t((i64)items * 3 * c->N), dim3(256), 0, st, prod, out, items, C, (const ModTab*)c->d_tab, c->logn);
  HS_CHECK_HIP(hipGetLastError());
}

}  // namespace hs
