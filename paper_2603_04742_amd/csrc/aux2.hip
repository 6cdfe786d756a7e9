// Elementwise kernels of the "split" path: every step that needs a transform is written as
// (elementwise prologue) -> batched two-pass NTT -> (elementwise epilogue), so rings whose limb does
// not fit in LDS (N = 32768) run keygen, encoding, encryption and decryption too.  The same path
// can be forced at smaller N (hs_set_option), which is how its parity is tested against the
// oracle at sizes the oracle handles quickly.
#include "hs_device.hpp"
#include "kernels.hpp"
#include "extra.hpp"

namespace hs {

__device__ __forceinline__ ModD modx(const ModTab& t) { return ModD{t.q, t.qinv}; }

__device__ __forceinline__ u32 galois_index3(u32 k, u32 g, int logn) {
  const u32 n2m = (2u << logn) - 1;
  const u32 e = 2 * brev_bits(k, logn) + 1;
  const u32 e2 = (u32)(((u64)g * e) & n2m);
  return brev_bits((e2 - 1) >> 1, logn);
}

__device__ __forceinline__ u64 smod_i64(i64 v, u64 q) {
  i64 r = v % (i64)q;
  return (u64)(r < 0 ? r + (i64)q : r);
}
// The same for |v| < q (samples, centered plaintext coefficients): no division.
__device__ __forceinline__ u64 smod_small(i64 v, u64 q) { return (u64)(v < 0 ? v + (i64)q : v); }

// Row-wise elementwise kernels: grid (N / (256 ROW_EPT), rows) with rows looped over gridDim.y, so a
// block's row (and with it the modulus) is uniform and no per-element division is needed.
static constexpr int ROW_EPT = 4;
#define ROW_LOOP(ROWS)                                                                   \
  for (int row = blockIdx.y; row < (ROWS); row += gridDim.y)                             \
    for (int e_ = 0; e_ < ROW_EPT; e_++)                                                 \
      if (const i64 k = ((i64)blockIdx.x * ROW_EPT + e_) * blockDim.x + threadIdx.x; k < n)

// out[o][l][k] = src[o][k] mod modulus (mod0 + l), for small signed integers.
__global__ void k_ints_to_limbs(const int* __restrict__ src, i64 src_stride, int nobj, u64* out, int nl, int mod0,
                                const ModTab* __restrict__ tab, int logn) {
  const i64 n = 1 << logn;
  const i64 total = (i64)nobj * nl * n;
  for (i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x; idx < total; idx += (i64)gridDim.x * blockDim.x) {
    const i64 k = idx & (n - 1);
    const i64 r = idx >> logn;
    const int l = (int)(r % nl), o = (int)(r / nl);
    out[idx] = smod_i64(src[o * src_stride + k], (u64)tab[mod0 + l].q);
  }
}

// Key-switching / public key limb from NTT(e) (already transformed): b = e - a s + [digit] P s',
// a uniform in NTT form (ChaCha20, 128 bits per coefficient).  One thread per 4 coefficients.
__global__ void k_ksk_combine(const KskArgs* __restrict__ args, const u64* __restrict__ e_ntt, int count, const ModTab* __restrict__ tab, int logn) {
  const int n = 1 << logn;
  const int blocks_per = n / 4;
  const i64 gid = blockIdx.x * (i64)blockDim.x + threadIdx.x;
  if (gid >= (i64)count * blocks_per) return;
  const int ai = (int)(gid / blocks_per), blk = (int)(gid % blocks_per);
  const KskArgs A = args[ai];
  const ModTab t = tab[A.mod_index];
  const ModD m = modx(t);
  const u64 q = (u64)t.q;
  u32 w[16];
  chacha_block(A.seed, A.purpose_a, A.idx_a, (u32)blk, w);
  const u64* e = e_ntt + (size_t)ai * n;
#pragma unroll
  for (int c = 0; c < 4; c++) {
    const int i = blk * 4 + c;
    const u64 lo = (u64)w[4 * c] | ((u64)w[4 * c + 1] << 32), hi = (u64)w[4 * c + 2] | ((u64)w[4 * c + 3] << 32);
    const u64 av = d2u(canon(mul_tw(u2d(hi % q), A.r64.x, A.r64.y, m) + u2d(lo % q), m));
    const double s = u2d(A.sk[i]);
    double v = u2d(e[i]) - mulmod(u2d(av), s, m);
    if (A.sprime_mode == 1) v += mul_tw(u2d(A.sk[galois_index3((u32)i, A.galois, logn)]), A.pfac.x, A.pfac.y, m);
    else if (A.sprime_mode == 2) v += mul_tw(mulmod(s, s, m), A.pfac.x, A.pfac.y, m);
    A.b[i] = d2u(canon(v, m));
    A.a[i] = av;
  }
}

// Slot packing without the transform: the slot value of chunk g goes to position slot_pos[k] of
// row g (mod t); the inverse mod-t NTT follows.
__global__ void k_pack_slots(PackArgs A, int nchunks, const u32* __restrict__ slot_pos, u64 t, int logn) {
  const i64 n = 1 << logn;
  const i64 total = (i64)nchunks * n;
  for (i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x; idx < total; idx += (i64)gridDim.x * blockDim.x) {
    const int g = (int)(idx >> logn);
    const i64 k = idx & (n - 1);
    const int mode = A.mode == 3 ? (g < A.nG ? 0 : 2) : A.mode;
    const i64* cd = A.chunk + 8 * (A.mode == 3 && g >= A.nG ? g - A.nG : g);
    const i64 start = cd[0], cols = cd[1], h = cd[2];
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
    A.out[(size_t)g * n + slot_pos[k]] = smod_i64(val, t);
  }
}

// Centered lift of mod-t coefficients to every data prime: out[g][l][k].
__global__ void k_lift_plain(const u64* __restrict__ coef, int n_plain, u64* out, int L, u64 t, const ModTab* __restrict__ tab, int logn) {
  const i64 n = 1 << logn;
  ROW_LOOP(n_plain * L) {
    const int l = row % L, g = row / L;
    const u64 v = coef[(size_t)g * n + k];
    const i64 c = v > (t - 1) / 2 ? (i64)v - (i64)t : (i64)v;
    out[(size_t)row * n + k] = smod_small(c, (u64)tab[l].q);
  }
}

// Encryption prologue: U = u, E1 = e1, D0 = e0 + floor(Q m / t + 1/2), each reduced to every data
// prime: out [n_ct][3][L][N] coefficient form (then transformed).
__global__ void k_enc_prep(const u64* __restrict__ mcoef, const int* __restrict__ samples, int n_ct, u64* out, int L, u64 t, u64 q_mod_t,
                           const double2* __restrict__ qdt, const ModTab* __restrict__ tab, int logn) {
  const i64 n = 1 << logn;
  ROW_LOOP(n_ct * L) {
    const int l = row % L, g = row / L;
    const ModTab tb = tab[l];
    const ModD m = modx(tb);
    const u64 q = (u64)tb.q;
    const int* u = samples + (size_t)g * 3 * n;
    const u64 mv = mcoef[(size_t)g * n + k];
    const double d1 = mul_tw((double)mv, qdt[l].x, qdt[l].y, m);
    // floor(((Q mod t) m + floor(t/2)) / t): the numerator is below 2^53 (t < 2^26), so the quotient of the
    // exactly represented doubles rounds to within 2^-18 of the true one and floor is exact
    const double d2 = floor(((double)(q_mod_t * mv) + (double)(t / 2)) / (double)t);
    u64* o = out + ((size_t)g * 3 * L) * n;
    o[((size_t)0 * L + l) * n + k] = smod_small(u[k], q);
    o[((size_t)1 * L + l) * n + k] = smod_small(u[2 * n + k], q);
    o[((size_t)2 * L + l) * n + k] = d2u(canon(reduce((double)u[n + k] + d1 + d2, m), m));
  }
}

// Encryption epilogue (NTT domain): c0 = pk0 U + D0, c1 = pk1 U + E1.
__global__ void k_enc_combine(const u64* __restrict__ prep, const u64* __restrict__ pk, u64* out, int n_ct, int L, const ModTab* __restrict__ tab,
                              int logn) {
  const i64 n = 1 << logn;
  ROW_LOOP(n_ct * L) {
    const int l = row % L, g = row / L;
    const ModD m = modx(tab[l]);
    const u64* p = prep + ((size_t)g * 3 * L) * n;
    const double U = u2d(p[((size_t)0 * L + l) * n + k]);
    const double E1 = u2d(p[((size_t)1 * L + l) * n + k]);
    const double D0 = u2d(p[((size_t)2 * L + l) * n + k]);
    out[((size_t)g * 2 * L + l) * n + k] = d2u(canon(mulmod(U, u2d(pk[(size_t)l * n + k]), m) + D0, m));
    out[((size_t)g * 2 * L + L + l) * n + k] = d2u(canon(mulmod(U, u2d(pk[((size_t)L + l) * n + k]), m) + E1, m));
  }
}

// Decryption prologue (NTT domain): x = c0 + c1 s per limb.
__global__ void k_dec_prep(const u64* __restrict__ ct, const u64* __restrict__ sk, u64* X, int n_ct, int L, const ModTab* __restrict__ tab, int logn) {
  const i64 n = 1 << logn;
  ROW_LOOP(n_ct * L) {
    const int l = row % L, g = row / L;
    const ModD m = modx(tab[l]);
    const double c0 = u2d(ct[((size_t)g * 2 * L + l) * n + k]), c1 = u2d(ct[((size_t)g * 2 * L + L + l) * n + k]);
    X[(size_t)row * n + k] = d2u(canon(c0 + mulmod(c1, u2d(sk[(size_t)l * n + k]), m), m));
  }
}

// Decode + scatter after the forward mod-t NTT of M (rows = partitions).
__global__ void k_slots_scatter(const u64* __restrict__ Mntt, const u32* __restrict__ slot_pos, const int* __restrict__ rm, const i64* __restrict__ pinfo,
                                int nparts, i64* y, u64 t, int logn) {
  const i64 n = 1 << logn;
  const int P = blockIdx.y;
  if (P >= nparts) return;
  // pinfo per partition: (row0, rows, nonzero rows, row-map offset, group, slot offset)
  const i64* pi = pinfo + 6 * P;
  const i64 row0 = pi[0], rows = pi[1], nz = pi[2], rm0 = pi[3], grp = pi[4], off = pi[5];
  for (i64 p = blockIdx.x * (i64)blockDim.x + threadIdx.x; p < rows; p += (i64)gridDim.x * blockDim.x) {
    i64 v = 0;
    if (p < nz) {
      v = (i64)Mntt[(size_t)grp * n + slot_pos[off + p]];
      if (v > (i64)(t / 2)) v -= (i64)t;
    }
    y[row0 + rm[rm0 + p]] = v;
  }
}

// The diagonal method's packing.  A block diagonal is named by id = (bi ncb + bj) B + d with
// d = (j - i) mod B for the entry (bi B + i, bj B + j); ids ascend in (bi, bj, d) order.
// One thread per matrix row: flag every id that holds a stored entry (entries with an invalid
// column are skipped here and reported by the column check).
__global__ void k_diag_mark(const i64* __restrict__ row_ptr, const int* __restrict__ col, i64 R, i64 C, i64 B, i64 ncb, unsigned char* flags) {
  const i64 r = blockIdx.x * (i64)blockDim.x + threadIdx.x;
  if (r >= R) return;
  const i64 bi = r / B, i = r - bi * B;
  for (i64 k = row_ptr[r]; k < row_ptr[r + 1]; k++) {
    const i64 c = col[k];
    if (c < 0 || c >= C) continue;
    const i64 bj = c / B, j = c - bj * B;
    flags[(bi * ncb + bj) * B + (j - i + B) % B] = 1;
  }
}

// Slot i of diagonal (bi, bj, d) receives A[bi B + i][bj B + (i + d) mod B] mod t at position
// slot_pos[i] of that diagonal's row (then the inverse mod-t NTT).  The diagonal's row is found by
// binary search in the ascending id list.  The column check has passed before this runs.
__global__ void k_diag_place(const i64* __restrict__ row_ptr, const int* __restrict__ col, const i64* __restrict__ val, i64 R, i64 B, i64 ncb,
                             const i64* __restrict__ ids, int nd, u64* out, const u32* __restrict__ slot_pos, u64 t, int logn) {
  const i64 r = blockIdx.x * (i64)blockDim.x + threadIdx.x;
  if (r >= R) return;
  const i64 bi = r / B, i = r - bi * B;
  const u32 pos = slot_pos[i];
  for (i64 k = row_ptr[r]; k < row_ptr[r + 1]; k++) {
    const i64 c = col[k], bj = c / B, j = c - bj * B;
    const i64 id = (bi * ncb + bj) * B + (j - i + B) % B;
    int lo = 0, hi = nd - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (ids[mid] < id) lo = mid + 1; else hi = mid;
    }
    out[((size_t)lo << logn) + pos] = smod_i64(val[k], t);
  }
}

// Vector block bj, twice over: slots j and B + j hold v[bj B + j] mod t (0 past the last column),
// every other slot 0; written at slot_pos order (then the inverse mod-t NTT).
__global__ void k_diag_vector(const i64* __restrict__ v, i64 C, i64 B, int ncb, u64* out, const u32* __restrict__ slot_pos, u64 t, int logn) {
  const i64 n = 1 << logn;
  const i64 total = (i64)ncb * n;
  for (i64 idx = blockIdx.x * (i64)blockDim.x + threadIdx.x; idx < total; idx += (i64)gridDim.x * blockDim.x) {
    const i64 bj = idx >> logn, k = idx & (n - 1);
    const i64 j = k < B ? k : (k < 2 * B ? k - B : -1);
    const i64 cc = bj * B + j;
    const u64 x = (j >= 0 && cc < C) ? smod_i64(v[cc], t) : 0;
    out[(size_t)bj * n + slot_pos[k]] = x;
  }
}

// ------------------------------------------------------------------ launchers
static dim3 grid_for(i64 total) { return dim3((unsigned)std::min<i64>((total + 255) / 256, 256 * 64)); }
static dim3 grid_rows(i64 rows, i64 n) {
  return dim3((unsigned)std::max<i64>(1, (n + 256 * ROW_EPT - 1) / (256 * ROW_EPT)), (unsigned)std::min<i64>(std::max<i64>(rows, 1), 65535));
}

#define HSX_LAUNCH(KERNEL, GRID, STREAM, ...)                                  \
  do {                                                                         \
    ProfScope _prof(#KERNEL, STREAM);                                          \
    hipLaunchKernelGGL(KERNEL, GRID, dim3(256), 0, STREAM, __VA_ARGS__);       \
    HS_CHECK_HIP(hipGetLastError());                                           \
  } while (0)

void launch_ints_to_limbs(const hs_ctx* c, const int* src, i64 src_stride, int nobj, u64* out, int nl, int mod0, hipStream_t st) {
  if (nobj <= 0) return;
  HSX_LAUNCH(k_ints_to_limbs, grid_for((i64)nobj * nl * c->N), st, src, src_stride, nobj, out, nl, mod0, (const ModTab*)c->d_tab, c->logn);
}
void launch_ksk_combine(const hs_ctx* c, const KskArgs* d_args, const u64* e_ntt, int count, hipStream_t st) {
  if (count <= 0) return;
  const i64 threads = (i64)count * (c->N / 4);
  hipLaunchKernelGGL(k_ksk_combine, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, st, d_args, e_ntt, count, (const ModTab*)c->d_tab, c->logn);
  HS_CHECK_HIP(hipGetLastError());
}
void launch_pack_slots(const hs_ctx* c, const PackArgs& a, int nchunks, hipStream_t st) {
  if (nchunks <= 0) return;
  HSX_LAUNCH(k_pack_slots, grid_for((i64)nchunks * c->N), st, a, nchunks, (const u32*)c->d_slot_pos, c->t, c->logn);
}
void launch_lift_plain(const hs_ctx* c, const u64* coef, int n_plain, u64* out, hipStream_t st) {
  if (n_plain <= 0) return;
  HSX_LAUNCH(k_lift_plain, grid_rows((i64)n_plain * c->L, c->N), st, coef, n_plain, out, c->L, c->t, (const ModTab*)c->d_tab, c->logn);
}
void launch_enc_prep(const hs_ctx* c, const u64* mcoef, const int* samples, int n_ct, u64* out, hipStream_t st) {
  if (n_ct <= 0) return;
  HSX_LAUNCH(k_enc_prep, grid_rows((i64)n_ct * c->L, c->N), st, mcoef, samples, n_ct, out, c->L, c->t, c->q_mod_t, (const double2*)c->d_qdt,
             (const ModTab*)c->d_tab, c->logn);
}
void launch_enc_combine(const hs_ctx* c, const u64* prep, const u64* pk, u64* out, int n_ct, hipStream_t st) {
  if (n_ct <= 0) return;
  HSX_LAUNCH(k_enc_combine, grid_rows((i64)n_ct * c->L, c->N), st, prep, pk, out, n_ct, c->L, (const ModTab*)c->d_tab, c->logn);
}
void launch_dec_prep(const hs_ctx* c, const u64* ct, const u64* sk, u64* X, int n_ct, hipStream_t st) {
  if (n_ct <= 0) return;
  HSX_LAUNCH(k_dec_prep, grid_rows((i64)n_ct * c->L, c->N), st, ct, sk, X, n_ct, c->L, (const ModTab*)c->d_tab, c->logn);
}
void launch_slots_scatter(const hs_ctx* c, const u64* Mntt, const int* rm, const i64* pinfo, int nparts, i64* y, hipStream_t st) {
  if (nparts <= 0) return;
  hipLaunchKernelGGL(k_slots_scatter, dim3(std::max<int>(1, (int)((c->N / 2 + 255) / 256)), nparts), dim3(256), 0, st, Mntt,
                     (const u32*)c->d_slot_pos, rm, pinfo, nparts, y, c->t, c->logn);
  HS_CHECK_HIP(hipGetLastError());
}

void launch_diag_mark(const i64* row_ptr, const int* col, i64 R, i64 C, i64 B, i64 ncb, unsigned char* flags, hipStream_t st) {
  if (R <= 0) return;
  HSX_LAUNCH(k_diag_mark, dim3((unsigned)((R + 255) / 256)), st, row_ptr, col, R, C, B, ncb, flags);
}
void launch_diag_place(const hs_ctx* c, const i64* row_ptr, const int* col, const i64* val, i64 R, i64 B, i64 ncb, const i64* ids, int nd,
                       u64* out, hipStream_t st) {
  if (R <= 0 || nd <= 0) return;
  HSX_LAUNCH(k_diag_place, dim3((unsigned)((R + 255) / 256)), st, row_ptr, col, val, R, B, ncb, ids, nd, out, (const u32*)c->d_slot_pos, c->t,
             c->logn);
}
void launch_diag_vector(const hs_ctx* c, const i64* v, i64 C, i64 B, int ncb, u64* out, hipStream_t st) {
  if (ncb <= 0) return;
  HSX_LAUNCH(k_diag_vector, grid_for((i64)ncb * c->N), st, v, C, B, ncb, out, (const u32*)c->d_slot_pos, c->t, c->logn);
}

}  // namespace hs
