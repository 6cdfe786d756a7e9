/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, deliberately unoptimised reference implementation of encrypted sparse
 * matrix-vector multiplication over the Compressed Sparse Sorted Column (CSSC) format
 * (arXiv 2603.04742) on BFV-style RLWE.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code, header, table or
 * constant generator with the GPU library; the GPU path must never call into it.
 *
 * Paper passages followed (section / algorithm / equation of arXiv 2603.04742):
 *   - CSSC definition and CSR->CSSC conversion: Sec. 4.3, Appendix B (Alg. "Conversion from CSR
 *     to CSSC Format").
 *   - Chunk generation: Sec. 4.4.1, Alg. generateChunk.
 *   - Vector reorganisation: Sec. 4.4.2, Alg. reorgVector.
 *   - Cloud products and aggregation (totalSum + masks): Sec. 4.5, Alg. Aggregation and the mask
 *     equation.
 *   - Protocol and row-map scatter: Sec. 4.4, Alg. "Sparse Matrix-Vector Multiplication".
 *   - Row partitioning of large matrices: Sec. 4.7.
 *   - HE operations (Add, Mult, CMult, Rot): Sec. 2.1.
   - Rotation keys: Sec. 5 (experimental setup) generates power-of-two rotation keys; read as left
     rotations by 2^i, a rotation by any other amount applied as its binary digits, lowest first.
     Optionally (not the paper's reading) the key set also holds right rotations by 2^i and a
     rotation applies the signed digits of its non-adjacent form, as BFV libraries commonly do.
 * The paper leaves the HE scheme internals to its library; the conventions pinned here (prime
 * choice, NTT order, slot order, sampling, key switching, BFV multiplication) are listed in the
 * design notes and repeated next to the code that implements them.
 *
 * Arithmetic: every modular product is (unsigned __int128)a*b % m.  Big integers (CRT, scaling)
 * use a tiny schoolbook bignum on 32-bit limbs.
 */
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <algorithm>
#include <map>
#include <array>

#include "cdt_sigma3p2.h"
#ifdef _OPENMP
#include <omp.h>
#endif

typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;
typedef int32_t i32;
typedef unsigned __int128 u128;

namespace {

/* ------------------------------------------------------------------ modular arithmetic */
u64 mulmod(u64 a, u64 b, u64 m) { return (u64)(((u128)a * b) % m); }
/* a, b < m < 2^63 */
u64 addmod(u64 a, u64 b, u64 m) { u64 s = a + b; return s >= m ? s - m : s; }
u64 submod(u64 a, u64 b, u64 m) { return a >= b ? a - b : a + (m - b); }
u64 negmod(u64 a, u64 m) { return a == 0 ? 0 : m - a; }
u64 powmod(u64 b, u64 e, u64 m) {
  u64 r = 1 % m;
  b %= m;
  while (e) {
    if (e & 1) r = mulmod(r, b, m);
    b = mulmod(b, b, m);
    e >>= 1;
  }
  return r;
}
u64 invmod(u64 a, u64 p) { return powmod(a, p - 2, p); } /* p prime */
u64 smod(i64 v, u64 m) { /* signed integer -> [0, m) */
  i64 r = v % (i64)m;
  return (u64)(r < 0 ? r + (i64)m : r);
}

/* Deterministic Miller-Rabin for n < 2^64 (bases 2..37). */
bool is_prime(u64 n) {
  if (n < 2) return false;
  static const u64 bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (u64 b : bases) {
    if (n % b == 0) return n == b;
  }
  u64 d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; s++; }
  for (u64 a : bases) {
    u64 x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; r++) {
      x = mulmod(x, x, n);
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

/* Primes q < 2^bits with q = 1 mod 2N, largest first. */
std::vector<u64> ntt_primes(u64 N, int bits, int count) {
  std::vector<u64> out;
  u64 step = 2 * N;
  u64 top = (bits >= 64) ? ~0ULL : ((1ULL << bits) - 1);
  u64 q = (top / step) * step + 1;
  if (q > top) q -= step;
  while ((int)out.size() < count && q > step) {
    if (is_prime(q)) out.push_back(q);
    q -= step;
  }
  return out;
}

/* The smallest primitive 2N-th root of unity mod q (q = 1 mod 2N): find one root psi0, then
   take the minimum over all of them, psi0^(2k+1), k = 0..N-1. */
u64 min_primitive_root(u64 q, u64 N) {
  u64 psi0 = 0;
  for (u64 x = 2; x < q; x++) {
    u64 c = powmod(x, (q - 1) / (2 * N), q);
    if (powmod(c, N, q) == q - 1) { psi0 = c; break; }
  }
  u64 best = psi0, cur = psi0, sq = mulmod(psi0, psi0, q);
  for (u64 k = 1; k < N; k++) {
    cur = mulmod(cur, sq, q);
    if (cur < best) best = cur;
  }
  return best;
}

u32 bitrev(u32 x, int bits) {
  u32 r = 0;
  for (int i = 0; i < bits; i++) { r = (r << 1) | (x & 1); x >>= 1; }
  return r;
}

/* ------------------------------------------------------------------ negacyclic NTT
 * Output order (pinned): NTT(a)[k] = a(psi^(2*bitrev(k)+1)) mod q, i.e. evaluations at the odd
 * powers of psi in bit-reversed order.  Forward = Cooley-Tukey with merged psi-twisting, inverse =
 * Gentleman-Sande (Longa & Naehrig 2016).  Checked in the tests against direct evaluation and
 * against schoolbook negacyclic convolution. */
struct NttTable {
  u64 q = 0, psi = 0, ninv = 0;
  int logn = 0;
  std::vector<u64> fw, iv; /* fw[i] = psi^bitrev(i), iv[i] = psi^-bitrev(i) */
  void init(u64 q_, u64 psi_, int logn_) {
    q = q_; psi = psi_; logn = logn_;
    u64 N = 1ULL << logn;
    fw.assign(N, 0); iv.assign(N, 0);
    u64 pinv = invmod(psi, q);
    for (u64 i = 0; i < N; i++) {
      u32 r = bitrev((u32)i, logn);
      fw[i] = powmod(psi, r, q);
      iv[i] = powmod(pinv, r, q);
    }
    ninv = invmod(N % q, q);
  }
  void forward(u64* a) const {
    u64 N = 1ULL << logn;
    u64 t = N;
    for (u64 m = 1; m < N; m <<= 1) {
      t >>= 1;
      for (u64 i = 0; i < m; i++) {
        u64 j1 = 2 * i * t, S = fw[m + i];
        for (u64 j = j1; j < j1 + t; j++) {
          u64 U = a[j], V = mulmod(a[j + t], S, q);
          a[j] = addmod(U, V, q);
          a[j + t] = submod(U, V, q);
        }
      }
    }
  }
  void inverse(u64* a) const {
    u64 N = 1ULL << logn;
    u64 t = 1;
    for (u64 m = N; m > 1; m >>= 1) {
      u64 h = m >> 1, j1 = 0;
      for (u64 i = 0; i < h; i++) {
        u64 S = iv[h + i];
        for (u64 j = j1; j < j1 + t; j++) {
          u64 U = a[j], V = a[j + t];
          a[j] = addmod(U, V, q);
          a[j + t] = mulmod(submod(U, V, q), S, q);
        }
        j1 += 2 * t;
      }
      t <<= 1;
    }
    for (u64 j = 0; j < N; j++) a[j] = mulmod(a[j], ninv, q);
  }
};

/* ------------------------------------------------------------------ big integers
 * Non-negative integers as little-endian 32-bit limbs; sign kept separately where needed. */
typedef std::vector<u32> Big;
void bnorm(Big& a) { while (!a.empty() && a.back() == 0) a.pop_back(); }
Big bfrom(u64 v) { Big r; while (v) { r.push_back((u32)v); v >>= 32; } return r; }
int bcmp(const Big& a, const Big& b) {
  if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
  for (size_t i = a.size(); i-- > 0;) if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  return 0;
}
Big badd(const Big& a, const Big& b) {
  Big r(std::max(a.size(), b.size()) + 1, 0);
  u64 c = 0;
  for (size_t i = 0; i < r.size(); i++) {
    u64 s = c + (i < a.size() ? a[i] : 0) + (i < b.size() ? b[i] : 0);
    r[i] = (u32)s; c = s >> 32;
  }
  bnorm(r); return r;
}
Big bsub(const Big& a, const Big& b) { /* a >= b */
  Big r(a.size(), 0);
  i64 br = 0;
  for (size_t i = 0; i < a.size(); i++) {
    i64 s = (i64)a[i] - (i < b.size() ? (i64)b[i] : 0) - br;
    br = s < 0; if (s < 0) s += (1LL << 32);
    r[i] = (u32)s;
  }
  bnorm(r); return r;
}
Big bmul(const Big& a, const Big& b) {
  if (a.empty() || b.empty()) return Big();
  std::vector<u64> acc(a.size() + b.size() + 1, 0);
  for (size_t i = 0; i < a.size(); i++) {
    u64 c = 0;
    for (size_t j = 0; j < b.size(); j++) {
      u64 s = acc[i + j] + (u64)a[i] * b[j] + c;
      acc[i + j] = (u32)s; c = s >> 32;
    }
    size_t k = i + b.size();
    while (c) { u64 s = acc[k] + c; acc[k] = (u32)s; c = s >> 32; k++; }
  }
  Big r(acc.size()); for (size_t i = 0; i < acc.size(); i++) r[i] = (u32)acc[i];
  bnorm(r); return r;
}
Big bmulu(const Big& a, u64 v) { return bmul(a, bfrom(v)); }
Big bshl1(const Big& a) { return badd(a, a); }
u64 bmodu(const Big& a, u64 m) { /* Horner */
  u64 r = 0;
  for (size_t i = a.size(); i-- > 0;) r = (u64)((((u128)r << 32) + a[i]) % m);
  return r;
}
/* floor(a / b) and a mod b: schoolbook long division on 32-bit limbs (Knuth, TAOCP vol. 2,
   Algorithm 4.3.1 D). */
void bdivmod(const Big& a_, const Big& b_, Big& q, Big& r) {
  Big a = a_, b = b_; bnorm(a); bnorm(b);
  q.clear(); r.clear();
  if (b.empty()) { fprintf(stderr, "oracle: division by zero\n"); abort(); }
  if (bcmp(a, b) < 0) { r = a; return; }
  int n = (int)b.size(), m = (int)a.size();
  if (n == 1) {
    q.assign(m, 0); u64 rem = 0;
    for (int i = m - 1; i >= 0; i--) { u64 cur = (rem << 32) | a[i]; q[i] = (u32)(cur / b[0]); rem = cur % b[0]; }
    bnorm(q); r = bfrom(rem); return;
  }
  int s = __builtin_clz(b[n - 1]);
  std::vector<u32> vn(n), un(m + 1);
  for (int i = n - 1; i > 0; i--) vn[i] = (b[i] << s) | (s ? (u32)((u64)b[i - 1] >> (32 - s)) : 0);
  vn[0] = b[0] << s;
  un[m] = s ? (u32)((u64)a[m - 1] >> (32 - s)) : 0;
  for (int i = m - 1; i > 0; i--) un[i] = (a[i] << s) | (s ? (u32)((u64)a[i - 1] >> (32 - s)) : 0);
  un[0] = a[0] << s;
  q.assign(m - n + 1, 0);
  const u64 B = 1ULL << 32;
  for (int j = m - n; j >= 0; j--) {
    u64 num = ((u64)un[j + n] << 32) | un[j + n - 1];
    u64 qhat = num / vn[n - 1], rhat = num % vn[n - 1];
    while (qhat >= B || qhat * vn[n - 2] > ((rhat << 32) | un[j + n - 2])) {
      qhat--; rhat += vn[n - 1];
      if (rhat >= B) break;
    }
    i64 k = 0, tt;
    for (int i = 0; i < n; i++) {
      u64 p = qhat * vn[i];
      tt = (i64)un[i + j] - k - (i64)(p & 0xffffffffULL);
      un[i + j] = (u32)tt;
      k = (i64)(p >> 32) - (tt >> 32);
    }
    tt = (i64)un[j + n] - k; un[j + n] = (u32)tt;
    q[j] = (u32)qhat;
    if (tt < 0) {
      q[j]--; k = 0;
      for (int i = 0; i < n; i++) { u64 t2 = (u64)un[i + j] + vn[i] + (u64)k; un[i + j] = (u32)t2; k = (i64)(t2 >> 32); }
      un[j + n] = (u32)((u64)un[j + n] + (u64)k);
    }
  }
  r.assign(n, 0);
  for (int i = 0; i < n; i++) r[i] = (un[i] >> s) | (s ? (u32)((u64)un[i + 1] << (32 - s)) : 0);
  bnorm(q); bnorm(r);
}
Big bprod(const std::vector<u64>& ms) { Big r = bfrom(1); for (u64 m : ms) r = bmulu(r, m); return r; }

/* CRT basis: M = prod m_i, M_i = M / m_i, inv_i = M_i^-1 mod m_i. */
struct CrtBasis {
  std::vector<u64> m; Big M; std::vector<Big> Mi; std::vector<u64> inv;
  explicit CrtBasis(const std::vector<u64>& ms = {}) : m(ms) {
    M = bprod(ms);
    for (size_t i = 0; i < ms.size(); i++) {
      std::vector<u64> others; for (size_t j = 0; j < ms.size(); j++) if (j != i) others.push_back(ms[j]);
      Mi.push_back(bprod(others));
      inv.push_back(invmod(bmodu(Mi.back(), ms[i]), ms[i]));
    }
  }
};
/* CRT: residues x_i mod m_i -> the integer in [0, M).  sum_i M_i [x_i inv_i]_{m_i} < n M, so at
   most n - 1 subtractions of M remain. */
Big crt(const std::vector<u64>& x, const CrtBasis& B) {
  Big acc;
  for (size_t i = 0; i < B.m.size(); i++) acc = badd(acc, bmulu(B.Mi[i], mulmod(x[i], B.inv[i], B.m[i])));
  while (bcmp(acc, B.M) >= 0) acc = bsub(acc, B.M);
  return acc;
}

/* ------------------------------------------------------------------ ChaCha20 (RFC 8439) */
inline u32 rotl(u32 v, int c) { return (v << c) | (v >> (32 - c)); }
#define ORC_QR(a, b, c, d) \
  a += b; d ^= a; d = rotl(d, 16); c += d; b ^= c; b = rotl(b, 12); \
  a += b; d ^= a; d = rotl(d, 8);  c += d; b ^= c; b = rotl(b, 7);
void chacha20_block(const u32 key[8], u32 counter, const u32 nonce[3], u32 out[16]) {
  u32 st[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u,
                key[0], key[1], key[2], key[3], key[4], key[5], key[6], key[7],
                counter, nonce[0], nonce[1], nonce[2]};
  u32 x[16];
  memcpy(x, st, sizeof x);
  for (int i = 0; i < 10; i++) {
    ORC_QR(x[0], x[4], x[8], x[12]); ORC_QR(x[1], x[5], x[9], x[13]);
    ORC_QR(x[2], x[6], x[10], x[14]); ORC_QR(x[3], x[7], x[11], x[15]);
    ORC_QR(x[0], x[5], x[10], x[15]); ORC_QR(x[1], x[6], x[11], x[12]);
    ORC_QR(x[2], x[7], x[8], x[13]); ORC_QR(x[3], x[4], x[9], x[14]);
  }
  for (int i = 0; i < 16; i++) out[i] = x[i] + st[i];
}

/* The random stream of one sampled object: key = seed (little-endian 64 bits, then 192 zero
   bits), nonce = (purpose, index low 32, index high 32), counter = block number.  Word w of the
   stream is word (w mod 16) of block (w div 16). */
struct Stream {
  u32 key[8], nonce[3], blk[16];
  i64 cur = -1;
  Stream(u64 seed, u32 purpose, u64 index) {
    memset(key, 0, sizeof key);
    key[0] = (u32)seed; key[1] = (u32)(seed >> 32);
    nonce[0] = purpose; nonce[1] = (u32)index; nonce[2] = (u32)(index >> 32);
  }
  u32 word(u64 w) {
    i64 b = (i64)(w / 16);
    if (b != cur) { chacha20_block(key, (u32)b, nonce, blk); cur = b; }
    return blk[w % 16];
  }
};

enum : u32 {
  P_SK = 1, P_PK_A = 2, P_PK_E = 3, P_KSK_A = 4, P_KSK_E = 5,
  P_ENC_U = 6, P_ENC_E0 = 7, P_ENC_E1 = 8
};

/* Ternary: coefficient i = (word i mod 3) - 1. */
std::vector<i64> sample_ternary(u64 seed, u32 purpose, u64 index, u64 N) {
  Stream s(seed, purpose, index);
  std::vector<i64> r(N);
  for (u64 i = 0; i < N; i++) r[i] = (i64)(s.word(i) % 3) - 1;
  return r;
}
/* Discrete Gaussian (sigma 3.2) by CDT: 64 bits per coefficient (words 2i, 2i+1), top bit =
   sign, low 63 bits r; |e| = smallest k with r < T[k]. */
std::vector<i64> sample_gauss(u64 seed, u32 purpose, u64 index, u64 N) {
  Stream s(seed, purpose, index);
  std::vector<i64> r(N);
  for (u64 i = 0; i < N; i++) {
    u64 x = (u64)s.word(2 * i) | ((u64)s.word(2 * i + 1) << 32);
    u64 v = x & 0x7fffffffffffffffULL;
    int mag = 0;
    while (!(v < ORC_CDT[mag])) mag++;
    r[i] = (x >> 63) ? -(i64)mag : (i64)mag;
  }
  return r;
}
/* Uniform mod q: coefficient i = (128-bit little-endian value of words 4i..4i+3) mod q. */
std::vector<u64> sample_uniform(u64 seed, u32 purpose, u64 index, u64 q, u64 N) {
  Stream s(seed, purpose, index);
  std::vector<u64> r(N);
  for (u64 i = 0; i < N; i++) {
    u128 v = 0;
    for (int k = 3; k >= 0; k--) v = (v << 32) | s.word(4 * i + k);
    r[i] = (u64)(v % q);
  }
  return r;
}

/* ------------------------------------------------------------------ scheme context */
struct Ctx {
  int logn = 0; u64 N = 0; u64 t = 0;
  int L = 0, K = 0, alpha = 0, dnum = 0, qbits = 0, pbits = 0, agg_mode = 0;
  int slot_rows = 1;             /* 1: data in slot row 0 only; 2: two row partitions per ciphertext */
  int lazy_relin = 0;            /* 1: chunks without totalSum rotations keep (d0, d1, d2) until the
                                    inter-chunk sum, relinearised once per result ciphertext */
  int n_aux = 0;                 /* extra primes for the exact ct x ct tensor */
  bool has_tensor = false;       /* the basis product exceeds 4 N Q^2 (else no ct x ct) */
  std::vector<u64> mod;          /* [L data primes][K special primes][n_aux tensor primes] */
  std::vector<NttTable> tab;
  NttTable ttab;                 /* plaintext modulus t */
  std::vector<u32> slot_pos;     /* slot j -> index k of NTT_t output */
  Big Q, P;
  CrtBasis crtQ, crtT;           /* data primes; whole tensor basis */
  u64 Q_mod_t = 0;
  std::vector<u64> Q_div_t_mod;  /* floor(Q/t) mod q_i */
  /* keys */
  bool has_keys = false;
  std::vector<i64> s;            /* secret, coefficient form */
  std::vector<u64> s_ntt;        /* [L+K+n_aux][N] */
  std::vector<u64> pk0, pk1;     /* [L][N] */
  std::vector<std::vector<u64>> gk; /* power-of-two rotation keys, index as rot_key_step: [2][dnum][L+K][N] (b then a) */
  bool signed_digits = false;        /* right keys held: rotations use signed digits */
  std::map<u64, std::vector<u64>> gk_step; /* optional exact-step rotation keys, by step k */
  std::vector<u64> rk;           /* relinearisation key, same layout */
  u64 keyseed = 0;
};

u64* limb(std::vector<u64>& v, u64 N, int i) { return v.data() + (u64)i * N; }

/* A left rotation by k slots within each slot row has Galois element 3^k mod 2N (Sec. 2.1,
   HE-Rot; 3 generates the slot-row rotations of the power-of-two cyclotomic ring and has order
   N/2 modulo 2N, so a right rotation by k is the left rotation by N/2 - k). */
u64 galois_elt_step(const Ctx& c, u64 k) { return powmod(3, k % (c.N / 2), 2 * c.N); }
/* Power-of-two rotation keys: index i < logn - 1 rotates left by 2^i; with the optional right keys,
   index (logn - 1) + i rotates right by 2^i.  rot_key_step gives the signed step (+2^i or -2^i). */
int n_pow2(const Ctx& c) { return c.logn - 1; }
i64 rot_key_step(const Ctx& c, int idx) { return idx < n_pow2(c) ? (1LL << idx) : -(1LL << (idx - n_pow2(c))); }
u64 galois_elt_key(const Ctx& c, int idx) {
  i64 st = rot_key_step(c, idx);
  return galois_elt_step(c, st > 0 ? (u64)st : c.N / 2 - (u64)(-st));
}
/* Sampling ids of the rotation keys: left 2^i -> i, right 2^i -> 64 + i; below the
   relinearisation id (255). */
u32 rot_key_id(const Ctx& c, int idx) { return idx < n_pow2(c) ? (u32)idx : 64u + (u32)(idx - n_pow2(c)); }
/* Sampling id of an exact-step rotation key: above the power-of-two ids and the
   relinearisation id (255), one per step. */
u32 step_key_id(u64 k) { return 256u + (u32)k; }

/* The power-of-two key switches of a left rotation by k slots, 0 <= k < N/2, as key indices in
   the order they are applied, lowest first: the binary digits of k (left keys only); with the
   right keys, the digits of the non-adjacent form of k (signed binary, no two adjacent digits
   nonzero; Reitwiesner), where a digit of +-N/2 rotates every row by a whole row, the identity,
   and is left out. */
std::vector<int> rotation_digits(const Ctx& c, u64 k) {
  std::vector<int> out;
  const int nl = n_pow2(c);
  if (!c.signed_digits) {
    for (int i = 0; i < nl; i++)
      if ((k >> i) & 1) out.push_back(i);
    return out;
  }
  int i = 0;
  while (k) {
    if (k & 1) {
      if ((k & 3) == 1) { if (i < nl) out.push_back(i); k -= 1; }       /* digit +1 */
      else { if (i < nl) out.push_back(nl + i); k += 1; }                /* digit -1 */
    }
    k >>= 1;
    i++;
  }
  return out;
}

/* Coefficient-domain automorphism a(X) -> a(X^g) mod (X^N + 1) over Z_m. */
std::vector<u64> automorph_coeff(const std::vector<u64>& a, u64 g, u64 N, u64 m) {
  std::vector<u64> r(N, 0);
  for (u64 i = 0; i < N; i++) {
    u64 e = (u64)(((u128)g * i) % (2 * N));
    if (e < N) r[e] = addmod(r[e], a[i], m);
    else r[e - N] = submod(r[e - N], a[i], m);
  }
  return r;
}
std::vector<i64> automorph_int(const std::vector<i64>& a, u64 g, u64 N) {
  std::vector<i64> r(N, 0);
  for (u64 i = 0; i < N; i++) {
    u64 e = (u64)(((u128)g * i) % (2 * N));
    if (e < N) r[e] += a[i]; else r[e - N] -= a[i];
  }
  return r;
}

/* NTT of a small signed polynomial reduced mod modulus m. */
std::vector<u64> ntt_of_int(const Ctx& c, const std::vector<i64>& a, int m) {
  std::vector<u64> r(c.N);
  for (u64 i = 0; i < c.N; i++) r[i] = smod(a[i], c.mod[m]);
  c.tab[m].forward(r.data());
  return r;
}

bool ctx_init(Ctx& c, int logn, int L, int qbits, int K, int pbits, u64 t, int agg_mode, int slot_rows = 1, int lazy_relin = 0) {
  c.logn = logn; c.N = 1ULL << logn; c.t = t; c.L = L; c.K = K; c.qbits = qbits; c.pbits = pbits;
  c.agg_mode = agg_mode;
  if (slot_rows != 1 && slot_rows != 2) return false;
  c.slot_rows = slot_rows;
  if (lazy_relin != 0 && lazy_relin != 1) return false;
  c.lazy_relin = lazy_relin;
  c.alpha = K; c.dnum = (L + K - 1) / K;
  /* t < 2^26: the integer numerator (Q mod t) m + floor(t/2) of the scaled encoding then stays
     far below 2^64 */
  if (t % (2 * c.N) != 1 || !is_prime(t) || t >= (1ULL << 26)) return false;
  /* Prime choice: the primes q = 1 mod 2N below 2^b in decreasing order; the first K are the
     special primes, the next L the data primes (same width b for both), then tensor primes. */
  if (qbits != pbits) return false;
  /* tensor basis for exact ct x ct: enough extra primes that Q*P*aux > 4 N Q^2 */
  int total = L + K;
  std::vector<u64> pr = ntt_primes(c.N, qbits, L + K + 40);
  if ((int)pr.size() < L + K) return false;
  c.mod.clear();
  for (int i = 0; i < L; i++) c.mod.push_back(pr[K + i]);
  for (int i = 0; i < K; i++) c.mod.push_back(pr[i]);
  std::vector<u64> qs(c.mod.begin(), c.mod.begin() + L), ps(c.mod.begin() + L, c.mod.begin() + L + K);
  c.Q = bprod(qs); c.P = bprod(ps);
  Big need = bmulu(bmul(c.Q, c.Q), 4 * c.N);
  Big have = bmul(c.Q, c.P);
  int aux = 0;
  while (bcmp(have, need) <= 0 && L + K + aux < (int)pr.size()) { have = bmulu(have, pr[L + K + aux]); aux++; }
  c.n_aux = aux;
  /* when the primes of this width run out first, the exact products would wrap: no ct x ct */
  c.has_tensor = bcmp(have, need) > 0;
  for (int i = 0; i < aux; i++) c.mod.push_back(pr[L + K + i]);
  total = L + K + aux;
  c.tab.resize(total);
  for (int i = 0; i < total; i++) c.tab[i].init(c.mod[i], min_primitive_root(c.mod[i], c.N), logn);
  c.ttab.init(t, min_primitive_root(t, c.N), logn);
  /* Slot order: row 0 slot j <-> root zeta^(3^j mod 2N); row 1 slot j <-> zeta^(-3^j mod 2N).
     The NTT index holding the evaluation at zeta^e is k with 2*bitrev(k)+1 = e. */
  c.slot_pos.assign(c.N, 0);
  u64 half = c.N / 2, e = 1;
  for (u64 j = 0; j < half; j++) {
    u64 e1 = 2 * c.N - e;
    c.slot_pos[j] = bitrev((u32)((e - 1) / 2), logn);
    c.slot_pos[half + j] = bitrev((u32)((e1 - 1) / 2), logn);
    e = (e * 3) % (2 * c.N);
  }
  c.crtQ = CrtBasis(qs);
  c.crtT = CrtBasis(c.mod);
  c.Q_mod_t = bmodu(c.Q, t);
  Big qd, qr; bdivmod(c.Q, bfrom(t), qd, qr);
  c.Q_div_t_mod.resize(L);
  for (int i = 0; i < L; i++) c.Q_div_t_mod[i] = bmodu(qd, c.mod[i]);
  return true;
}

/* ------------------------------------------------------------------ plaintext encoding
 * decode: slot j = m(zeta^{e_j}) mod t;  encode is its inverse (N slots -> N coefficients). */
std::vector<u64> decode(const Ctx& c, const std::vector<u64>& m) {
  std::vector<u64> A(m);
  c.ttab.forward(A.data());
  std::vector<u64> slots(c.N);
  for (u64 j = 0; j < c.N; j++) slots[j] = A[c.slot_pos[j]];
  return slots;
}
std::vector<u64> encode(const Ctx& c, const std::vector<u64>& slots) {
  std::vector<u64> A(c.N);
  for (u64 j = 0; j < c.N; j++) A[c.slot_pos[j]] = slots[j] % c.t;
  c.ttab.inverse(A.data());
  return A;
}
/* Plaintext for ct x pt: centered lift of each coefficient (c > (t-1)/2 -> c - t), NTT mod q_i. */
std::vector<u64> plain_ntt(const Ctx& c, const std::vector<u64>& m) {
  std::vector<u64> out((u64)c.L * c.N);
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < c.L; i++) {
    u64* o = limb(out, c.N, i);
    for (u64 k = 0; k < c.N; k++) {
      i64 v = m[k] > (c.t - 1) / 2 ? (i64)m[k] - (i64)c.t : (i64)m[k];
      o[k] = smod(v, c.mod[i]);
    }
    c.tab[i].forward(o);
  }
  return out;
}

/* ------------------------------------------------------------------ keys */
std::vector<u64> make_ksk(Ctx& c, const std::vector<i64>& s_prime, u32 key_id) {
  u64 N = c.N; int LK = c.L + c.K;
  std::vector<u64> out(2ULL * c.dnum * LK * N);
  u64 Pmod[64];
  for (int m = 0; m < c.L; m++) Pmod[m] = bmodu(c.P, c.mod[m]);
  for (int j = 0; j < c.dnum; j++) {
    u64 idx_e = ((u64)key_id << 16) | ((u64)j << 8);
    std::vector<i64> e = sample_gauss(c.keyseed, P_KSK_E, idx_e, N);
    for (int m = 0; m < LK; m++) {
      u64 q = c.mod[m];
      std::vector<u64> a = sample_uniform(c.keyseed, P_KSK_A, idx_e | (u64)m, q, N);
      std::vector<u64> en = ntt_of_int(c, e, m);
      bool in_digit = (m < c.L) && (m / c.alpha == j);
      std::vector<u64> sp;
      if (in_digit) sp = ntt_of_int(c, s_prime, m);
      u64* b = out.data() + (((u64)0 * c.dnum + j) * LK + m) * N;
      u64* A = out.data() + (((u64)1 * c.dnum + j) * LK + m) * N;
      const u64* sn = c.s_ntt.data() + (u64)m * N;
      for (u64 k = 0; k < N; k++) {
        u64 v = submod(en[k], mulmod(a[k], sn[k], q), q);
        if (in_digit) v = addmod(v, mulmod(Pmod[m], sp[k], q), q);
        b[k] = v; A[k] = a[k];
      }
    }
  }
  return out;
}

void keygen(Ctx& c, u64 seed) {
  u64 N = c.N; int total = (int)c.mod.size();
  c.keyseed = seed;
  c.s = sample_ternary(seed, P_SK, 0, N);
  c.s_ntt.assign((u64)total * N, 0);
  for (int m = 0; m < total; m++) {
    std::vector<u64> v = ntt_of_int(c, c.s, m);
    memcpy(c.s_ntt.data() + (u64)m * N, v.data(), N * 8);
  }
  std::vector<i64> e = sample_gauss(seed, P_PK_E, 0, N);
  c.pk0.assign((u64)c.L * N, 0); c.pk1.assign((u64)c.L * N, 0);
  for (int i = 0; i < c.L; i++) {
    u64 q = c.mod[i];
    std::vector<u64> a = sample_uniform(seed, P_PK_A, (u64)i, q, N);
    std::vector<u64> en = ntt_of_int(c, e, i);
    for (u64 k = 0; k < N; k++) {
      c.pk0[(u64)i * N + k] = submod(en[k], mulmod(a[k], c.s_ntt[(u64)i * N + k], q), q);
      c.pk1[(u64)i * N + k] = a[k];
    }
  }
  c.gk.clear();
  c.gk_step.clear();
  c.signed_digits = false;
  for (int i = 0; i < n_pow2(c); i++) {
    std::vector<i64> sg = automorph_int(c.s, galois_elt_key(c, i), N);
    c.gk.push_back(make_ksk(c, sg, rot_key_id(c, i)));
  }
  /* s^2 as an integer negacyclic product (|coeff| <= N) */
  std::vector<i64> s2(N, 0);
  for (u64 i = 0; i < N; i++) {
    if (!c.s[i]) continue;
    for (u64 j = 0; j < N; j++) {
      i64 p = c.s[i] * c.s[j];
      if (!p) continue;
      u64 k = i + j;
      if (k < N) s2[k] += p; else s2[k - N] -= p;
    }
  }
  c.rk = make_ksk(c, s2, 255);
  c.has_keys = true;
}

/* ------------------------------------------------------------------ encrypt / decrypt
 * Ciphertexts: [2][L][N], NTT form.  c0 + c1*s = floor(Q*m/t) + noise (mod Q). */
std::vector<u64> encrypt(Ctx& c, const std::vector<u64>& m, u64 seed, u64 idx) {
  u64 N = c.N;
  std::vector<i64> u = sample_ternary(seed, P_ENC_U, idx, N);
  std::vector<i64> e0 = sample_gauss(seed, P_ENC_E0, idx, N);
  std::vector<i64> e1 = sample_gauss(seed, P_ENC_E1, idx, N);
  std::vector<u64> ct(2ULL * c.L * N);
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < c.L; i++) {
    u64 q = c.mod[i];
    std::vector<u64> un = ntt_of_int(c, u, i);
    std::vector<u64> d(N), f(N);
    for (u64 k = 0; k < N; k++) {
      /* floor(Q*m/t + 1/2) = floor(Q/t)*m + floor(((Q mod t)*m + floor(t/2)) / t) */
      u64 delta = addmod(mulmod(c.Q_div_t_mod[i], m[k], q), (c.Q_mod_t * m[k] + c.t / 2) / c.t, q);
      d[k] = addmod(smod(e0[k], q), delta, q);
      f[k] = smod(e1[k], q);
    }
    c.tab[i].forward(d.data()); c.tab[i].forward(f.data());
    for (u64 k = 0; k < N; k++) {
      ct[(u64)i * N + k] = addmod(mulmod(c.pk0[(u64)i * N + k], un[k], q), d[k], q);
      ct[((u64)c.L + i) * N + k] = addmod(mulmod(c.pk1[(u64)i * N + k], un[k], q), f[k], q);
    }
  }
  return ct;
}

/* [c0 + c1*s]_Q in coefficient form, per limb in [0, q_i). */
std::vector<u64> phase(const Ctx& c, const std::vector<u64>& ct) {
  u64 N = c.N;
  std::vector<u64> x((u64)c.L * N);
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < c.L; i++) {
    u64 q = c.mod[i];
    for (u64 k = 0; k < N; k++)
      x[(u64)i * N + k] = addmod(ct[(u64)i * N + k], mulmod(ct[((u64)c.L + i) * N + k], c.s_ntt[(u64)i * N + k], q), q);
    c.tab[i].inverse(x.data() + (u64)i * N);
  }
  return x;
}

/* m = round(t * x / Q) mod t, x = CRT(phase) in [0, Q). */
std::vector<u64> decrypt(const Ctx& c, const std::vector<u64>& ct) {
  u64 N = c.N;
  std::vector<u64> x = phase(c, ct);
  std::vector<u64> m(N);
  Big twoQ = bshl1(c.Q);
#pragma omp parallel for schedule(dynamic, 64)
  for (u64 k = 0; k < N; k++) {
    std::vector<u64> r(c.L);
    for (int i = 0; i < c.L; i++) r[i] = x[(u64)i * N + k];
    Big X = crt(r, c.crtQ);
    Big num = badd(bmulu(X, 2 * c.t), c.Q); /* floor((2 t X + Q) / 2Q) */
    Big qq, rr; bdivmod(num, twoQ, qq, rr);
    m[k] = bmodu(qq, c.t);
  }
  return m;
}

/* Noise of a ciphertext that should encrypt m: max |[c0 + c1 s - floor(Q m / t + 1/2)]_Q|
   (centered), returned as log2 of the bound.  Used by the tests as an invariant check. */
double noise_log2(const Ctx& c, const std::vector<u64>& ct, const std::vector<u64>& m) {
  u64 N = c.N;
  std::vector<u64> x = phase(c, ct);
  double worst = 0;
  Big halfQ; { Big a, b; bdivmod(c.Q, bfrom(2), a, b); halfQ = a; }
  for (u64 k = 0; k < N; k++) {
    std::vector<u64> r(c.L);
    for (int i = 0; i < c.L; i++) {
      u64 q = c.mod[i];
      u64 delta = addmod(mulmod(c.Q_div_t_mod[i], m[k], q), (c.Q_mod_t * m[k] + c.t / 2) / c.t, q);
      r[i] = submod(x[(u64)i * N + k], delta, q);
    }
    Big X = crt(r, c.crtQ);
    Big mag = bcmp(X, halfQ) > 0 ? bsub(c.Q, X) : X;
    double d = 0;
    for (size_t w = mag.size(); w-- > 0;) d = d * 4294967296.0 + mag[w];
    if (d > worst) worst = d;
  }
  return worst > 0 ? __builtin_log2(worst) : 0.0;
}

/* ------------------------------------------------------------------ homomorphic operations */
void ct_add(const Ctx& c, std::vector<u64>& a, const std::vector<u64>& b) {
  for (int p = 0; p < 2; p++)
    for (int i = 0; i < c.L; i++) {
      u64 q = c.mod[i];
      for (u64 k = 0; k < c.N; k++) {
        u64 o = ((u64)p * c.L + i) * c.N + k;
        a[o] = addmod(a[o], b[o], q);
      }
    }
}
/* HE-CMult: both polynomials times the NTT-form plaintext, slot-wise. */
std::vector<u64> ct_mul_plain(const Ctx& c, const std::vector<u64>& ct, const std::vector<u64>& pt) {
  std::vector<u64> r(ct.size());
  for (int p = 0; p < 2; p++)
    for (int i = 0; i < c.L; i++)
      for (u64 k = 0; k < c.N; k++) {
        u64 o = ((u64)p * c.L + i) * c.N + k;
        r[o] = mulmod(ct[o], pt[(u64)i * c.N + k], c.mod[i]);
      }
  return r;
}

/* Fast basis conversion of coefficient-form residues x_i (source moduli s_i, product S) to a
   target modulus m:  sum_i [x_i * (S/s_i)^-1]_{s_i} * (S/s_i) mod m.  The constants are
   precomputed once per (source set, target). */
struct BasisConv {
  std::vector<u64> src, inv_hat; std::vector<std::vector<u64>> hat_mod; /* [target][i] */
  std::vector<u64> tgt;
  BasisConv() {}
  BasisConv(const std::vector<u64>& s, const std::vector<u64>& targets) : src(s), tgt(targets) {
    for (size_t i = 0; i < s.size(); i++) {
      u64 h = 1;
      for (size_t j = 0; j < s.size(); j++) if (j != i) h = mulmod(h, s[j] % s[i], s[i]);
      inv_hat.push_back(invmod(h, s[i]));
    }
    for (u64 m : targets) {
      std::vector<u64> row;
      for (size_t i = 0; i < s.size(); i++) {
        u64 h = 1;
        for (size_t j = 0; j < s.size(); j++) if (j != i) h = mulmod(h, s[j] % m, m);
        row.push_back(h);
      }
      hat_mod.push_back(row);
    }
  }
  u64 apply(const u64* x, size_t ti) const {
    u64 m = tgt[ti], acc = 0;
    for (size_t i = 0; i < src.size(); i++) {
      u64 y = mulmod(x[i], inv_hat[i], src[i]);
      acc = addmod(acc, mulmod(y % m, hat_mod[ti][i], m), m);
    }
    return acc;
  }
};

/* Hybrid key switching (special modulus P, digits of alpha = K consecutive data primes):
   d (NTT form over Q) under key ksk for s' -> (out0, out1) over Q with out0 + out1*s ~ d*s'.
   ModUp = fast basis conversion from [0, q) residues of each digit; ModDown = (x - Conv_P->Q
   ([x]_P)) * P^-1 mod q_i.  Both from non-centered residues. */
void keyswitch(const Ctx& c, const std::vector<u64>& d, const std::vector<u64>& ksk,
               std::vector<u64>& out0, std::vector<u64>& out1) {
  u64 N = c.N; int L = c.L, K = c.K, LK = L + K;
  std::vector<u64> dc(d);
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < L; i++) c.tab[i].inverse(dc.data() + (u64)i * N);
  std::vector<u64> acc0((u64)LK * N, 0), acc1((u64)LK * N, 0);
  std::vector<u64> all(c.mod.begin(), c.mod.begin() + LK);
  for (int j = 0; j < c.dnum; j++) {
    int lo = j * c.alpha, hi = std::min((j + 1) * c.alpha, L);
    std::vector<u64> src(c.mod.begin() + lo, c.mod.begin() + hi);
    BasisConv conv(src, all);
#pragma omp parallel for schedule(dynamic)
    for (int m = 0; m < LK; m++) {
      u64 q = c.mod[m];
      std::vector<u64> x(hi - lo);
      std::vector<u64> ext(N);
      if (m >= lo && m < hi) {
        memcpy(ext.data(), d.data() + (u64)m * N, N * 8);   /* own limb: already in NTT form */
      } else {
        for (u64 k = 0; k < N; k++) {
          for (int i = lo; i < hi; i++) x[i - lo] = dc[(u64)i * N + k];
          ext[k] = conv.apply(x.data(), (size_t)m);
        }
        c.tab[m].forward(ext.data());
      }
      const u64* kb = ksk.data() + (((u64)0 * c.dnum + j) * LK + m) * N;
      const u64* ka = ksk.data() + (((u64)1 * c.dnum + j) * LK + m) * N;
      for (u64 k = 0; k < N; k++) {
        acc0[(u64)m * N + k] = addmod(acc0[(u64)m * N + k], mulmod(ext[k], kb[k], q), q);
        acc1[(u64)m * N + k] = addmod(acc1[(u64)m * N + k], mulmod(ext[k], ka[k], q), q);
      }
    }
  }
  std::vector<u64> psrc(c.mod.begin() + L, c.mod.begin() + LK), qtgt(c.mod.begin(), c.mod.begin() + L);
  BasisConv down(psrc, qtgt);
  std::vector<u64>* accs[2] = {&acc0, &acc1};
  std::vector<u64>* outs[2] = {&out0, &out1};
  for (int w = 0; w < 2; w++) {
    std::vector<u64>& acc = *accs[w];
    std::vector<u64> pc((u64)K * N);
    for (int k = 0; k < K; k++) {
      memcpy(pc.data() + (u64)k * N, acc.data() + ((u64)L + k) * N, N * 8);
      c.tab[L + k].inverse(pc.data() + (u64)k * N);
    }
    outs[w]->assign((u64)L * N, 0);
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < L; i++) {
      u64 q = c.mod[i];
      std::vector<u64> x(K);
      std::vector<u64> cv(N);
      for (u64 k = 0; k < N; k++) {
        for (int kk = 0; kk < K; kk++) x[kk] = pc[(u64)kk * N + k];
        cv[k] = down.apply(x.data(), (size_t)i);
      }
      c.tab[i].forward(cv.data());
      u64 pinv = invmod(bmodu(c.P, q), q);
      for (u64 k = 0; k < N; k++)
        (*outs[w])[(u64)i * N + k] = mulmod(submod(acc[(u64)i * N + k], cv[k], q), pinv, q);
    }
  }
}

/* Automorphism of an NTT-form polynomial, carried out in the coefficient domain. */
std::vector<u64> automorph_poly_ntt(const Ctx& c, const std::vector<u64>& a, u64 g, int nlimbs) {
  std::vector<u64> r((u64)nlimbs * c.N);
#pragma omp parallel for schedule(dynamic)
  for (int i = 0; i < nlimbs; i++) {
    std::vector<u64> x(a.begin() + (u64)i * c.N, a.begin() + (u64)(i + 1) * c.N);
    c.tab[i].inverse(x.data());
    std::vector<u64> y = automorph_coeff(x, g, c.N, c.mod[i]);
    c.tab[i].forward(y.data());
    memcpy(r.data() + (u64)i * c.N, y.data(), c.N * 8);
  }
  return r;
}

/* One key-switched automorphism (left rotation): (sigma_g(c0) + ks0, ks1), ks = KS(sigma_g(c1))
   with the key for sigma_g(s) -> s. */
std::vector<u64> rotate_with_key(const Ctx& c, const std::vector<u64>& ct, u64 g, const std::vector<u64>& key) {
  u64 LN = (u64)c.L * c.N;
  std::vector<u64> c0(ct.begin(), ct.begin() + LN), c1(ct.begin() + LN, ct.end());
  std::vector<u64> a0 = automorph_poly_ntt(c, c0, g, c.L), a1 = automorph_poly_ntt(c, c1, g, c.L);
  std::vector<u64> k0, k1;
  keyswitch(c, a1, key, k0, k1);
  std::vector<u64> r(2 * LN);
  for (int l = 0; l < c.L; l++)
    for (u64 k = 0; k < c.N; k++) {
      u64 o = (u64)l * c.N + k;
      r[o] = addmod(a0[o], k0[o], c.mod[l]);
      r[LN + o] = k1[o];
    }
  return r;
}
/* HE-Rot by k slots (left, within each row of N/2 slots).  With a rotation key for exactly k,
   one key switch with it; otherwise the power-of-two digits of k (rotation_digits: binary, or
   signed with the right keys), each one rotation with its own key.  Both decrypt to the same rotated slots; their noise (and so
   their limbs) differ. */
std::vector<u64> rotate(const Ctx& c, const std::vector<u64>& ct, u64 k, int* nks) {
  std::vector<u64> r(ct);
  k %= c.N / 2;
  auto it = c.gk_step.find(k);
  if (it != c.gk_step.end()) {
    if (nks) (*nks)++;
    return rotate_with_key(c, r, galois_elt_step(c, k), it->second);
  }
  for (int idx : rotation_digits(c, k)) {
    r = rotate_with_key(c, r, galois_elt_key(c, idx), c.gk[idx]);
    if (nks) (*nks)++;
  }
  return r;
}

/* Adds the right rotation keys (index (logn - 1) + i, right by 2^i); rotations then apply the
   signed digits of the non-adjacent form. */
void add_right_keys(Ctx& c) {
  if (c.signed_digits) return;
  for (int i = n_pow2(c); i < 2 * n_pow2(c); i++) {
    std::vector<i64> sg = automorph_int(c.s, galois_elt_key(c, i), c.N);
    c.gk.push_back(make_ksk(c, sg, rot_key_id(c, i)));
  }
  c.signed_digits = true;
}

/* Adds a rotation key for a left rotation by exactly k slots (k mod N/2; nothing for 0, for a
   power of two, which the power-of-two key already covers, or for a step already held). */
void add_step_key(Ctx& c, u64 k) {
  k %= c.N / 2;
  if (k == 0 || (k & (k - 1)) == 0 || c.gk_step.count(k)) return;
  std::vector<i64> sg = automorph_int(c.s, galois_elt_step(c, k), c.N);
  c.gk_step[k] = make_ksk(c, sg, step_key_id(k));
}

/* HE-Mult (both operands encrypted), before relinearisation: the exact scaled tensor
     (d0, d1, d2) = round(t/Q * (c0 e0, c0 e1 + c1 e0, c1 e1)) mod Q
   of the centered lifts, computed through the exact integer negacyclic products (CRT over the
   data, special and tensor primes, whose product exceeds 4 N Q^2).  Returns [3][L][N], NTT form;
   it decrypts under (1, s, s^2). */
std::vector<u64> ct_tensor(const Ctx& c, const std::vector<u64>& x, const std::vector<u64>& y) {
  u64 N = c.N; int L = c.L, T = (int)c.mod.size();
  Big halfQ; { Big a, b; bdivmod(c.Q, bfrom(2), a, b); halfQ = a; }
  /* centered lifts of the four input polynomials, coefficient form, reduced to every modulus */
  std::vector<std::vector<u64>> lift(4, std::vector<u64>((u64)T * N));
  const std::vector<u64>* srcs[2] = {&x, &y};
  for (int s = 0; s < 2; s++)
    for (int p = 0; p < 2; p++) {
      std::vector<u64> cf((u64)L * N);
#pragma omp parallel for schedule(dynamic)
      for (int i = 0; i < L; i++) {
        memcpy(cf.data() + (u64)i * N, srcs[s]->data() + ((u64)p * L + i) * N, N * 8);
        c.tab[i].inverse(cf.data() + (u64)i * N);
      }
      std::vector<u64>& out = lift[s * 2 + p];
#pragma omp parallel for schedule(dynamic, 64)
      for (u64 k = 0; k < N; k++) {
        std::vector<u64> r(L); for (int i = 0; i < L; i++) r[i] = cf[(u64)i * N + k];
        Big X = crt(r, c.crtQ);
        bool neg = bcmp(X, halfQ) > 0;
        Big mag = neg ? bsub(c.Q, X) : X;
        for (int m = 0; m < T; m++) {
          u64 v = bmodu(mag, c.mod[m]);
          out[(u64)m * N + k] = neg ? negmod(v, c.mod[m]) : v;
        }
      }
#pragma omp parallel for schedule(dynamic)
      for (int m = 0; m < T; m++) c.tab[m].forward(out.data() + (u64)m * N);
    }
  /* exact products over the tensor basis */
  std::vector<std::vector<u64>> prod(3, std::vector<u64>((u64)T * N));
#pragma omp parallel for schedule(dynamic)
  for (int m = 0; m < T; m++) {
    u64 q = c.mod[m];
    for (u64 k = 0; k < N; k++) {
      u64 o = (u64)m * N + k;
      prod[0][o] = mulmod(lift[0][o], lift[2][o], q);
      prod[1][o] = addmod(mulmod(lift[0][o], lift[3][o], q), mulmod(lift[1][o], lift[2][o], q), q);
      prod[2][o] = mulmod(lift[1][o], lift[3][o], q);
    }
  }
  Big M = c.crtT.M, halfM; { Big a, b; bdivmod(M, bfrom(2), a, b); halfM = a; }
  Big twoQ = bshl1(c.Q);
  std::vector<std::vector<u64>> d(3, std::vector<u64>((u64)L * N));
  for (int w = 0; w < 3; w++) {
#pragma omp parallel for schedule(dynamic)
    for (int m = 0; m < T; m++) c.tab[m].inverse(prod[w].data() + (u64)m * N);
#pragma omp parallel for schedule(dynamic, 64)
    for (u64 k = 0; k < N; k++) {
      std::vector<u64> r(T); for (int m = 0; m < T; m++) r[m] = prod[w][(u64)m * N + k];
      Big X = crt(r, c.crtT);
      bool neg = bcmp(X, halfM) > 0;
      Big mag = neg ? bsub(M, X) : X;
      /* round(t*mag/Q) = floor((2 t mag + Q) / 2Q); no ties since t and Q are odd */
      Big qq, rr; bdivmod(badd(bmulu(mag, 2 * c.t), c.Q), twoQ, qq, rr);
      for (int i = 0; i < L; i++) {
        u64 v = bmodu(qq, c.mod[i]);
        d[w][(u64)i * N + k] = neg ? negmod(v, c.mod[i]) : v;
      }
    }
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < L; i++) c.tab[i].forward(d[w].data() + (u64)i * N);
  }
  std::vector<u64> r(3ULL * L * N);
  for (int w = 0; w < 3; w++) memcpy(r.data() + (u64)w * L * N, d[w].data(), (u64)L * N * 8);
  return r;
}
/* Relinearisation of (d0, d1, d2): (d0, d1) + KeySwitch(d2) under the relinearisation key (a key
   switch for s^2 -> s), so the result decrypts under (1, s) to the same plaintext. */
std::vector<u64> relinearize(const Ctx& c, const std::vector<u64>& d3) {
  u64 N = c.N, LN = (u64)c.L * N;
  std::vector<u64> d2(d3.begin() + 2 * LN, d3.end());
  std::vector<u64> k0, k1;
  keyswitch(c, d2, c.rk, k0, k1);
  std::vector<u64> r(2 * LN);
  for (int i = 0; i < c.L; i++)
    for (u64 k = 0; k < N; k++) {
      u64 o = (u64)i * N + k;
      r[o] = addmod(d3[o], k0[o], c.mod[i]);
      r[LN + o] = addmod(d3[LN + o], k1[o], c.mod[i]);
    }
  return r;
}
/* HE-Mult with relinearisation immediately after the product. */
std::vector<u64> ct_mul_ct(const Ctx& c, const std::vector<u64>& x, const std::vector<u64>& y) {
  return relinearize(c, ct_tensor(c, x, y));
}

/* ------------------------------------------------------------------ CSSC (Sec. 4.3, App. B) */
struct Cssc {
  i64 rows = 0; int Lw = 0;       /* Lw = max nonzeros in a row = number of CSSC columns */
  std::vector<i64> nnz_row, VA, CP;
  std::vector<i32> CI, RM;
};
/* CSR -> CSSC: rows sorted by nonzero count, descending (stable: equal counts keep ascending
   row order); the left-aligned rows are read column-major into VA/CI with column pointers CP. */
Cssc csr_to_cssc(i64 R, const i64* row_ptr, const i32* col, const i64* val) {
  Cssc s; s.rows = R;
  s.nnz_row.resize(R);
  i64 Lw = 0;
  for (i64 i = 0; i < R; i++) { s.nnz_row[i] = row_ptr[i + 1] - row_ptr[i]; Lw = std::max(Lw, s.nnz_row[i]); }
  s.Lw = (int)Lw;
  s.RM.resize(R);
  for (i64 i = 0; i < R; i++) s.RM[i] = (i32)i;
  std::stable_sort(s.RM.begin(), s.RM.end(), [&](i32 a, i32 b) { return s.nnz_row[a] > s.nnz_row[b]; });
  s.CP.assign(Lw + 1, 0);
  i64 w = 0;
  for (i64 j = 0; j < Lw; j++) {
    s.CP[j] = w;
    for (i64 p = 0; p < R; p++) {
      i64 i = s.RM[p];
      if (j < s.nnz_row[i]) {
        i64 k = row_ptr[i] + j;
        s.VA.push_back(val[k]); s.CI.push_back(col[k]); w++;
      }
    }
  }
  s.CP[Lw] = w;
  return s;
}

struct Chunk { int start, c; i64 h; };
/* generateChunk with the padded fit rule: column i joins the chunk started at `start` iff
   i < n_C and h * (i - start + 1) <= s, with h = NNZ[start] (paper mode) or NNZ[0] (uniform). */
std::vector<Chunk> make_chunks(const Cssc& m, i64 s, int uniform) {
  std::vector<Chunk> out;
  int nC = m.Lw, i = 0;
  while (i < nC) {
    int start = i;
    i64 h = uniform ? (m.CP[1] - m.CP[0]) : (m.CP[start + 1] - m.CP[start]);
    while (i < nC && h * (i - start + 1) <= s) i++;
    out.push_back(Chunk{start, i - start, h});
  }
  return out;
}
/* Slot k of chunk: block b = k div h, sorted row p = k mod h; value of CSSC column start+b at
   row p when present, else padding. get(idx) maps a CSSC entry index to the slot value. */
template <class F>
void chunk_slots_into(std::vector<u64>& slots, u64 off, const Cssc& m, const Chunk& ch, u64 t, F get) {
  for (i64 b = 0; b < ch.c; b++) {
    int col = ch.start + (int)b;
    if (col >= m.Lw) break;   /* a joint chunk may reach past this partition's columns */
    i64 nn = m.CP[col + 1] - m.CP[col];
    for (i64 p = 0; p < std::min(nn, ch.h); p++) slots[off + b * ch.h + p] = smod(get(m.CP[col] + p), t);
  }
}
template <class F>
std::vector<u64> chunk_slots(const Cssc& m, const Chunk& ch, u64 N, u64 t, F get) {
  std::vector<u64> slots(N, 0);
  chunk_slots_into(slots, 0, m, ch, t, get);
  return slots;
}

/* The joint column profile of two row partitions packed into one ciphertext (slot row 0 and slot
   row 1): column j has height max(NNZ_A[j], NNZ_B[j]) (heights past a partition's last column are
   0), so generateChunk on it gives chunks that fit both rows with the same rotation schedule. */
Cssc joint_profile(const Cssc& a, const Cssc& b) {
  Cssc j; j.Lw = std::max(a.Lw, b.Lw);
  j.CP.assign(j.Lw + 1, 0);
  for (int c = 0; c < j.Lw; c++) {
    i64 na = c < a.Lw ? a.CP[c + 1] - a.CP[c] : 0, nb = c < b.Lw ? b.CP[c + 1] - b.CP[c] : 0;
    j.CP[c + 1] = j.CP[c] + std::max(na, nb);
  }
  return j;
}

u64 num_bits(u64 c) { u64 n = 0; while (c) { n++; c >>= 1; } return n; }

/* Alg. Aggregation, intra-chunk part (totalSum), with the block-add fix:
   e = 1; for j = numBits(c)-2 .. 0: w += Rot(w, e r); e *= 2; if bit_j(c): w = ctV + Rot(w, r);
   e += 1.  Afterwards slot p < r holds the sum over the chunk's c column blocks. */
std::vector<u64> total_sum(const Ctx& c, const std::vector<u64>& ctV, i64 r, i64 ccols, int* nks, int* nrot) {
  std::vector<u64> w(ctV);
  u64 e = 1;
  int nb = (int)num_bits((u64)ccols);
  for (int j = nb - 2; j >= 0; j--) {
    std::vector<u64> rt = rotate(c, w, e * (u64)r, nks); if (nrot) (*nrot)++;
    ct_add(c, w, rt);
    e *= 2;
    if (((u64)ccols >> j) & 1) {
      std::vector<u64> r2 = rotate(c, w, (u64)r, nks); if (nrot) (*nrot)++;
      w = ctV; ct_add(c, w, r2);
      e += 1;
    }
  }
  return w;
}

/* The rotation amounts (mod N/2) that total_sum applies to a chunk of height r and ccols
   columns, in the order it applies them. */
std::vector<u64> total_sum_steps(const Ctx& c, i64 r, i64 ccols) {
  std::vector<u64> out;
  u64 e = 1, half = c.N / 2;
  int nb = (int)num_bits((u64)ccols);
  for (int j = nb - 2; j >= 0; j--) {
    out.push_back((e * (u64)r) % half);
    e *= 2;
    if (((u64)ccols >> j) & 1) { out.push_back((u64)r % half); e += 1; }
  }
  return out;
}

struct Partition { i64 row0, rows; Cssc m; };
/* One result ciphertext: partition pa in slot row 0 and, with two slot rows, partition pb (or -1)
   in slot row 1, sharing the chunks. */
struct Group { int pa, pb; std::vector<Chunk> chunks; };
struct Matrix {
  i64 R = 0, C = 0; int encrypted = 0;
  std::vector<Partition> parts;
  std::vector<Group> groups;
  std::vector<std::vector<u64>> pts;  /* per chunk: NTT-form plaintext [L][N] or ciphertext */
  std::vector<std::vector<u64>> masks; /* per chunk: mask plaintext (paper mode) */
};

}  // namespace

/* ====================================================================== C API (for tests) */
extern "C" {

/* Threads of the OpenMP build (independent limbs and coefficients split across host cores; the
   arithmetic and its order per value are unchanged).  Returns the count in effect; the plain
   build has no OpenMP and always returns 1. */
int orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

void* orc_ctx_new(int logn, int L, int qbits, int K, int pbits, u64 t, int agg_mode, int slot_rows, int lazy_relin) {
  Ctx* c = new Ctx();
  if (!ctx_init(*c, logn, L, qbits, K, pbits, t, agg_mode, slot_rows, lazy_relin)) { delete c; return nullptr; }
  return c;
}
void orc_ctx_free(void* h) { delete (Ctx*)h; }
int orc_n_moduli(void* h) { return (int)((Ctx*)h)->mod.size(); }
int orc_n_aux(void* h) { return ((Ctx*)h)->n_aux; }
void orc_moduli(void* h, u64* out) { Ctx* c = (Ctx*)h; for (size_t i = 0; i < c->mod.size(); i++) out[i] = c->mod[i]; }
u64 orc_psi(void* h, int m) { Ctx* c = (Ctx*)h; return m < 0 ? c->ttab.psi : c->tab[m].psi; }
void orc_slot_pos(void* h, u32* out) { Ctx* c = (Ctx*)h; for (u64 j = 0; j < c->N; j++) out[j] = c->slot_pos[j]; }

/* u64 utilities exposed for pins */
int orc_is_prime(u64 n) { return is_prime(n); }
u64 orc_mulmod(u64 a, u64 b, u64 m) { return mulmod(a, b, m); }
void orc_chacha20_block(const u32* key, u32 counter, const u32* nonce, u32* out) { chacha20_block(key, counter, nonce, out); }
void orc_cdt(u64* out) { for (int i = 0; i < 20; i++) out[i] = ORC_CDT[i]; }
void orc_sample(u64 seed, u32 purpose, u64 index, u64 N, int kind, u64 q, i64* out) {
  if (kind == 0) { auto v = sample_ternary(seed, purpose, index, N); memcpy(out, v.data(), N * 8); }
  else if (kind == 1) { auto v = sample_gauss(seed, purpose, index, N); memcpy(out, v.data(), N * 8); }
  else { auto v = sample_uniform(seed, purpose, index, q, N); memcpy(out, v.data(), N * 8); }
}

void orc_ntt(void* h, int m, u64* a) { Ctx* c = (Ctx*)h; if (m < 0) c->ttab.forward(a); else c->tab[m].forward(a); }
void orc_intt(void* h, int m, u64* a) { Ctx* c = (Ctx*)h; if (m < 0) c->ttab.inverse(a); else c->tab[m].inverse(a); }
void orc_encode(void* h, const u64* slots, u64* m) {
  Ctx* c = (Ctx*)h; std::vector<u64> s(slots, slots + c->N); auto r = encode(*c, s); memcpy(m, r.data(), c->N * 8);
}
void orc_decode(void* h, const u64* m, u64* slots) {
  Ctx* c = (Ctx*)h; std::vector<u64> s(m, m + c->N); auto r = decode(*c, s); memcpy(slots, r.data(), c->N * 8);
}
void orc_plain_ntt(void* h, const u64* m, u64* out) {
  Ctx* c = (Ctx*)h; std::vector<u64> s(m, m + c->N); auto r = plain_ntt(*c, s); memcpy(out, r.data(), r.size() * 8);
}
/* Galois element of rotation key index i (left 2^i for i < logn - 1, else right 2^(i - logn + 1)). */
u64 orc_galois_elt(void* h, int i) { return galois_elt_key(*(Ctx*)h, i); }
/* Adds the optional right rotation keys; the number of power-of-two rotation keys held. */
void orc_add_right_keys(void* h) { add_right_keys(*(Ctx*)h); }
int orc_n_rotation_keys(void* h) { return (int)((Ctx*)h)->gk.size(); }
/* The key switches of a rotation by k (mod N/2) without an exact-step key, as signed steps
   +-2^i in the order applied; returns the count (at most log2 N). */
int orc_rotation_digits(void* h, u64 k, i64* out) {
  Ctx* c = (Ctx*)h; auto v = rotation_digits(*c, k % (c->N / 2));
  for (size_t i = 0; i < v.size(); i++) out[i] = rot_key_step(*c, v[i]);
  return (int)v.size();
}

void orc_keygen(void* h, u64 seed) { keygen(*(Ctx*)h, seed); }
void orc_export_sk(void* h, i64* s) { Ctx* c = (Ctx*)h; memcpy(s, c->s.data(), c->N * 8); }
void orc_export_sk_ntt(void* h, u64* s) { Ctx* c = (Ctx*)h; memcpy(s, c->s_ntt.data(), c->s_ntt.size() * 8); }
void orc_export_pk(void* h, u64* out) {
  Ctx* c = (Ctx*)h; u64 n = (u64)c->L * c->N;
  memcpy(out, c->pk0.data(), n * 8); memcpy(out + n, c->pk1.data(), n * 8);
}
/* key_id < 0: relinearisation key; else rotation key index key_id (left by 2^key_id below
   log2 N - 1, else right by 2^(key_id - log2 N + 1)).  Layout [2][dnum][L+K][N]. */
void orc_export_ksk(void* h, int key_id, u64* out) {
  Ctx* c = (Ctx*)h; const std::vector<u64>& k = key_id < 0 ? c->rk : c->gk[key_id];
  memcpy(out, k.data(), k.size() * 8);
}

void orc_encrypt(void* h, const u64* m, u64 seed, u64 idx, u64* ct) {
  Ctx* c = (Ctx*)h; std::vector<u64> mm(m, m + c->N); auto r = encrypt(*c, mm, seed, idx); memcpy(ct, r.data(), r.size() * 8);
}
void orc_decrypt(void* h, const u64* ct, u64* m) {
  Ctx* c = (Ctx*)h; std::vector<u64> x(ct, ct + 2ULL * c->L * c->N); auto r = decrypt(*c, x); memcpy(m, r.data(), c->N * 8);
}
double orc_noise_log2(void* h, const u64* ct, const u64* m) {
  Ctx* c = (Ctx*)h; std::vector<u64> x(ct, ct + 2ULL * c->L * c->N), mm(m, m + c->N); return noise_log2(*c, x, mm);
}
void orc_ct_mul_plain(void* h, const u64* ct, const u64* pt_ntt, u64* out) {
  Ctx* c = (Ctx*)h; u64 n = 2ULL * c->L * c->N;
  std::vector<u64> x(ct, ct + n), p(pt_ntt, pt_ntt + (u64)c->L * c->N);
  auto r = ct_mul_plain(*c, x, p); memcpy(out, r.data(), n * 8);
}
int orc_ct_mul_ct(void* h, const u64* a, const u64* b, u64* out) {
  Ctx* c = (Ctx*)h; u64 n = 2ULL * c->L * c->N;
  if (!c->has_tensor) return -1;
  std::vector<u64> x(a, a + n), y(b, b + n); auto r = ct_mul_ct(*c, x, y); memcpy(out, r.data(), n * 8);
  return 0;
}
/* The three-component product before relinearisation, [3][L][N] NTT form. */
int orc_ct_tensor(void* h, const u64* a, const u64* b, u64* out) {
  Ctx* c = (Ctx*)h; u64 n = 2ULL * c->L * c->N;
  if (!c->has_tensor) return -1;
  std::vector<u64> x(a, a + n), y(b, b + n); auto r = ct_tensor(*c, x, y); memcpy(out, r.data(), r.size() * 8);
  return 0;
}
int orc_has_tensor(void* h) { return ((Ctx*)h)->has_tensor ? 1 : 0; }
void orc_keyswitch(void* h, const u64* d, int key_id, u64* out) {
  Ctx* c = (Ctx*)h; u64 n = (u64)c->L * c->N;
  std::vector<u64> x(d, d + n), o0, o1;
  keyswitch(*c, x, key_id < 0 ? c->rk : c->gk[key_id], o0, o1);
  memcpy(out, o0.data(), n * 8); memcpy(out + n, o1.data(), n * 8);
}
void orc_automorph_ntt(void* h, const u64* a, u64 g, u64* out) {
  Ctx* c = (Ctx*)h; std::vector<u64> x(a, a + (u64)c->L * c->N); auto r = automorph_poly_ntt(*c, x, g, c->L);
  memcpy(out, r.data(), r.size() * 8);
}
void orc_add_step_keys(void* h, const i64* steps, i64 n) {
  Ctx* c = (Ctx*)h; i64 half = (i64)c->N / 2;
  for (i64 i = 0; i < n; i++) add_step_key(*c, (u64)(((steps[i] % half) + half) % half));
}
/* Exact-step rotation key for k, layout [2][dnum][L+K][N]; returns 0 when none is held. */
int orc_export_step_key(void* h, u64 k, u64* out) {
  Ctx* c = (Ctx*)h; auto it = c->gk_step.find(k % (c->N / 2));
  if (it == c->gk_step.end()) return 0;
  memcpy(out, it->second.data(), it->second.size() * 8);
  return 1;
}
/* Rotation amounts of one chunk's totalSum (at most 2 log2 N of them); returns the count. */
int orc_total_sum_steps(void* h, i64 r, i64 cc, u64* out) {
  auto v = total_sum_steps(*(Ctx*)h, r, cc);
  for (size_t i = 0; i < v.size(); i++) out[i] = v[i];
  return (int)v.size();
}
void orc_rotate(void* h, const u64* ct, u64 k, u64* out) {
  Ctx* c = (Ctx*)h; u64 n = 2ULL * c->L * c->N; std::vector<u64> x(ct, ct + n);
  auto r = rotate(*c, x, k, nullptr); memcpy(out, r.data(), n * 8);
}
void orc_total_sum(void* h, const u64* ct, i64 r, i64 cc, u64* out) {
  Ctx* c = (Ctx*)h; u64 n = 2ULL * c->L * c->N; std::vector<u64> x(ct, ct + n);
  auto w = total_sum(*c, x, r, cc, nullptr, nullptr); memcpy(out, w.data(), n * 8);
}

/* CSR -> CSSC into caller arrays (VA, CI sized nnz; RM sized R; CP sized Lw+1). Returns Lw. */
int orc_cssc_lw(i64 R, const i64* row_ptr) {
  i64 Lw = 0; for (i64 i = 0; i < R; i++) Lw = std::max(Lw, row_ptr[i + 1] - row_ptr[i]); return (int)Lw;
}
void orc_cssc(i64 R, const i64* row_ptr, const i32* col, const i64* val, i64* VA, i32* CI, i32* RM, i64* CP) {
  Cssc s = csr_to_cssc(R, row_ptr, col, val);
  if (!s.VA.empty()) { memcpy(VA, s.VA.data(), s.VA.size() * 8); memcpy(CI, s.CI.data(), s.CI.size() * 4); }
  if (R) memcpy(RM, s.RM.data(), R * 4);
  memcpy(CP, s.CP.data(), s.CP.size() * 8);
}
/* chunk descriptors (start, c, h) for a CSSC column-pointer array; returns the count. */
int orc_chunks(int Lw, const i64* CP, i64 s, int uniform, i64* out3) {
  Cssc m; m.Lw = Lw; m.CP.assign(CP, CP + Lw + 1);
  auto ch = make_chunks(m, s, uniform);
  for (size_t i = 0; i < ch.size(); i++) { out3[3 * i] = ch[i].start; out3[3 * i + 1] = ch[i].c; out3[3 * i + 2] = ch[i].h; }
  return (int)ch.size();
}

/* ---- whole protocol (Alg. Sparse Matrix-Vector Multiplication) ----
 * Client A: row partitions of s = N/2 rows (Sec. 4.7), CSSC, chunks, slot packing, encoding (and
 * encryption of the values with mat_seed when encrypted != 0). */
void* orc_matrix_new(void* h, i64 R, i64 C, const i64* row_ptr, const i32* col, const i64* val,
                     int encrypted, u64 mat_seed) {
  Ctx* c = (Ctx*)h;
  if (encrypted && !c->has_tensor) return nullptr;
  Matrix* M = new Matrix(); M->R = R; M->C = C; M->encrypted = encrypted;
  i64 s = (i64)c->N / 2;
  u64 ct_idx = 0;
  for (i64 r0 = 0; r0 < R; r0 += s) {
    Partition P; P.row0 = r0; P.rows = std::min(s, R - r0);
    std::vector<i64> rp(P.rows + 1);
    for (i64 i = 0; i <= P.rows; i++) rp[i] = row_ptr[r0 + i] - row_ptr[r0];
    P.m = csr_to_cssc(P.rows, rp.data(), col + row_ptr[r0], val + row_ptr[r0]);
    M->parts.push_back(P);
  }
  const int nP = (int)M->parts.size();
  for (int p = 0; p < nP; p += c->slot_rows) {
    Group G; G.pa = p; G.pb = (c->slot_rows == 2 && p + 1 < nP) ? p + 1 : -1;
    G.chunks = G.pb < 0 ? make_chunks(M->parts[p].m, s, c->agg_mode == 1)
                        : make_chunks(joint_profile(M->parts[p].m, M->parts[G.pb].m), s, c->agg_mode == 1);
    for (const Chunk& ch : G.chunks) {
      std::vector<u64> slots(c->N, 0);
      const Cssc& ma = M->parts[G.pa].m;
      chunk_slots_into(slots, 0, ma, ch, c->t, [&](i64 k) { return ma.VA[k]; });
      if (G.pb >= 0) {
        const Cssc& mb = M->parts[G.pb].m;
        chunk_slots_into(slots, c->N / 2, mb, ch, c->t, [&](i64 k) { return mb.VA[k]; });
      }
      std::vector<u64> mcoef = encode(*c, slots);
      if (encrypted) M->pts.push_back(encrypt(*c, mcoef, mat_seed, ct_idx));
      else M->pts.push_back(plain_ntt(*c, mcoef));
      ct_idx++;
      if (c->agg_mode == 0) {
        std::vector<u64> ms(c->N, 0);
        for (i64 p2 = 0; p2 < ch.h; p2++) {
          ms[p2] = 1;
          if (G.pb >= 0) ms[c->N / 2 + p2] = 1;
        }
        M->masks.push_back(plain_ntt(*c, encode(*c, ms)));
      }
    }
    M->groups.push_back(G);
  }
  return M;
}
void orc_matrix_free(void* m) { delete (Matrix*)m; }
int orc_matrix_n_parts(void* m) { return (int)((Matrix*)m)->parts.size(); }
int orc_matrix_n_groups(void* m) { return (int)((Matrix*)m)->groups.size(); }
int orc_matrix_n_chunks(void* m) { return (int)((Matrix*)m)->pts.size(); }
/* chunk k (global numbering): out = (group = result ciphertext, start, c, h); with one slot row a
   group is a partition */
void orc_matrix_chunk(void* m, int k, i64* out4) {
  Matrix* M = (Matrix*)m; int g = 0;
  for (size_t p = 0; p < M->groups.size(); p++)
    for (const Chunk& ch : M->groups[p].chunks) {
      if (g == k) { out4[0] = (i64)p; out4[1] = ch.start; out4[2] = ch.c; out4[3] = ch.h; return; }
      g++;
    }
}
void orc_matrix_pt(void* m, int k, u64* out) { Matrix* M = (Matrix*)m; memcpy(out, M->pts[k].data(), M->pts[k].size() * 8); }
void orc_matrix_mask(void* m, int k, u64* out) { Matrix* M = (Matrix*)m; memcpy(out, M->masks[k].data(), M->masks[k].size() * 8); }

/* Client B: reorganised vector per chunk (Alg. reorgVector), encoded and encrypted; ciphertext
   index = global chunk number.  out: [n_chunks][2][L][N]. */
void orc_encrypt_vector(void* h, void* m, const i64* v, u64 seed, u64* out) {
  Ctx* c = (Ctx*)h; Matrix* M = (Matrix*)m; u64 ctsz = 2ULL * c->L * c->N; u64 g = 0;
  for (const Group& G : M->groups)
    for (const Chunk& ch : G.chunks) {
      std::vector<u64> slots(c->N, 0);
      const Cssc& ma = M->parts[G.pa].m;
      chunk_slots_into(slots, 0, ma, ch, c->t, [&](i64 k) { return v[ma.CI[k]]; });
      if (G.pb >= 0) {
        const Cssc& mb = M->parts[G.pb].m;
        chunk_slots_into(slots, c->N / 2, mb, ch, c->t, [&](i64 k) { return v[mb.CI[k]]; });
      }
      auto ct = encrypt(*c, encode(*c, slots), seed, g);
      memcpy(out + g * ctsz, ct.data(), ctsz * 8);
      g++;
    }
}

/* Cloud: per chunk HE product, totalSum, mask (paper mode), sum per group (partition, or pair of
   partitions with two slot rows).  x: [n_chunks][2][L][N]; out: [n_groups][2][L][N].  stats
   (optional): [key switches, rotations].
   Lazy relinearisation (encrypted matrix values, lazy_relin = 1; not in the paper, which
   relinearises after every product): a chunk of one column has no totalSum rotation, so its
   unrelinearised product (d0, d1, d2) is masked component by component and summed with the
   group's other such chunks; the sum is relinearised once and added to the group's result.
   The mask product and the sum are linear in each component, so the result decrypts to the
   same plaintext; only its limbs (noise) differ. */
void orc_he_spmv(void* h, void* m, const u64* x, u64* out, i64* stats) {
  Ctx* c = (Ctx*)h; Matrix* M = (Matrix*)m; u64 ctsz = 2ULL * c->L * c->N, LN = (u64)c->L * c->N;
  int g = 0, nks = 0, nrot = 0;
  for (size_t p = 0; p < M->groups.size(); p++) {
    std::vector<u64> res(ctsz, 0), lazy;
    for (const Chunk& ch : M->groups[p].chunks) {
      std::vector<u64> xv(x + (u64)g * ctsz, x + (u64)(g + 1) * ctsz);
      if (M->encrypted && c->lazy_relin && ch.c == 1) {
        std::vector<u64> d3 = ct_tensor(*c, M->pts[g], xv);
        if (lazy.empty()) lazy.assign(3 * LN, 0);
        for (int w = 0; w < 3; w++)
          for (int i = 0; i < c->L; i++)
            for (u64 k = 0; k < c->N; k++) {
              u64 o = (u64)w * LN + (u64)i * c->N + k, q = c->mod[i];
              u64 v = c->agg_mode == 0 ? mulmod(d3[o], M->masks[g][(u64)i * c->N + k], q) : d3[o];
              lazy[o] = addmod(lazy[o], v, q);
            }
        g++;
        continue;
      }
      std::vector<u64> prod = M->encrypted ? ct_mul_ct(*c, M->pts[g], xv) : ct_mul_plain(*c, xv, M->pts[g]);
      std::vector<u64> w = total_sum(*c, prod, ch.h, ch.c, &nks, &nrot);
      if (c->agg_mode == 0) w = ct_mul_plain(*c, w, M->masks[g]);
      ct_add(*c, res, w);
      g++;
    }
    if (!lazy.empty()) ct_add(*c, res, relinearize(*c, lazy));
    memcpy(out + p * ctsz, res.data(), ctsz * 8);
  }
  if (stats) { stats[0] = nks; stats[1] = nrot; }
}

/* Secret-key holder: decrypt each partition's result and scatter with the row map; rows with no
   nonzeros get 0.  y: [R], centered in (-t/2, t/2]. */
void orc_decrypt_result(void* h, void* m, const u64* res, i64* y) {
  Ctx* c = (Ctx*)h; Matrix* M = (Matrix*)m; u64 ctsz = 2ULL * c->L * c->N;
  for (size_t gi = 0; gi < M->groups.size(); gi++) {
    const Group& G = M->groups[gi];
    std::vector<u64> ct(res + gi * ctsz, res + (gi + 1) * ctsz);
    std::vector<u64> slots = decode(*c, decrypt(*c, ct));
    for (int half = 0; half < 2; half++) {
      const int pi = half == 0 ? G.pa : G.pb;
      if (pi < 0) continue;
      const Partition& P = M->parts[pi];
      const u64 off = half == 0 ? 0 : c->N / 2;
      i64 nz = P.m.Lw > 0 ? P.m.CP[1] - P.m.CP[0] : 0;
      for (i64 q = 0; q < P.rows; q++) {
        i64 row = P.row0 + P.m.RM[q];
        if (q < nz) { u64 s = slots[off + q]; y[row] = s > c->t / 2 ? (i64)s - (i64)c->t : (i64)s; }
        else y[row] = 0;
      }
    }
  }
}

/* ---- the paper's diagonal baseline (Sec. 5, baseline approaches; the diagonal-method figure) ----
 * The matrix is cut into square blocks of side B = min(N/4, max(R, C)) (zero padded at the right
 * and bottom edges).  Block (bi, bj) keeps its non-zero generalised diagonals d:
 * diag[i] = A[bi B + i][bj B + (i + d) mod B], each encoded as one plaintext (slots [0, B) of row
 * 0).  Vector block bj is encrypted twice over (x_bj || x_bj in slots [0, 2B)), so a left rotation
 * by d puts x_bj[(i + d) mod B] in slot i.  Result block bi = sum over its diagonals (bj, d) of
 * diag (.) Rot(x_bj, d), in (bj, d) order; the product of block row bi lies in slots [0, B). */
struct DiagM {
  i64 R = 0, C = 0, B = 0; int nrb = 0, ncb = 0;
  std::vector<i64> key;                 /* per diagonal: bi, bj, d (3 words), sorted */
  std::vector<std::vector<u64>> pts;    /* NTT-form plaintexts */
};
void* orc_diag_new(void* h, i64 R, i64 C, const i64* row_ptr, const i32* col, const i64* val) {
  Ctx* c = (Ctx*)h;
  DiagM* D = new DiagM(); D->R = R; D->C = C;
  D->B = std::min<i64>((i64)c->N / 4, std::max<i64>(std::max<i64>(R, C), 1));
  D->nrb = (int)((R + D->B - 1) / D->B); D->ncb = (int)((C + D->B - 1) / D->B);
  std::map<std::array<i64, 3>, std::vector<i64>> diags;
  for (i64 r = 0; r < R; r++)
    for (i64 k = row_ptr[r]; k < row_ptr[r + 1]; k++) {
      i64 cc = col[k], bi = r / D->B, bj = cc / D->B, i = r % D->B, j = cc % D->B;
      i64 d = ((j - i) % D->B + D->B) % D->B;
      auto& v = diags[{bi, bj, d}];
      if (v.empty()) v.assign(D->B, 0);
      v[i] = val[k];
    }
  for (auto& kv : diags) {
    std::vector<u64> slots(c->N, 0);
    for (i64 i = 0; i < D->B; i++) slots[i] = smod(kv.second[i], c->t);
    D->pts.push_back(plain_ntt(*c, encode(*c, slots)));
    for (int q = 0; q < 3; q++) D->key.push_back(kv.first[q]);
  }
  return D;
}
void orc_diag_free(void* d) { delete (DiagM*)d; }
int orc_diag_count(void* d) { return (int)((DiagM*)d)->pts.size(); }
void orc_diag_info(void* d, i64* out5) {
  DiagM* D = (DiagM*)d; out5[0] = D->B; out5[1] = D->nrb; out5[2] = D->ncb; out5[3] = (i64)D->pts.size(); out5[4] = 0;
}
void orc_diag_key(void* d, int k, i64* out3) { DiagM* D = (DiagM*)d; for (int q = 0; q < 3; q++) out3[q] = D->key[3 * (size_t)k + q]; }
void orc_diag_pt(void* d, int k, u64* out) { DiagM* D = (DiagM*)d; memcpy(out, D->pts[k].data(), D->pts[k].size() * 8); }
/* vector blocks, each x_bj || x_bj, encrypted with (seed, index bj): out [ncb][2][L][N] */
void orc_diag_encrypt_vector(void* h, void* d, const i64* v, u64 seed, u64* out) {
  Ctx* c = (Ctx*)h; DiagM* D = (DiagM*)d; u64 ctsz = 2ULL * c->L * c->N;
  for (int bj = 0; bj < D->ncb; bj++) {
    std::vector<u64> slots(c->N, 0);
    for (i64 j = 0; j < D->B; j++) {
      i64 cc = bj * D->B + j;
      u64 x = cc < D->C ? smod(v[cc], c->t) : 0;
      slots[j] = x; slots[D->B + j] = x;
    }
    auto ct = encrypt(*c, encode(*c, slots), seed, (u64)bj);
    memcpy(out + bj * ctsz, ct.data(), ctsz * 8);
  }
}
/* out [nrb][2][L][N]; stats (optional): [diagonal products] */
void orc_diag_spmv(void* h, void* d, const u64* x, u64* out, i64* stats) {
  Ctx* c = (Ctx*)h; DiagM* D = (DiagM*)d; u64 ctsz = 2ULL * c->L * c->N;
  std::map<std::pair<i64, i64>, std::vector<u64>> rot;   /* (bj, d) -> Rot(x_bj, d) */
  for (int bi = 0; bi < D->nrb; bi++) {
    std::vector<u64> res(ctsz, 0);
    for (size_t k = 0; k < D->pts.size(); k++) {
      if (D->key[3 * k] != bi) continue;
      i64 bj = D->key[3 * k + 1], dd = D->key[3 * k + 2];
      auto it = rot.find({bj, dd});
      if (it == rot.end()) {
        std::vector<u64> xb(x + bj * ctsz, x + (bj + 1) * ctsz);
        it = rot.emplace(std::make_pair(bj, dd), dd ? rotate(*c, xb, (u64)dd, nullptr) : xb).first;
      }
      ct_add(*c, res, ct_mul_plain(*c, it->second, D->pts[k]));
    }
    memcpy(out + bi * ctsz, res.data(), ctsz * 8);
  }
  if (stats) stats[0] = (i64)D->pts.size();
}
/* y [R] centered: row bi B + i from slot i of result block bi */
void orc_diag_decrypt(void* h, void* d, const u64* res, i64* y) {
  Ctx* c = (Ctx*)h; DiagM* D = (DiagM*)d; u64 ctsz = 2ULL * c->L * c->N;
  for (int bi = 0; bi < D->nrb; bi++) {
    std::vector<u64> ct(res + bi * ctsz, res + (bi + 1) * ctsz);
    std::vector<u64> slots = decode(*c, decrypt(*c, ct));
    for (i64 i = 0; i < D->B && bi * D->B + i < D->R; i++) {
      u64 sv = slots[i];
      y[bi * D->B + i] = sv > c->t / 2 ? (i64)sv - (i64)c->t : (i64)sv;
    }
  }
}

}  // extern "C"
