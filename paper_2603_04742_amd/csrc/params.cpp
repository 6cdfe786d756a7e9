// Host-side parameter generation for the encrypted-SpMV library: NTT-friendly primes, roots of
// unity, twiddle tables, slot order and the RNS constants used by the kernels.
#include <algorithm>
#include <cstring>

#include "hs_internal.hpp"

namespace hs {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }
const char* last_error_cstr() { return g_last_error.c_str(); }

u64 mul_mod(u64 a, u64 b, u64 m) { return (u64)((u128)a * b % m); }
u64 pow_mod(u64 b, u64 e, u64 m) {
  u64 acc = 1 % m;
  for (b %= m; e; e >>= 1, b = mul_mod(b, b, m))
    if (e & 1) acc = mul_mod(acc, b, m);
  return acc;
}
u64 inv_mod(u64 a, u64 q) { return pow_mod(a % q, q - 2, q); }  // q prime

// Miller-Rabin with the first twelve primes as witnesses: deterministic below 2^64.
bool is_prime_u64(u64 n) {
  static const u64 W[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (u64 w : W)
    if (n % w == 0) return n == w;
  int r = __builtin_ctzll(n - 1);
  u64 d = (n - 1) >> r;
  for (u64 w : W) {
    u64 x = pow_mod(w, d, n);
    if (x == 1 || x == n - 1) continue;
    int i = 1;
    for (; i < r; i++) {
      x = mul_mod(x, x, n);
      if (x == n - 1) break;
    }
    if (i == r) return false;
  }
  return true;
}

// Largest primes below 2^bits that are 1 mod 2N, in decreasing order.
std::vector<u64> primes_1_mod_2n(u64 N, int bits, int count) {
  std::vector<u64> r;
  const u64 m = 2 * N, limit = 1ULL << bits;
  for (u64 q = ((limit - 1) / m) * m + 1; (int)r.size() < count && q > m; q -= m)
    if (q < limit && is_prime_u64(q)) r.push_back(q);
  return r;
}

// Smallest primitive 2N-th root of unity mod q.  Any x^((q-1)/2N) whose N-th power is -1 has
// order exactly 2N; all such roots are its odd powers.
u64 smallest_root_2n(u64 q, u64 N) {
  u64 g = 0;
  for (u64 x = 2; !g; x++) {
    u64 c = pow_mod(x, (q - 1) / (2 * N), q);
    if (pow_mod(c, N, q) == q - 1) g = c;
  }
  const u64 g2 = mul_mod(g, g, q);
  u64 best = g;
  for (u64 k = 1, cur = g; k < N; k++) {
    cur = mul_mod(cur, g2, q);
    best = std::min(best, cur);
  }
  return best;
}

static u32 bit_reverse(u32 x, int bits) {
  u32 r = 0;
  for (int i = 0; i < bits; i++, x >>= 1) r = (r << 1) | (x & 1);
  return r;
}

// little-endian multiword helpers
typedef std::vector<u64> Words;
static Words words_mul_small(const Words& a, u64 v) {
  Words r(a.size() + 1, 0);
  u128 carry = 0;
  for (size_t i = 0; i < a.size(); i++) {
    u128 p = (u128)a[i] * v + carry;
    r[i] = (u64)p;
    carry = p >> 64;
  }
  r[a.size()] = (u64)carry;
  while (r.size() > 1 && r.back() == 0) r.pop_back();
  return r;
}
static Words words_product(const std::vector<u64>& ms) {
  Words r{1};
  for (u64 m : ms) r = words_mul_small(r, m);
  return r;
}
static int words_cmp(const Words& a, const Words& b) {
  if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
  for (size_t i = a.size(); i-- > 0;)
    if (a[i] != b[i]) return a[i] < b[i] ? -1 : 1;
  return 0;
}
static u64 words_mod(const Words& a, u64 m) {
  u128 r = 0;
  for (size_t i = a.size(); i-- > 0;) r = ((r << 64) | a[i]) % m;
  return (u64)r;
}
static Words words_shl1(const Words& a, u64 bit_in) {
  Words r(a.size() + 1, 0);
  u64 carry = bit_in;
  for (size_t i = 0; i < a.size(); i++) {
    r[i] = (a[i] << 1) | carry;
    carry = a[i] >> 63;
  }
  r[a.size()] = carry;
  while (r.size() > 1 && r.back() == 0) r.pop_back();
  return r;
}
static Words words_sub(const Words& a, const Words& b) {  // a >= b
  Words r(a.size(), 0);
  u64 br = 0;
  for (size_t i = 0; i < a.size(); i++) {
    const u64 y = i < b.size() ? b[i] : 0;
    const u64 d = a[i] - y;
    const u64 b1 = a[i] < y;
    r[i] = d - br;
    const u64 b2 = d < br;
    br = b1 | b2;
  }
  while (r.size() > 1 && r.back() == 0) r.pop_back();
  return r;
}
static Words words_add(const Words& a, const Words& b) {
  Words r(std::max(a.size(), b.size()) + 1, 0);
  u64 c = 0;
  for (size_t i = 0; i + 1 < r.size(); i++) {
    const u64 x = i < a.size() ? a[i] : 0, y = i < b.size() ? b[i] : 0;
    const u64 s = x + y;
    const u64 c1 = s < x;
    r[i] = s + c;
    const u64 c2 = r[i] < s;
    c = c1 | c2;
  }
  r.back() = c;
  while (r.size() > 1 && r.back() == 0) r.pop_back();
  return r;
}
static Words words_shr1(const Words& a) {
  Words r(a.size(), 0);
  for (size_t i = 0; i < a.size(); i++) r[i] = (a[i] >> 1) | (i + 1 < a.size() ? a[i + 1] << 63 : 0);
  while (r.size() > 1 && r.back() == 0) r.pop_back();
  return r;
}
// floor(2^s / d) by binary long division
static Words words_pow2_div(int s, const Words& d) {
  Words q(s / 64 + 1, 0), r{0};
  for (int bit = s; bit >= 0; bit--) {
    r = words_shl1(r, bit == s ? 1 : 0);
    if (words_cmp(r, d) >= 0) {
      r = words_sub(r, d);
      q[bit / 64] |= 1ULL << (bit % 64);
    }
  }
  while (q.size() > 1 && q.back() == 0) q.pop_back();
  return q;
}
static std::vector<u64> padded(const Words& w, int n) {
  std::vector<u64> r(n, 0);
  for (size_t i = 0; i < w.size() && (int)i < n; i++) r[i] = w[i];
  return r;
}

static u64 product_mod(const std::vector<u64>& ms, u64 m) {
  u64 r = 1 % m;
  for (u64 x : ms) r = mul_mod(r, x % m, m);
  return r;
}

template <class T>
static T* upload(const std::vector<T>& v) {
  T* d = nullptr;
  if (v.empty()) return nullptr;
  HS_CHECK_HIP(hipMalloc(&d, v.size() * sizeof(T)));
  HS_CHECK_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return d;
}

size_t ct_words(const hs_ctx* c) { return 2ULL * c->L * c->N; }

void build_ctx(hs_ctx* c) {
  const hs_params& p = c->prm;
  HS_REQUIRE(p.log_n >= 3 && p.log_n <= 15, HS_EPARAM, "log_n must be in [3, 15]");
  HS_REQUIRE(p.n_q >= 1 && p.n_p >= 1 && p.n_q <= 32 && p.n_p <= 4, HS_EPARAM, "need 1 <= n_q <= 32 and 1 <= n_p <= 4");
  HS_REQUIRE(p.q_bits == p.p_bits && p.q_bits >= 20 && p.q_bits <= 50, HS_EPARAM, "prime widths must be equal and in [20, 50]");
  HS_REQUIRE(p.sigma == 3.2, HS_EPARAM, "only sigma = 3.2 is supported");
  c->logn = (int)p.log_n;
  c->N = 1ULL << c->logn;
  c->t = p.t;
  // t < 2^26 keeps (Q mod t) m + floor(t/2) of the scaled encoding below 2^53, so the encryption
  // kernels' double quotient is exact
  HS_REQUIRE(is_prime_u64(c->t) && c->t % (2 * c->N) == 1 && c->t < (1ULL << 26), HS_EPARAM,
             "t must be a prime < 2^26 with t = 1 mod 2N");
  HS_REQUIRE(p.agg_mode <= 1, HS_EPARAM, "agg_mode must be 0 or 1");
  HS_REQUIRE(p.slot_rows <= 2, HS_EPARAM, "slot_rows must be 0, 1 or 2");
  HS_REQUIRE(p.relin_mode <= 1, HS_EPARAM, "relin_mode must be 0 or 1");
  c->L = (int)p.n_q;
  c->K = (int)p.n_p;
  c->alpha = c->K;
  c->dnum = (c->L + c->alpha - 1) / c->alpha;
  bool tensor_basis_ok = false;

  // tensor primes for the exact ct x ct: enough that prod(all) > 4 N Q^2
  std::vector<u64> pr = primes_1_mod_2n(c->N, (int)p.q_bits, c->L + c->K + 48);
  HS_REQUIRE((int)pr.size() >= c->L + c->K, HS_EPARAM, "not enough NTT-friendly primes of that width");
  c->mod.clear();
  for (int i = 0; i < c->L; i++) c->mod.push_back(pr[c->K + i]);
  for (int i = 0; i < c->K; i++) c->mod.push_back(pr[i]);
  {
    // smallest number of further primes with prod(data, special, tensor) > 4 N Q^2
    std::vector<u64> qq(c->mod.begin(), c->mod.begin() + c->L);
    std::vector<u64> need_f(qq);
    need_f.insert(need_f.end(), qq.begin(), qq.end());
    need_f.push_back(4 * c->N);
    const Words need = words_product(need_f);
    std::vector<u64> have_f(c->mod);
    int aux = 0;
    while (words_cmp(words_product(have_f), need) <= 0 && c->L + c->K + aux < (int)pr.size()) {
      have_f.push_back(pr[c->L + c->K + aux]);
      aux++;
    }
    c->n_aux = aux;
    for (int i = 0; i < aux; i++) c->mod.push_back(pr[c->L + c->K + i]);
    // when the NTT-friendly primes of this width run out first, the basis cannot hold the exact
    // products: the ciphertext product stays unavailable (HS_EPARAM) rather than wrap
    tensor_basis_ok = words_cmp(words_product(have_f), need) > 0;
  }
  c->n_mod = (int)c->mod.size();

  // roots and twiddles for every modulus, plus the plaintext modulus t (last)
  std::vector<u64> all(c->mod);
  all.push_back(c->t);
  const u64 N = c->N;
  std::vector<double2> tw(all.size() * 2 * N);
  std::vector<double> twc(all.size() * N);
  c->psi.clear();
  c->h_tab.assign(all.size(), ModTab{});
  std::vector<u64> pw(N);
  for (size_t mi = 0; mi < all.size(); mi++) {
    const u64 q = all[mi];
    const u64 psi = smallest_root_2n(q, N);
    c->psi.push_back(psi);
    pw[0] = 1;
    for (u64 k = 1; k < N; k++) pw[k] = mul_mod(pw[k - 1], psi, q);
    double2* fw = &tw[mi * 2 * N];
    double2* iv = fw + N;
    for (u64 i = 0; i < N; i++) {
      const u32 r = bit_reverse((u32)i, c->logn);
      fw[i] = make_const(pw[r], q);
      twc[mi * N + i] = (double)pw[r];
      iv[i] = make_const(r == 0 ? 1 : q - pw[N - r], q);  // psi^-r = -psi^(N-r)
    }
    ModTab& t = c->h_tab[mi];
    t.q = (double)q;
    t.qinv = 1.0 / (double)q;
    t.ninv = make_const(inv_mod(N % q, q), q);
  }
  c->d_tw = upload(tw);
  c->d_twc = upload(twc);
  for (size_t mi = 0; mi < all.size(); mi++) {
    c->h_tab[mi].fw = c->d_tw + mi * 2 * N;
    c->h_tab[mi].iv = c->d_tw + mi * 2 * N + N;
    c->h_tab[mi].fwc = c->d_twc + mi * N;
  }
  c->d_tab = upload(c->h_tab);

  // slot order: row 0 slot j <-> zeta^(3^j), row 1 slot j <-> zeta^(-3^j) (mod 2N exponents)
  std::vector<u32> pos(N);
  u64 e = 1;
  for (u64 j = 0; j < N / 2; j++) {
    pos[j] = bit_reverse((u32)((e - 1) / 2), c->logn);
    const u64 e1 = 2 * N - e;
    pos[N / 2 + j] = bit_reverse((u32)((e1 - 1) / 2), c->logn);
    e = e * 3 % (2 * N);
  }
  c->d_slot_pos = upload(pos);

  const int L = c->L, K = c->K, LK = L + K;
  std::vector<u64> qs(c->mod.begin(), c->mod.begin() + L), ps(c->mod.begin() + L, c->mod.begin() + LK);
  // floor(Q/t) mod q_i = -(Q mod t) * t^-1 mod q_i, since Q = 0 mod q_i
  c->q_mod_t = product_mod(qs, c->t);
  std::vector<double2> qdt(L), pmod(L), pinv(L);
  for (int i = 0; i < L; i++) {
    const u64 q = qs[i];
    const u64 v = mul_mod((q - c->q_mod_t % q) % q, inv_mod(c->t % q, q), q);
    qdt[i] = make_const(v, q);
    const u64 pm = product_mod(ps, q);
    pmod[i] = make_const(pm, q);
    pinv[i] = make_const(inv_mod(pm, q), q);
  }
  c->d_qdt = upload(qdt);
  c->d_pmod = upload(pmod);
  c->d_pinv = upload(pinv);

  // ModUp constants per digit
  std::vector<double2> up_inv((size_t)c->dnum * c->alpha, double2{0, 0}), up_hat((size_t)c->dnum * c->alpha * LK, double2{0, 0});
  for (int j = 0; j < c->dnum; j++) {
    const int lo = j * c->alpha, hi = std::min(L, lo + c->alpha);
    std::vector<u64> D(qs.begin() + lo, qs.begin() + hi);
    for (int a = 0; a < hi - lo; a++) {
      std::vector<u64> others;
      for (int b = 0; b < hi - lo; b++)
        if (b != a) others.push_back(D[b]);
      up_inv[(size_t)j * c->alpha + a] = make_const(inv_mod(product_mod(others, D[a]), D[a]), D[a]);
      for (int m = 0; m < LK; m++) up_hat[((size_t)j * c->alpha + a) * LK + m] = make_const(product_mod(others, c->mod[m]), c->mod[m]);
    }
  }
  c->d_up_inv = upload(up_inv);
  c->d_up_hat = upload(up_hat);
  // ModDown constants
  std::vector<double2> dn_inv(K), dn_hat((size_t)K * L);
  for (int k = 0; k < K; k++) {
    std::vector<u64> others;
    for (int b = 0; b < K; b++)
      if (b != k) others.push_back(ps[b]);
    dn_inv[k] = make_const(inv_mod(product_mod(others, ps[k]), ps[k]), ps[k]);
    for (int i = 0; i < L; i++) dn_hat[(size_t)k * L + i] = make_const(product_mod(others, qs[i]), qs[i]);
  }
  c->d_dn_inv = upload(dn_inv);
  c->d_dn_hat = upload(dn_hat);

  // decryption constants
  Words Q = words_product(qs);
  c->dec_words = (int)Q.size() + 1;
  std::vector<double2> dinv(L);
  std::vector<u64> dhat((size_t)L * c->dec_words, 0), dq(c->dec_words, 0);
  for (int i = 0; i < L; i++) {
    std::vector<u64> others;
    for (int b = 0; b < L; b++)
      if (b != i) others.push_back(qs[b]);
    Words hat = words_product(others);
    dinv[i] = make_const(inv_mod(words_mod(hat, qs[i]), qs[i]), qs[i]);
    for (size_t w = 0; w < hat.size(); w++) dhat[(size_t)i * c->dec_words + w] = hat[w];
  }
  for (size_t w = 0; w < Q.size(); w++) dq[w] = Q[w];
  c->d_dec_inv = upload(dinv);
  c->d_dec_hat = upload(dhat);
  c->d_dec_q = upload(dq);

  // exact ciphertext product: CRT over all n_mod moduli (M > 4 N Q^2), Barrett division by 2Q
  {
    const int T = c->n_mod;
    const Words M = words_product(c->mod);
    const int WQ = c->dec_words;
    const int WM = (int)M.size() + 1;
    Words tM = words_mul_small(M, c->t);
    const Words A_max = words_add(tM, Q);
    const int WA = (int)A_max.size() + 1;
    const Words D = words_shl1(Q, 0);
    const int WD = (int)D.size();
    // word capacity of the tensor kernels: the widest value (S mod M with one spare word, A, the
    // CRT sum mod Q with one spare word) rounded up to an instantiated size
    const int need = std::max(std::max(WM + 1, WA), WQ + 1);
    const int kw = need <= 8 ? 8 : need <= 16 ? 16 : need <= 24 ? 24 : 0;
    const Words mu = words_pow2_div(64 * std::max(kw, 1), D);
    const int WMU = (int)mu.size();
    if (tensor_basis_ok && kw && WMU <= kw) {
      std::vector<double2> minv(T), r32(T);
      std::vector<u64> mhat((size_t)T * WM, 0);
      for (int i = 0; i < T; i++) {
        std::vector<u64> others;
        for (int j = 0; j < T; j++)
          if (j != i) others.push_back(c->mod[j]);
        const Words h = words_product(others);
        minv[i] = make_const(inv_mod(words_mod(h, c->mod[i]), c->mod[i]), c->mod[i]);
        for (size_t w = 0; w < h.size(); w++) mhat[(size_t)i * WM + w] = h[w];
        r32[i] = make_const((1ULL << 32) % c->mod[i], c->mod[i]);
      }
      c->tq_words = WQ; c->tm_words = WM; c->td_words = WD; c->tmu_words = WMU; c->ta_words = WA; c->t_kw = kw;
      c->d_t_halfq = upload(padded(words_shr1(Q), WQ));
      c->d_t_mhat_inv = upload(minv);
      c->d_t_mhat = upload(mhat);
      c->d_t_m = upload(padded(M, WM + 1));
      c->d_t_halfm = upload(padded(words_shr1(M), WM));
      c->d_t_d = upload(padded(D, WD));
      c->d_t_mu = upload(padded(mu, WMU + 1));
      c->d_t_r32 = upload(r32);
      c->has_tensor = true;
    }
  }
}

void free_ctx(hs_ctx* c) {
  void* ptrs[] = {c->d_tab, c->d_tw, c->d_twc, c->d_slot_pos, c->d_qdt, c->d_pmod, c->d_pinv, c->d_up_inv,
                  c->d_up_hat, c->d_dn_inv, c->d_dn_hat, c->d_dec_inv, c->d_dec_hat, c->d_dec_q,
                  c->d_t_halfq, c->d_t_mhat_inv, c->d_t_mhat, c->d_t_m, c->d_t_halfm, c->d_t_d, c->d_t_mu, c->d_t_r32};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
    c->side = nullptr;
  }
  for (hipEvent_t e : c->async_ev) {
    (void)hipEventSynchronize(e);
    (void)hipEventDestroy(e);
  }
  c->async_ev.clear();
  c->pool.release_all();
}

// ------------------------------------------------------------------ pool
void* Pool::get(size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  {
    std::lock_guard<std::mutex> g(mu_);
    auto it = free_.lower_bound(bytes);
    if (it != free_.end() && it->first <= bytes + bytes / 4) {
      void* p = it->second;
      free_.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    release_all();
    e = hipMalloc(&p, bytes);
    if (e != hipSuccess) throw Error{HS_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed"};
  }
  std::lock_guard<std::mutex> g(mu_);
  size_of_[p] = bytes;
  return p;
}
void* Arena::get(size_t bytes) {
  const size_t b = (bytes + 255) & ~(size_t)255;
  if (b > cap_ - used_)
    throw Error{HS_ENOMEM, "the fixed scratch region holds " + std::to_string(cap_) + " bytes; this call needs more than " +
                               std::to_string(used_ + b)};
  void* p = base_ + used_;
  used_ += b;
  return p;
}
void Pool::put(void* p) {
  std::lock_guard<std::mutex> g(mu_);
  auto it = size_of_.find(p);
  if (it != size_of_.end()) free_.emplace(it->second, p);
}
void Pool::release_all() {
  std::lock_guard<std::mutex> g(mu_);
  for (auto& kv : free_) {
    (void)hipFree(kv.second);
    size_of_.erase(kv.second);
  }
  free_.clear();
}

}  // namespace hs
