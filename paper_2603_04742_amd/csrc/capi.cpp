// C ABI of the encrypted-SpMV library: host orchestration of the HIP kernels.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <stdexcept>
#include <thread>
#include <unordered_map>

#include "kernels.hpp"
#include "extra.hpp"

namespace hs {
const char* last_error_cstr();

static thread_local int64_t g_counters[5] = {0, 0, 0, 0, 0};

// process-wide options (hs_set_option)
// process-wide defaults of the execution options, by HS_OPT_* key (hs_set_option); a context's own
// setting (hs_ctx_set_option) takes precedence.  Every default is 0 (automatic).
static std::atomic<int> g_opt[10] = {{0}, {0}, {0}, {0}, {0}, {0}, {0}, {0}, {0}, {0}};
int option(const hs_ctx* c, int key) {
  if (key <= 0 || key >= 10) return 0;
  if (c && c->opt[key] >= 0) return c->opt[key];
  return g_opt[key].load();
}

template <class F>
static int guarded(F&& f) {
  try {
    f();
    return HS_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return HS_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return HS_EINVAL;
  }
}

static hipStream_t S(void* s) { return (hipStream_t)s; }

template <class T>
static void h2d(T* d, const T* h, size_t n, hipStream_t st) {
  if (n) HS_CHECK_HIP(hipMemcpyAsync(d, h, n * sizeof(T), hipMemcpyHostToDevice, st));
}
template <class T>
static void d2h(T* h, const T* d, size_t n, hipStream_t st) {
  if (n) HS_CHECK_HIP(hipMemcpyAsync(h, d, n * sizeof(T), hipMemcpyDeviceToHost, st));
}
// Matrices and ciphertext vectors take their device memory from the context's pool (returned on
// destroy): hipMalloc/hipFree per object cost tens of microseconds each and hipFree waits for the
// device.  Every API call that writes such an object synchronises its stream before returning,
// except the plaintext encoding of hs_cssc_pack, which finishes on the context's side stream
// (M->ready); destroy waits for the whole device, so memory handed back on destroy is idle.
template <class T>
static T* pmalloc(hs_ctx* c, size_t n) {
  return (T*)c->pool.get((n ? n : 1) * sizeof(T));
}
static void pfree(hs_ctx* c, void* p) {
  if (p) c->pool.put(p);
}
// Calls that return with work still in flight on the caller's stream (hs_mul_plain,
// hs_ctvec_copy, hs_batch_plan_run) record an event here; destroying a matrix or a vector waits
// for these events (and for the matrix's own encoding) before its memory goes back to the pool.
// Every other call synchronises its stream before returning, so no wait for the whole device is
// needed.
static void note_async(hs_ctx* c, hipStream_t st) {
  std::lock_guard<std::mutex> g(c->async_mu);
  for (size_t i = 0; i < c->async_ev.size();)  // drop completed ones
    if (hipEventQuery(c->async_ev[i]) == hipSuccess) {
      (void)hipEventDestroy(c->async_ev[i]);
      c->async_ev[i] = c->async_ev.back();
      c->async_ev.pop_back();
    } else {
      i++;
    }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
    (void)hipStreamSynchronize(st);  // no event: finish the work instead
    return;
  }
  if (hipEventRecord(e, st) != hipSuccess) {
    (void)hipEventDestroy(e);
    (void)hipStreamSynchronize(st);
    return;
  }
  c->async_ev.push_back(e);
}
static void drain_async(hs_ctx* c) {
  std::lock_guard<std::mutex> g(c->async_mu);
  for (hipEvent_t e : c->async_ev) {
    (void)hipEventSynchronize(e);
    (void)hipEventDestroy(e);
  }
  c->async_ev.clear();
}
// Pinned host staging per thread for the structure copies of hs_cssc_pack (pageable copies cost
// a driver-side staging copy and a wait each).  Every call that uses it synchronises its stream
// before returning, so a thread's buffer is never in use by two copies at once.  The buffers live
// until the process ends (freeing pinned memory from thread-exit handlers can run after the HIP
// runtime has shut down).
struct PinnedStage {
  void* p = nullptr;
  size_t bytes = 0;
  void* get(size_t n) {
    if (n > bytes) {
      if (p) (void)hipHostFree(p);
      p = nullptr;
      bytes = 0;
      const size_t want = std::max<size_t>(n + n / 2, 1 << 16);
      if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) throw Error{HS_ENOMEM, "pinned host allocation failed"};
      bytes = want;
    }
    return p;
  }
};
static thread_local PinnedStage t_stage_down, t_stage_up;
template <class T>
static T* dmalloc(size_t n) {
  T* p = nullptr;
  if (!n) n = 1;
  if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) throw Error{HS_ENOMEM, "device allocation failed"};
  return p;
}

// ------------------------------------------------------------------ Gaussian CDT (library copy)
// T[k] = floor(2^63 P(|e| <= k)) for the discrete Gaussian with sigma = 3.2 truncated at 19,
// rho(x) = exp(-x^2 / 20.48).  Computed in 128-bit fixed point with 120 fractional bits:
// exp(-x) = (exp(-x/64))^64 with a 40-term Taylor series; the ratio by binary long division.
static u128 fx_mul(u128 a, u128 b) {
  const u64 a0 = (u64)a, a1 = (u64)(a >> 64), b0 = (u64)b, b1 = (u64)(b >> 64);
  const u128 p00 = (u128)a0 * b0, p01 = (u128)a0 * b1, p10 = (u128)a1 * b0, p11 = (u128)a1 * b1;
  const u128 mid = (p00 >> 64) + (u64)p01 + (u64)p10;
  const u128 hi = p11 + (p01 >> 64) + (p10 >> 64) + (mid >> 64);
  return (hi << 8) | ((u64)mid >> 56);
}
static void compute_cdt(u64 out[20]) {
  const int F = 120;
  const u128 one = (u128)1 << F;
  u128 rho[20];
  for (int j = 0; j < 20; j++) {
    // y = 25 j^2 / 2^15  (= x / 64 with x = j^2 / 20.48 = 25 j^2 / 512)
    const u128 y = (u128)(25 * j * j) << (F - 15);
    u128 sum = one, term = one;
    for (int n = 1; n <= 40; n++) {
      term = fx_mul(term, y) / (u128)n;
      if (n & 1) sum -= term; else sum += term;
    }
    for (int sq = 0; sq < 6; sq++) sum = fx_mul(sum, sum);
    rho[j] = sum;
  }
  u128 cum[20];
  u128 acc = rho[0];
  cum[0] = acc;
  for (int k = 1; k < 20; k++) { acc += 2 * rho[k]; cum[k] = acc; }
  const u128 total = cum[19];
  for (int k = 0; k < 19; k++) {
    u128 rem = cum[k];
    u64 q = 0;
    for (int bit = 62; bit >= 0; bit--) {
      rem <<= 1;
      if (rem >= total) { rem -= total; q |= 1ULL << bit; }
    }
    out[k] = q;
  }
  out[19] = 1ULL << 63;
}

// ------------------------------------------------------------------ sampling purposes
enum : u32 { P_SK = 1, P_PK_A = 2, P_PK_E = 3, P_KSK_A = 4, P_KSK_E = 5, P_ENC_U = 6, P_ENC_E0 = 7, P_ENC_E1 = 8 };
static const u32 RELIN_ID = 255;

// Left rotation by k slots within each slot row (k < 0: right by -k): Galois element 3^k mod 2N
// (Sec. 2.1, HE-Rot); 3 has order N/2 modulo 2N, so k is taken mod N/2.
static u64 galois_step(const hs_ctx* c, i64 k) {
  const i64 half = (i64)c->N / 2;
  return pow_mod(3, (u64)(((k % half) + half) % half), 2 * c->N);
}
// Power-of-two rotation keys (Sec. 5): key index i < log2 N - 1 rotates left by 2^i; the optional
// right keys (hs_keyset_add_right_rotation_keys), index log2 N - 1 + i, rotate right by 2^i.
// Sampling ids: i, and 64 + i; RELIN_ID above them.
static int n_pow2(const hs_ctx* c) { return c->logn - 1; }
static i64 key_index_step(const hs_ctx* c, int idx) { return idx < n_pow2(c) ? (1LL << idx) : -(1LL << (idx - n_pow2(c))); }
static u32 key_index_id(const hs_ctx* c, int idx) { return idx < n_pow2(c) ? (u32)idx : 64u + (u32)(idx - n_pow2(c)); }
// Sampling id of the exact-step rotation key for k: above the power-of-two ids and RELIN_ID.
static u32 step_key_id(i64 k) { return 256u + (u32)k; }
static bool is_pow2(i64 k) { return k > 0 && (k & (k - 1)) == 0; }
// Key of a rotation micro-op: a power-of-two key (+-2^i), or the exact-step key for k.
static const u64* rotation_key(const hs_keyset* ks, i64 step) {
  if (is_pow2(step)) return ks->gk[__builtin_ctzll((unsigned long long)step)];
  if (is_pow2(-step)) return ks->gk[n_pow2(ks->ctx) + __builtin_ctzll((unsigned long long)-step)];
  auto it = ks->step_keys.find(step);
  if (it == ks->step_keys.end()) throw Error{HS_EKEY, "internal: no rotation key for a planned step"};
  return it->second;
}
// The key switches of a left rotation by k slots, 0 <= k < N/2, in the order they are applied:
// one with the exact-step key when the key-set holds one for k; otherwise, lowest first, the
// binary digits of k (left keys only), or with the right keys the digits of the non-adjacent
// form of k (signed binary digits, no two adjacent ones nonzero, which has the fewest nonzero
// digits of any signed binary expansion), each a power-of-two rotation +-2^i, a digit of N/2
// (a whole row, the identity) left out.
static std::vector<i64> rotation_digits(const hs_ctx* c, const hs_keyset* ks, i64 k) {
  std::vector<i64> out;
  if (!is_pow2(k) && ks->step_keys.count(k)) {
    out.push_back(k);
    return out;
  }
  if ((int)ks->gk.size() < 2 * n_pow2(c)) {
    for (int i = 0; i < n_pow2(c); i++)
      if ((k >> i) & 1) out.push_back(1LL << i);
    return out;
  }
  const i64 half = (i64)c->N / 2;
  for (i64 v = k, bit = 1; v; v >>= 1, bit <<= 1) {
    if (!(v & 1)) continue;
    const i64 z = (v & 3) == 1 ? 1 : -1;
    if (bit < half) out.push_back(z * bit);
    v -= z;
  }
  return out;
}

// ------------------------------------------------------------------ key generation
static bool use_split(const hs_ctx* c);
static void ntt_any(hs_ctx* c, u64* data, i64 rows, int nl, int mod0, int inverse, hipStream_t st, std::vector<DBuf>& hold,
                    Alloc* al = nullptr);

static u64* make_ksk(hs_ctx* c, hs_keyset* ks, u32 key_id, int sprime_mode, u32 galois, hipStream_t st) {
  const int LK = c->L + c->K;
  const size_t N = c->N;
  u64* key = dmalloc<u64>(2ULL * c->dnum * LK * N);
  DBuf e(&c->pool, (size_t)c->dnum * N * sizeof(int));
  launch_sample_small(c, e.as<int>(), c->dnum, (i64)N, ks->seed, P_KSK_E, ((u64)key_id << 16), 1ULL << 8, 1, st);
  std::vector<KskArgs> args;
  std::vector<u64> ps(c->mod.begin() + c->L, c->mod.begin() + LK);
  for (int j = 0; j < c->dnum; j++) {
    for (int m = 0; m < LK; m++) {
      const u64 q = c->mod[m];
      KskArgs a{};
      a.b = key + (((size_t)0 * c->dnum + j) * LK + m) * N;
      a.a = key + (((size_t)1 * c->dnum + j) * LK + m) * N;
      a.e_coef = e.as<int>() + (size_t)j * N;
      a.sk = ks->sk + (size_t)m * N;
      a.mod_index = m;
      a.seed = ks->seed;
      a.purpose_a = P_KSK_A;
      a.idx_a = ((u64)key_id << 16) | ((u64)j << 8) | (u64)m;
      a.sprime_mode = sprime_mode;
      a.galois = galois;
      const bool in_digit = m < c->L && m / c->alpha == j;
      u64 pm = 1;
      for (u64 p : ps) pm = mul_mod(pm, p % q, q);
      a.pfac = in_digit ? make_const(pm, q) : double2{0.0, 0.0};
      const u64 r64 = (u64)(((u128)1 << 64) % q);
      a.r64 = make_const(r64, q);
      args.push_back(a);
    }
  }
  DBuf dargs(&c->pool, args.size() * sizeof(KskArgs));
  h2d(dargs.as<KskArgs>(), args.data(), args.size(), st);
  if (use_split(c)) {
    // e_j reduced to every modulus, transformed, then combined with a, s and s'
    std::vector<DBuf> hold;
    DBuf en(&c->pool, (size_t)c->dnum * LK * N * sizeof(u64));
    launch_ints_to_limbs(c, e.as<int>(), (i64)N, c->dnum, en.as<u64>(), LK, 0, st);
    ntt_any(c, en.as<u64>(), (i64)c->dnum * LK, LK, 0, 0, st, hold);
    launch_ksk_combine(c, dargs.as<KskArgs>(), en.as<u64>(), (int)args.size(), st);
    HS_CHECK_HIP(hipStreamSynchronize(st));
  } else {
    launch_ksk_limbs(c, dargs.as<KskArgs>(), (int)args.size(), st);
    HS_CHECK_HIP(hipStreamSynchronize(st));
  }
  return key;
}

// ------------------------------------------------------------------ CSSC structure (host)
static std::vector<hs_chunk> make_chunks(const std::vector<i64>& cp, i64 s, int uniform, int part) {
  std::vector<hs_chunk> out;
  const int nC = (int)cp.size() - 1;
  int i = 0;
  while (i < nC) {
    const int start = i;
    const i64 h = uniform ? cp[1] - cp[0] : cp[start + 1] - cp[start];
    while (i < nC && h * (i - start + 1) <= s) i++;
    out.push_back(hs_chunk{part, start, i - start, h});
  }
  return out;
}

// ------------------------------------------------------------------ he_spmv plan
// Micro-op of a chunk's totalSum: one key-switched rotation by `step` slots, in -> out (+ addend).
struct MicroOp {
  int in, out, addend;  // buffer ids per chunk: 0 = V (product), 1 = WA, 2 = WB, 3 = TA, 4 = TB; -1 none
  i64 step;             // a power of two, or a step the key-set holds an exact key for
};

// The rotation amounts (mod N/2) of one chunk's totalSum, in the order it applies them.
static std::vector<i64> total_sum_steps(const hs_ctx* c, i64 r, int cols) {
  std::vector<i64> out;
  const i64 half = (i64)c->N / 2;
  i64 e = 1;
  const int nb = 32 - __builtin_clz((unsigned)cols);
  for (int j = nb - 2; j >= 0; j--) {
    out.push_back((e * r) % half);
    e *= 2;
    if ((cols >> j) & 1) { out.push_back(r % half); e += 1; }
  }
  return out;
}

static std::vector<MicroOp> total_sum_program(const hs_ctx* c, const hs_keyset* ks, i64 r, int cols, int* n_logical) {
  std::vector<MicroOp> prog;
  int w = 0;  // current accumulator buffer
  i64 e = 1;
  const int nb = 32 - __builtin_clz((unsigned)cols);
  const i64 half = (i64)c->N / 2;
  auto rotate_into = [&](int src, i64 amount, int addend) {
    // rotation by `amount` as one key switch when the key-set holds a key for the whole step,
    // else as its power-of-two digits (rotation_digits); the last one lands in the W buffer
    // that is not the current accumulator, plus `addend`
    const std::vector<i64> bits = rotation_digits(c, ks, amount % half);
    if (bits.empty()) throw Error{HS_EINVAL, "internal: zero rotation in totalSum"};
    const int dst_w = (w == 1) ? 2 : 1;
    int cur = src;
    for (size_t b = 0; b < bits.size(); b++) {
      const bool last = b + 1 == bits.size();
      const int dst = last ? dst_w : (cur == 3 ? 4 : 3);
      prog.push_back(MicroOp{cur, dst, last ? addend : -1, bits[b]});
      cur = dst;
    }
    if (n_logical) (*n_logical)++;
    w = dst_w;
  };
  for (int j = nb - 2; j >= 0; j--) {
    rotate_into(w, e * r, w);     // w <- w + Rot(w, e r)
    e *= 2;
    if ((cols >> j) & 1) {
      rotate_into(w, r, 0);       // w <- ctV + Rot(w, r)
      e += 1;
    }
  }
  (void)e;
  prog.push_back(MicroOp{w, w, -2, -1});  // terminal marker: result buffer id
  return prog;
}

static KsShape ks_shape(const hs_ctx* c, int B) {
  KsShape S{};
  S.L = c->L; S.K = c->K; S.alpha = c->alpha; S.dnum = c->dnum;
  const int LK = c->L + c->K;
  int ndg = (512 + LK * B - 1) / (LK * B);
  ndg = std::max(1, std::min(ndg, c->dnum));
  S.dpg = (c->dnum + ndg - 1) / ndg;
  S.ndg = (c->dnum + S.dpg - 1) / S.dpg;
  return S;
}

// Levels of batched power-of-two rotations: every item of a level is independent of the others;
// level k + 1 may read what level k wrote.  All item arrays are uploaded once and the scratch is
// sized for the widest level, so the launches of all levels are enqueued without host waits.
static bool lds_limb_fits(const hs_ctx* c) { return c->logn <= 14; }

// Pipeline choice for one level of B rotations: the one-workgroup-per-limb kernels move the least
// data and win when the level has enough (target modulus x item) pairs to fill the GPU; the
// two-pass kernels spread each transform over N / 2048 workgroups and win for small levels.
// Batch-size bucket of the tuned pipeline table: B = 1 -> 0, 2 -> 1, 3..4 -> 2, ..., > 64 -> 7.
static int ks_bucket(int B) {
  int b = 0;
  while ((1 << b) < B && b < 7) b++;
  return b;
}

static bool use_two_pass(const hs_ctx* c, int B) {
  const int opt = option(c, HS_OPT_KS_PIPELINE);
  if (!lds_limb_fits(c)) return true;
  if (opt == 1) return false;
  if (opt == 2) return true;
  const int pick = c->ks_pick[ks_bucket(B)];
  if (pick >= 0) return pick == 1;
  // untuned default: the crossover measured on MI355X, about 28 items per level at N = 2^14 with the
  // register-accumulator ModUp (which halves the one-workgroup pipeline's time on large levels),
  // about 73 otherwise
  int thr = option(c, HS_OPT_KS_THRESHOLD);
  if (thr == 0) thr = (c->logn == 14 && option(c, HS_OPT_MODUP_ACC) != 1) ? 192 : 512;
  return (c->L + c->K) * B < thr;
}

// Scratch, item arrays and per-level shapes of a sequence of rotation levels (prepared on the
// host, then enqueued without host waits; the enqueue step alone can be captured into a graph).
struct LevelPlan {
  std::vector<int> B;
  std::vector<int> B1;      // two-pass levels: items that run their own first step (K1)
  std::vector<char> fused;  // two-pass level whose last kernel runs the next level's K1 for some items
  std::vector<KsShape> shape;
  std::vector<char> two;
  DBuf ditems, D, ACC, PC, T1, E, ACC2, T2, F;
  int64_t key_switches = 0, launches = 0;
};

// Cross-level fusion of consecutive two-pass levels: an item of level k + 1 whose input is the
// output of an item of level k gets its first step (Galois gather + inverse low pass of c1, K1)
// from that item's last kernel (K5); the level's items are reordered so that those still needing
// K1 come first.  One successor per output (a second item reading the same input keeps its K1).
static void fuse_levels(const hs_ctx* c, std::vector<std::vector<RotItem>>& lv, const std::vector<char>& two, std::vector<int>& B1,
                        std::vector<char>& fused) {
  const size_t nl = lv.size();
  B1.assign(nl, 0);
  fused.assign(nl, 0);
  for (size_t k = 0; k < nl; k++) B1[k] = (int)lv[k].size();
  if (option(c, HS_OPT_KS_FUSE) == 1) return;
  for (size_t k = 0; k + 1 < nl; k++) {
    if (!two[k] || !two[k + 1]) continue;
    std::map<const u64*, int> prod;   // output buffer -> item of level k
    for (size_t p = 0; p < lv[k].size(); p++) prod[lv[k][p].out] = (int)p;
    std::vector<int> pred(lv[k + 1].size(), -1);
    std::vector<char> taken(lv[k].size(), 0);
    for (size_t j = 0; j < lv[k + 1].size(); j++) {
      auto f = prod.find(lv[k + 1][j].in);
      if (f != prod.end() && !taken[f->second]) { pred[j] = f->second; taken[f->second] = 1; }
    }
    std::vector<RotItem> re;
    std::vector<int> rp;
    re.reserve(lv[k + 1].size());
    for (int pass = 0; pass < 2; pass++)
      for (size_t j = 0; j < lv[k + 1].size(); j++)
        if ((pred[j] >= 0) == (pass == 1)) { re.push_back(lv[k + 1][j]); rp.push_back(pred[j]); }
    int nk1 = 0;
    for (size_t j = 0; j < re.size(); j++) {
      if (rp[j] < 0) { nk1++; continue; }
      lv[k][rp[j]].next = (u32)(j + 1);
      fused[k] = 1;
    }
    lv[k + 1] = std::move(re);
    B1[k + 1] = nk1;
  }
}

static void prepare_levels(hs_ctx* c, const std::vector<std::vector<RotItem>>& levels_in, hipStream_t st, LevelPlan& P, Alloc& al) {
  size_t total = 0, widest = 0;
  std::vector<std::vector<RotItem>> levels;
  for (auto& l : levels_in) {
    if (l.empty()) continue;
    total += l.size();
    widest = std::max(widest, l.size());
    levels.push_back(l);
    for (auto& it : levels.back()) it.next = 0;
  }
  if (!total) return;
  const size_t N = c->N;
  const int LK = c->L + c->K;
  bool any1 = false, any2 = false;
  for (auto& l : levels) {
    const bool t = use_two_pass(c, (int)l.size());
    P.B.push_back((int)l.size());
    P.shape.push_back(ks_shape(c, (int)l.size()));
    P.two.push_back(t ? 1 : 0);
    if (t) any2 = true; else any1 = true;
    P.key_switches += (int64_t)l.size();
  }
  fuse_levels(c, levels, P.two, P.B1, P.fused);
  for (size_t k = 0; k < levels.size(); k++) P.launches += P.two[k] ? (P.B1[k] > 0 ? 5 : 4) : 4;
  std::vector<RotItem> flat;
  flat.reserve(total);
  for (auto& l : levels) flat.insert(flat.end(), l.begin(), l.end());
  const KsShape Smax = ks_shape(c, 1);  // the most digit groups any level uses
  P.ditems = DBuf(&al, total * sizeof(RotItem));
  if (any1) {
    P.D = DBuf(&al, widest * c->L * N * sizeof(u64));
    P.ACC = DBuf(&al, widest * Smax.ndg * 2 * LK * N * sizeof(double));
    P.PC = DBuf(&al, widest * 2 * c->K * N * sizeof(double));
  }
  if (any2) {
    P.T1 = DBuf(&al, widest * c->L * N * sizeof(double));
    P.E = DBuf(&al, widest * c->dnum * LK * N * sizeof(double));
    P.ACC2 = DBuf(&al, widest * 2 * c->L * N * sizeof(double));
    P.T2 = DBuf(&al, widest * 2 * c->K * N * sizeof(double));
    P.F = DBuf(&al, widest * 2 * c->L * N * sizeof(double));
  }
  h2d(P.ditems.as<RotItem>(), flat.data(), flat.size(), st);
}

static void enqueue_levels(hs_ctx* c, const LevelPlan& P, hipStream_t st) {
  size_t off = 0;
  for (size_t lv = 0; lv < P.B.size(); lv++) {
    const int B = P.B[lv];
    const RotItem* items = P.ditems.as<RotItem>() + off;
    if (P.two[lv]) {
      launch_rotate_batch2(c, items, B, P.shape[lv], P.T1.as<double>(), P.E.as<double>(), P.ACC2.as<double>(), P.T2.as<double>(),
                           P.F.as<double>(), st, P.B1[lv], P.fused[lv] ? items + B : nullptr);
    } else {
      launch_rotate_batch(c, items, B, P.shape[lv], P.D.as<u64>(), P.ACC.as<double>(), P.PC.as<double>(), st);
    }
    off += B;
  }
}

static void run_rotation_levels(hs_ctx* c, const std::vector<std::vector<RotItem>>& levels, hipStream_t st, Alloc* al = nullptr) {
  LevelPlan P;
  prepare_levels(c, levels, st, P, al ? *al : c->pool);
  enqueue_levels(c, P, st);
  g_counters[0] += P.key_switches;
  g_counters[2] += P.launches;
  // the item array and scratch return to the pool: wait until the kernels are done with them
  HS_CHECK_HIP(hipStreamSynchronize(st));
}

// Transform helper: one-workgroup-per-limb kernels when the limb fits in LDS (unless the two-pass
// path is requested), else the two-pass kernels with a scratch buffer kept in `hold` until the
// caller synchronises.
// Batched transform of `rows` limbs: one workgroup per limb, or the two-pass form (N / 2048
// workgroups per limb) for limbs larger than LDS and, automatically, for a handful of limbs, whose
// one-workgroup transforms would occupy a few CUs for a whole transform's latency.
static constexpr i64 kTwoPassMaxRows = 16, kTwoPassMaxRows14 = 64;  // N = 2^14: 512-element blocks
// N = 2^15 (a limb exceeds LDS): one workgroup per limb on half-limb LDS for batches that fill
// the GPU (k_ntt15, one workgroup per CU), the two-pass transforms below that
static constexpr i64 kOneWgMinRows15 = 256;
static bool ntt15_one_wg(const hs_ctx* c, i64 rows) {
  const int opt = option(c, HS_OPT_NTT_PATH);
  return c->logn == 15 && opt != 2 && (opt == 1 || rows >= kOneWgMinRows15);
}
static void ntt_any(hs_ctx* c, u64* data, i64 rows, int nl, int mod0, int inverse, hipStream_t st, std::vector<DBuf>& hold,
                    Alloc* al) {
  if (rows <= 0) return;
  const int opt = option(c, HS_OPT_NTT_PATH);
  const i64 two_max = c->logn == 14 ? kTwoPassMaxRows14 : kTwoPassMaxRows;
  if (ntt15_one_wg(c, rows)) {
    launch_ntt(c, data, rows, nl, mod0, inverse, st);
  } else if (!lds_limb_fits(c) || opt == 2 || (opt == 0 && c->logn >= 12 && rows <= two_max)) {
    hold.emplace_back(al ? al : &c->pool, (size_t)rows * c->N * sizeof(double));
    launch_ntt2(c, data, hold.back().as<double>(), rows, nl, mod0, inverse, st);
  } else {
    launch_ntt(c, data, rows, nl, mod0, inverse, st);
  }
}

// keygen / encoding / encryption / decryption as elementwise kernels around batched transforms
static bool use_split(const hs_ctx* c) { return !lds_limb_fits(c) || option(c, HS_OPT_AUX_PATH) == 2; }
// The same choice for the vector's encoding and encryption and for decryption: from N = 16384 on
// the split form wins (measured: its batched transforms spread a limb over two or more workgroups),
// while the matrix's encoding keeps the fused kernels, which run on the side stream.
static bool use_split_client(const hs_ctx* c) { return use_split(c) || (c->logn >= 14 && option(c, HS_OPT_AUX_PATH) == 0); }

// (dst, src) pairs of `words` u64 words each, in batched copy launches
static void copy_pairs(const std::vector<std::pair<u64*, const u64*>>& pairs, size_t words, hipStream_t st) {
  if (pairs.empty()) return;
  std::vector<const u64*> src;
  std::vector<u64*> dst;
  for (const auto& p : pairs) { dst.push_back(p.first); src.push_back(p.second); }
  std::vector<size_t> w(pairs.size(), words);
  launch_copy_batch(src.data(), dst.data(), w.data(), (int)pairs.size(), st);
}

// Exact ciphertext products a_i x b_i (NTT form [2][L][N] each) with relinearisation: n items,
// keys[i] = the relinearisation key of item i.  With lazy[i] set, item i is not relinearised: its
// scaled tensor goes to lazy[i] as [4][L][N] = (d0, d2, 0, d1) (out[i] is not written).
static void mul_ct_batch(hs_ctx* c, int n, const u64* const* a, const u64* const* b, u64* const* out, const u64* const* rkeys,
                         hipStream_t st, u64* const* lazy = nullptr, Alloc* al = nullptr) {
  if (n <= 0) return;
  HS_REQUIRE(c->has_tensor, HS_EPARAM, "parameters too large for the exact ciphertext product");
  const size_t N = c->N;
  const int L = c->L, T = c->n_mod;
  const size_t LN = (size_t)L * N;
  Alloc* A = al ? al : &c->pool;
  std::vector<DBuf> hold;
  DBuf X(A, (size_t)n * 4 * LN * sizeof(u64));
  // the operands' limbs reach coefficient form in X: the one-workgroup N = 2^15 transform reads
  // them where they are (row map), the others transform a gathered copy in place
  const bool rowmap = ntt15_one_wg(c, (i64)n * 4 * L);
  if (rowmap) {
    for (int i0 = 0; i0 < n; i0 += kNttRowItems) {
      const int m = std::min(kNttRowItems, n - i0);
      NttRows rm;
      rm.mode = 1; rm.per = 4 * L; rm.split = 2 * L;
      for (int i = 0; i < m; i++) { rm.opA[i] = a[i0 + i]; rm.opB[i] = b[i0 + i]; }
      launch_ntt15_rows(c, X.as<u64>() + (size_t)i0 * 4 * LN, (i64)m * 4 * L, L, 0, 1, rm, st);
    }
  } else {
    std::vector<const u64*> src(2 * n);
    std::vector<u64*> dst(2 * n);
    std::vector<size_t> words(2 * n, 2 * LN);
    for (int i = 0; i < n; i++) {
      src[2 * i] = a[i];
      src[2 * i + 1] = b[i];
      dst[2 * i] = X.as<u64>() + (size_t)i * 4 * LN;
      dst[2 * i + 1] = X.as<u64>() + (size_t)i * 4 * LN + 2 * LN;
    }
    launch_copy_batch(src.data(), dst.data(), words.data(), 2 * n, st);
    ntt_any(c, X.as<u64>(), (i64)n * 4 * L, L, 0, 1, st, hold, A);
  }
  TensorConst C{};
  C.qhat_inv = (const double2*)c->d_dec_inv; C.qhat = c->d_dec_hat; C.Q = c->d_dec_q; C.halfQ = c->d_t_halfq; C.WQ = c->tq_words;
  C.mhat_inv = (const double2*)c->d_t_mhat_inv; C.mhat = c->d_t_mhat; C.M = c->d_t_m; C.halfM = c->d_t_halfm; C.WM = c->tm_words;
  C.D = c->d_t_d; C.WD = c->td_words; C.mu = c->d_t_mu; C.WMU = c->tmu_words; C.WA = c->ta_words;
  C.r32 = (const double2*)c->d_t_r32; C.T = T; C.L = L; C.t = c->t; C.kw = c->t_kw;
  DBuf LIFT(A, (size_t)n * 4 * T * N * sizeof(u64));
  launch_crt_lift(c, C, X.as<u64>(), LIFT.as<u64>(), n * 4, st);
  ntt_any(c, LIFT.as<u64>(), (i64)n * 4 * T, T, 0, 0, st, hold, A);
  DBuf PROD(A, (size_t)n * 3 * T * N * sizeof(u64));
  launch_tensor(c, LIFT.as<u64>(), PROD.as<u64>(), n, T, st);
  ntt_any(c, PROD.as<u64>(), (i64)n * 3 * T, T, 0, 1, st, hold, A);
  DBuf D4(A, (size_t)n * 4 * LN * sizeof(u64));
  launch_scale_round(c, C, PROD.as<u64>(), D4.as<u64>(), n, st);
  std::vector<std::vector<RotItem>> lv(1);
  if (rowmap) {
    // unrelinearised products go straight to their lazy outputs (row map), the others stay in D4
    for (int i0 = 0; i0 < n; i0 += kNttRowItems) {
      const int m = std::min(kNttRowItems, n - i0);
      NttRows rm;
      rm.mode = 2; rm.per = 4 * L;
      for (int i = 0; i < m; i++) rm.out[i] = lazy ? lazy[i0 + i] : nullptr;
      launch_ntt15_rows(c, D4.as<u64>() + (size_t)i0 * 4 * LN, (i64)m * 4 * L, L, 0, 0, rm, st);
    }
  } else {
    ntt_any(c, D4.as<u64>(), (i64)n * 4 * L, L, 0, 0, st, hold, A);
    std::vector<const u64*> src;
    std::vector<u64*> dst;
    for (int i = 0; i < n; i++)
      if (lazy && lazy[i]) {
        src.push_back(D4.as<u64>() + (size_t)i * 4 * LN);
        dst.push_back(lazy[i]);
      }
    std::vector<size_t> words(src.size(), 4 * LN);
    launch_copy_batch(src.data(), dst.data(), words.data(), (int)src.size(), st);
  }
  for (int i = 0; i < n; i++) {
    if (lazy && lazy[i]) continue;
    RotItem it{};
    it.in = D4.as<u64>() + (size_t)i * 4 * LN;            // (d0, d2)
    it.addend = D4.as<u64>() + (size_t)i * 4 * LN + 2 * LN;  // (0, d1)
    it.out = out[i];
    it.key = rkeys[i];
    it.galois = 1;  // identity automorphism: a plain key switch of d2 under s^2 -> s
    lv[0].push_back(it);
  }
  run_rotation_levels(c, lv, st, A);
  g_counters[0] -= (int64_t)lv[0].size();  // relinearisations are not rotations
}

// Lazy relinearisation (hs_params.relin_mode = 1; matrices with encrypted values): a one-column
// chunk has no totalSum rotation, so its product stays unrelinearised, (d0, d2 | 0, d1) in the
// [4][L][N] layout above.  Per result ciphertext (group) two masked sums are formed over its
// chunks: LA = (sum m d0, sum m d2) over the one-column chunks (a zero ciphertext stands for the
// others) and Y2 = sum m (result) over the other chunks + (0, sum m d1) over the one-column ones;
// the group's result is LA's first component + KeySwitch(LA's second) + Y2, one key switch per
// group instead of one per chunk.  A group without one-column chunks takes Y2 as it is.
static bool lazy_chunk(const hs_ctx* c, const hs_matrix* m, int g) {
  return m->encrypted && c->prm.relin_mode == 1 && m->chunks[g].c == 1;
}

// Pack + encode G chunks (mode 0 matrix values, 1 vector, 2 mask) into mod-t coefficients.
static void pack_encode(hs_ctx* c, PackArgs pa, int G, hipStream_t st, std::vector<DBuf>& hold, bool split) {
  if (split) {
    launch_pack_slots(c, pa, G, st);
    ntt_any(c, pa.out, G, 1, c->n_mod, 1, st, hold);
  } else {
    launch_pack_encode(c, pa, G, st);
  }
}
// Mod-t coefficients -> NTT-form plaintexts over the data primes.
static void plain_ntt(hs_ctx* c, const u64* coef, u64* out, int G, hipStream_t st, std::vector<DBuf>& hold) {
  if (use_split(c)) {
    launch_lift_plain(c, coef, G, out, st);
    ntt_any(c, out, (i64)G * c->L, c->L, 0, 0, st, hold);
  } else {
    launch_plain_ntt(c, coef, out, G, st);
  }
}
// Public-key encryption of G encoded plaintexts (samples [G][3][N]: u, e0, e1).  From N = 16384 on
// the split form (elementwise kernels around one batched transform of all 3 L G limbs) beats the
// fused kernel, whose workgroups run three whole-limb transforms one after another.
static void encrypt_coefs(hs_ctx* c, const u64* coef, const int* samples, const u64* pk, u64* out, int G, hipStream_t st,
                          std::vector<DBuf>& hold) {
  if (use_split_client(c)) {
    hold.emplace_back(&c->pool, (size_t)G * 3 * c->L * c->N * sizeof(u64));
    u64* prep = hold.back().as<u64>();
    const i64 rows = (i64)G * 3 * c->L;
    if (lds_limb_fits(c) && option(c, HS_OPT_NTT_PATH) != 2 && option(c, HS_OPT_AUX_PATH) == 0 && rows > (c->logn == 14 ? kTwoPassMaxRows14 : kTwoPassMaxRows)) {
      launch_enc_ntt(c, coef, samples, G, prep, st);   // the one-workgroup transforms, prologue in their input
    } else {
      launch_enc_prep(c, coef, samples, G, prep, st);
      ntt_any(c, prep, rows, c->L, 0, 0, st, hold);
    }
    launch_enc_combine(c, prep, pk, out, G, st);
  } else {
    launch_encrypt(c, coef, samples, pk, out, G, st);
  }
}

static hs_ctvec* new_ctvec(hs_ctx* c, i64 n) {
  hs_ctvec* v = new hs_ctvec();
  v->ctx = c;
  v->n = n;
  v->d = pmalloc<u64>(c, std::max<i64>(n, 1) * ct_words(c));
  return v;
}

}  // namespace hs

using namespace hs;

extern "C" {

const char* hs_last_error(void) { return hs::last_error_cstr(); }

int hs_ctx_create(const hs_params* params, hs_ctx** out) {
  return guarded([&] {
    HS_REQUIRE(params && out, HS_EINVAL, "null argument");
    *out = nullptr;
    hs_ctx* c = new hs_ctx();
    c->prm = *params;
    try {
      HS_CHECK_HIP(hipGetDevice(&c->device));
      HS_REQUIRE(noalloc_scratch(&c->na_scratch, &c->na_bytes) == HS_OK, HS_EDEVICE, "address of the fixed scratch array");
      HS_CHECK_HIP(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
      build_ctx(c);
      HS_REQUIRE(c->dec_words <= 16, HS_EPARAM, "modulus too large for the decryption kernel (at most 16 words)");
      u64 cdt[20];
      compute_cdt(cdt);
      upload_cdt(cdt);
    } catch (...) {
      free_ctx(c);
      delete c;
      throw;
    }
    *out = c;
  });
}

void hs_ctx_destroy(hs_ctx* c) {
  if (!c) return;
  free_ctx(c);
  delete c;
}

int hs_ctx_moduli(const hs_ctx* c, uint64_t* out, int cap, int* n) {
  return guarded([&] {
    HS_REQUIRE(c && n, HS_EINVAL, "null argument");
    *n = c->n_mod;
    HS_REQUIRE(out && cap >= c->n_mod, HS_ECAPACITY, "output too small");
    for (int i = 0; i < c->n_mod; i++) out[i] = c->mod[i];
  });
}

int hs_ctx_tensor_widths(const hs_ctx* c, int64_t out[7]) {
  return guarded([&] {
    HS_REQUIRE(c && out, HS_EINVAL, "null argument");
    const int64_t v[7] = {c->n_mod, c->tq_words, c->tm_words, c->td_words, c->tmu_words, c->ta_words, c->t_kw};
    for (int i = 0; i < 7; i++) out[i] = c->has_tensor ? v[i] : 0;
  });
}

int hs_cdt_table(uint64_t out[20]) {
  return guarded([&] {
    HS_REQUIRE(out, HS_EINVAL, "null argument");
    compute_cdt(out);
  });
}

int hs_keygen(hs_ctx* c, uint64_t seed, void* stream, hs_keyset** out) {
  return guarded([&] {
    HS_REQUIRE(c && out, HS_EINVAL, "null argument");
    *out = nullptr;
    hipStream_t st = S(stream);
    hs_keyset* ks = new hs_keyset();
    ks->ctx = c;
    ks->seed = seed;
    try {
      const size_t N = c->N;
      const int LK = c->L + c->K;
      ks->ksk_words = 2ULL * c->dnum * LK * N;
      DBuf scoef(&c->pool, N * sizeof(int));
      launch_sample_small(c, scoef.as<int>(), 1, (i64)N, seed, P_SK, 0, 1, 0, st);
      ks->sk = dmalloc<u64>((size_t)c->n_mod * N);
      std::vector<DBuf> hold;
      if (use_split(c)) {
        launch_ints_to_limbs(c, scoef.as<int>(), (i64)N, 1, ks->sk, c->n_mod, 0, st);
        ntt_any(c, ks->sk, c->n_mod, c->n_mod, 0, 0, st, hold);
      } else {
        launch_sk_ntt(c, ks->sk, scoef.as<int>(), st);
      }
      // public key: (pk0, pk1) = (e - a s, a) over the data primes
      ks->pk = dmalloc<u64>(2ULL * c->L * N);
      DBuf e(&c->pool, N * sizeof(int));
      launch_sample_small(c, e.as<int>(), 1, (i64)N, seed, P_PK_E, 0, 1, 1, st);
      std::vector<KskArgs> args;
      for (int i = 0; i < c->L; i++) {
        const u64 q = c->mod[i];
        KskArgs a{};
        a.b = ks->pk + (size_t)i * N;
        a.a = ks->pk + ((size_t)c->L + i) * N;
        a.e_coef = e.as<int>();
        a.sk = ks->sk + (size_t)i * N;
        a.mod_index = i;
        a.seed = seed;
        a.purpose_a = P_PK_A;
        a.idx_a = (u64)i;
        a.sprime_mode = 0;
        a.pfac = double2{0.0, 0.0};
        a.r64 = make_const((u64)(((u128)1 << 64) % q), q);
        args.push_back(a);
      }
      DBuf dargs(&c->pool, args.size() * sizeof(KskArgs));
      h2d(dargs.as<KskArgs>(), args.data(), args.size(), st);
      if (use_split(c)) {
        DBuf en(&c->pool, (size_t)c->L * N * sizeof(u64));
        launch_ints_to_limbs(c, e.as<int>(), (i64)N, 1, en.as<u64>(), c->L, 0, st);
        ntt_any(c, en.as<u64>(), c->L, c->L, 0, 0, st, hold);
        launch_ksk_combine(c, dargs.as<KskArgs>(), en.as<u64>(), (int)args.size(), st);
        HS_CHECK_HIP(hipStreamSynchronize(st));
      } else {
        launch_ksk_limbs(c, dargs.as<KskArgs>(), (int)args.size(), st);
      }
      HS_CHECK_HIP(hipStreamSynchronize(st));
      for (int i = 0; i < n_pow2(c); i++)
        ks->gk.push_back(make_ksk(c, ks, key_index_id(c, i), 1, (u32)galois_step(c, key_index_step(c, i)), st));
      ks->rk = make_ksk(c, ks, RELIN_ID, 2, 0, st);
    } catch (...) {
      hs_keyset_destroy(ks);
      throw;
    }
    *out = ks;
  });
}

void hs_keyset_destroy(hs_keyset* ks) {
  if (!ks) return;
  if (ks->sk) (void)hipFree(ks->sk);
  if (ks->pk) (void)hipFree(ks->pk);
  for (u64* p : ks->gk) (void)hipFree(p);
  for (auto& kv : ks->step_keys) (void)hipFree(kv.second);
  if (ks->rk) (void)hipFree(ks->rk);
  delete ks;
}

int hs_keyset_export(const hs_keyset* ks, int which, int index, uint64_t* host_out, int64_t cap) {
  return guarded([&] {
    HS_REQUIRE(ks && host_out, HS_EINVAL, "null argument");
    const hs_ctx* c = ks->ctx;
    const u64* src = nullptr;
    size_t n = 0;
    if (which == 0) { src = ks->sk; n = (size_t)c->n_mod * c->N; }
    else if (which == 1) { src = ks->pk; n = 2ULL * c->L * c->N; }
    else if (which == 2) {
      HS_REQUIRE(index >= 0 && index < (int)ks->gk.size(), HS_EKEY, "no rotation key with that index");
      src = ks->gk[index]; n = ks->ksk_words;
    } else if (which == 3) { src = ks->rk; n = ks->ksk_words; }
    else if (which == 4) {
      auto it = ks->step_keys.find(index);
      HS_REQUIRE(it != ks->step_keys.end(), HS_EKEY, "no exact-step rotation key for that step");
      src = it->second; n = ks->ksk_words;
    } else throw Error{HS_EINVAL, "unknown key kind"};
    HS_REQUIRE((size_t)cap >= n, HS_ECAPACITY, "output too small");
    HS_CHECK_HIP(hipMemcpy(host_out, src, n * sizeof(u64), hipMemcpyDeviceToHost));
  });
}

int hs_keyset_add_right_rotation_keys(hs_ctx* c, hs_keyset* ks, void* stream) {
  return guarded([&] {
    HS_REQUIRE(c && ks, HS_EINVAL, "null argument");
    HS_REQUIRE(ks->ctx == c, HS_EKEY, "key-set from another context");
    hipStream_t st = S(stream);
    for (int i = (int)ks->gk.size(); i < 2 * n_pow2(c); i++)
      ks->gk.push_back(make_ksk(c, ks, key_index_id(c, i), 1, (u32)galois_step(c, key_index_step(c, i)), st));
  });
}

int hs_keyset_add_rotation_keys(hs_ctx* c, hs_keyset* ks, const int64_t* steps, int64_t n, void* stream) {
  return guarded([&] {
    HS_REQUIRE(c && ks && (n == 0 || steps), HS_EINVAL, "null argument");
    HS_REQUIRE(n >= 0, HS_EINVAL, "negative count");
    HS_REQUIRE(ks->ctx == c, HS_EKEY, "key-set from another context");
    hipStream_t st = S(stream);
    const i64 half = (i64)c->N / 2;
    for (i64 i = 0; i < n; i++) {
      const i64 k = ((steps[i] % half) + half) % half;
      if (k == 0 || is_pow2(k) || ks->step_keys.count(k)) continue;
      u64* key = make_ksk(c, ks, step_key_id(k), 1, (u32)galois_step(c, k), st);
      ks->step_keys[k] = key;
    }
  });
}

int hs_matrix_rotation_steps(const hs_matrix* m, int64_t* out, int64_t cap, int64_t* len) {
  return guarded([&] {
    HS_REQUIRE(m && len && (cap == 0 || out), HS_EINVAL, "null argument");
    std::vector<i64> all;
    for (const hs_chunk& ch : m->chunks)
      for (i64 k : total_sum_steps(m->ctx, ch.h, ch.c)) all.push_back(k);
    std::sort(all.begin(), all.end());
    all.erase(std::unique(all.begin(), all.end()), all.end());
    *len = (int64_t)all.size();
    HS_REQUIRE(cap >= (int64_t)all.size(), HS_ECAPACITY, "output too small");
    for (size_t i = 0; i < all.size(); i++) out[i] = all[i];
  });
}

int hs_cssc_pack(hs_ctx* c, int64_t rows, int64_t cols, const int64_t* row_ptr, const int32_t* col_idx,
                 const int64_t* vals, int encrypt_values, const hs_keyset* ks, uint64_t seed, void* stream,
                 hs_matrix** out) {
  return guarded([&] {
    HS_REQUIRE(c && out, HS_EINVAL, "null argument");
    *out = nullptr;
    HS_REQUIRE(rows >= 0 && cols >= 0 && rows < (1LL << 31) && cols < (1LL << 31), HS_EINVAL, "bad matrix shape");
    HS_REQUIRE(rows == 0 || row_ptr, HS_EINVAL, "null row_ptr");
    HS_REQUIRE(!encrypt_values || (ks && ks->ctx == c), HS_EKEY, "encrypted values need the key-set of this context");
    HS_REQUIRE(!encrypt_values || c->has_tensor, HS_EPARAM,
               "encrypted values need the exact ciphertext product, which these parameters do not support");
    hipStream_t st = S(stream);
    const size_t N = c->N;
    const i64 s = (i64)N / 2;
    // --- CSSC structure on the device (App. B): row counts, the stable descending order, RM and
    // CP.  When every row holds at most 255 nonzeros (one 8-bit sort digit) the order and CP come
    // from one histogram / scan / scatter and the host reads the partition statistics and CP back
    // in one copy; otherwise the statistics come back first, then a multi-pass sort builds the
    // order and CP.  The host cuts the chunks from CP (a few words per partition).
    const i64 nP0 = rows ? (rows + s - 1) / s : 0;
    const int BR = cssc_sort_block(s);
    const i64 nblk = rows ? (rows + BR - 1) / BR : 0;
    const size_t R1 = (size_t)std::max<i64>(rows, 1);
    auto seg = [](size_t bytes) { return (bytes + 255) & ~(size_t)255; };
    hs_matrix* M = new hs_matrix();
    M->ctx = c; M->R = rows; M->C = cols; M->encrypted = encrypt_values ? 1 : 0;
    std::vector<DBuf> keep;  // scratch released only after the final synchronisation
    keep.reserve(8);         // references into it stay valid
    try {
      const int srows = c->prm.slot_rows == 2 ? 2 : 1;
      PinnedStage& down = t_stage_down;
      // one-pass form; scratch: block histograms | block flags | digits | rank
      const size_t o1_bf = seg((size_t)std::max<i64>(nblk, 1) * 256 * 4), o1_dg = o1_bf + seg((size_t)std::max<i64>(nblk, 1) * 4),
                   o1_rk = o1_dg + seg(R1 * 4), s1_bytes = o1_rk + seg(R1 * 4);
      const size_t hdr_bytes = seg((1 + 3 * (size_t)nP0) * 8), cp1_words = 256 * (size_t)nP0;
      keep.emplace_back(&c->pool, s1_bytes);
      char* w1 = keep.back().as<char>();
      int* drank = (int*)(w1 + o1_rk);
      M->d_struct = pmalloc<char>(c, hdr_bytes + cp1_words * 8 + R1 * 4 + 4);
      i64* dhdr = (i64*)M->d_struct;
      M->d_cp = (i64*)(M->d_struct + hdr_bytes);
      M->d_rm = (i32*)(M->d_struct + hdr_bytes + cp1_words * 8);
      i64* hh = (i64*)down.get(hdr_bytes + cp1_words * 8 + 512);
      std::fill(hh, hh + hdr_bytes / 8, 0);
      if (rows) {
        launch_cssc_one_pass(row_ptr, rows, s, (int*)(w1 + o1_dg), (int*)w1, (int*)(w1 + o1_bf), dhdr, M->d_cp, M->d_rm, drank, st);
        d2h(hh, dhdr, hdr_bytes / 8 + cp1_words, st);
        HS_CHECK_HIP(hipStreamSynchronize(st));
      }
      i64 flags = 0;
      for (i64 p = 0; p < nP0; p++) flags |= hh[2 + 3 * p];
      HS_REQUIRE(!(flags & 1), HS_EINVAL, "row_ptr must start at 0 and be nondecreasing, with at most 2^30 entries per row");
      const bool one_pass = !(flags & 2);
      const i64 nnz = rows ? hh[0] : 0;
      M->nnz = nnz;
      HS_REQUIRE(nnz == 0 || (col_idx && vals), HS_EINVAL, "null col_idx/vals");
      for (i64 p = 0; p < nP0; p++) {
        hs_part P{};
        P.row0 = p * s;
        P.rows = std::min(s, rows - P.row0);
        P.Lw = (int)hh[1 + 3 * p];
        P.nnz_off = hh[3 + 3 * p];
        P.cp_off = p * 256;
        M->parts.push_back(P);
      }
      const int nP = (int)M->parts.size();
      if (one_pass) {
        M->h_cp.assign(hh + hdr_bytes / 8, hh + hdr_bytes / 8 + cp1_words);
      } else {
        // multi-pass form: the statistics (longest row per partition), then the order and CP
        const size_t nstat = 2 + 2 * (size_t)nP0;
        const size_t o_cnt = seg(nstat * 8), o_ka = o_cnt + seg(R1 * 4), o_kb = o_ka + seg(R1 * 4), o_ia = o_kb + seg(R1 * 4),
                     o_ib = o_ia + seg(R1 * 4), o_bh = o_ib + seg(R1 * 4), o_pm = o_bh + seg((size_t)nblk * 256 * 4),
                     scratch_bytes = o_pm + seg(2 * (size_t)nP0 * 8);
        keep.emplace_back(&c->pool, scratch_bytes);
        char* ws = keep.back().as<char>();
        unsigned long long* dstat = (unsigned long long*)ws;
        int* dcnt = (int*)(ws + o_cnt);
        i64* dpm = (i64*)(ws + o_pm);
        u64* hstat = (u64*)hh;
        launch_fill_u64((u64*)dstat, nstat, 0, st);
        launch_csr_rows(row_ptr, rows, s, dcnt, dstat, st);
        d2h(hstat, (const u64*)dstat, nstat, st);
        HS_CHECK_HIP(hipStreamSynchronize(st));
        HS_REQUIRE(hstat[0] == 0 && (i64)hstat[1] == nnz, HS_EINVAL, "malformed row_ptr");
        i64 maxLw = 0;
        for (int p = 0; p < nP; p++) {
          M->parts[p].Lw = (int)hstat[2 + 2 * p];
          maxLw = std::max<i64>(maxLw, M->parts[p].Lw);
        }
        // CP array lengths: with two slot rows both partitions of a pair are padded to the joint width
        std::vector<i64> pm(2 * (size_t)std::max(nP, 1), 0);  // cp_off | cp_len
        i64 cp_total = 0;
        for (int p = 0; p < nP; p++) {
          const int mate = srows == 2 ? (p % 2 == 0 ? p + 1 : p - 1) : -1;
          i64 len = (i64)M->parts[p].Lw + 1;
          if (mate >= 0 && mate < nP) len = std::max<i64>(len, (i64)M->parts[mate].Lw + 1);
          M->parts[p].cp_off = cp_total;
          pm[p] = cp_total;
          pm[nP + p] = len;
          cp_total += len;
        }
        pfree(c, M->d_struct);
        M->d_struct = nullptr;
        M->d_struct = pmalloc<char>(c, seg((size_t)std::max<i64>(cp_total, 1) * 8) + R1 * 4 + 4);
        M->d_cp = (i64*)M->d_struct;
        M->d_rm = (i32*)(M->d_struct + seg((size_t)std::max<i64>(cp_total, 1) * 8));
        M->h_cp.assign(cp_total, 0);
        h2d(dpm, pm.data(), pm.size(), st);
        int bits = 0;
        while (bits < 63 && (maxLw >> bits) != 0) bits++;
        const int passes = std::max(1, (bits + 7) / 8);
        const u32* sorted = launch_cssc_order(dcnt, dstat, rows, s, passes, (u32*)(ws + o_ka), (u32*)(ws + o_kb), (int*)(ws + o_ia),
                                              (int*)(ws + o_ib), (int*)(ws + o_bh), M->d_rm, drank, st);
        launch_cssc_cp(sorted, dstat, rows, s, dpm, dpm + nP, M->d_cp, st);
        d2h(M->h_cp.data(), M->d_cp, (size_t)cp_total, st);
        HS_CHECK_HIP(hipStreamSynchronize(st));
      }
      // the column check runs on the device (row_ptr is valid now); its flag is read back with the
      // final synchronisation (no kernel below uses a column index as an address)
      int* hbad_p = (int*)((char*)hh + hdr_bytes + cp1_words * 8 + 256);
      *hbad_p = 0;
      if (nnz) {
        keep.emplace_back(&c->pool, 256);
        int* dbad = keep.back().as<int>();
        launch_fill_u64((u64*)dbad, 1, 0, st);
        launch_csr_check(row_ptr, col_idx, rows, cols, dbad, st);
        d2h(hbad_p, dbad, 1, st);
      }
      std::vector<std::vector<i64>> cps(nP);
      for (int p = 0; p < nP; p++) {
        hs_part& P = M->parts[p];
        cps[p].assign(M->h_cp.begin() + P.cp_off, M->h_cp.begin() + P.cp_off + P.Lw + 1);
        P.nz_rows = P.Lw > 0 ? cps[p][1] : 0;
      }
      // result ciphertexts: one per partition, or (two slot rows) per pair of partitions whose
      // chunks follow the joint column profile max(NNZ_A[j], NNZ_B[j])
      for (int p = 0; p < nP; p += srows) {
        hs_group Gr{p, (srows == 2 && p + 1 < nP) ? p + 1 : -1, (int)M->chunks.size(), 0};
        std::vector<i64> jcp;
        if (Gr.pb >= 0) {
          const std::vector<i64>& a = cps[p];
          const std::vector<i64>& bb = cps[Gr.pb];
          const size_t W = std::max(a.size(), bb.size());
          jcp.assign(W, 0);
          for (size_t j = 0; j + 1 < W; j++) {
            const i64 na = j + 1 < a.size() ? a[j + 1] - a[j] : 0, nb = j + 1 < bb.size() ? bb[j + 1] - bb[j] : 0;
            jcp[j + 1] = jcp[j] + std::max(na, nb);
          }
        }
        std::vector<hs_chunk> ch = make_chunks(Gr.pb >= 0 ? jcp : cps[p], s, c->prm.agg_mode == 1, (int)M->groups.size());
        Gr.nchunks = (int)ch.size();
        M->chunks.insert(M->chunks.end(), ch.begin(), ch.end());
        M->groups.push_back(Gr);
      }
      const int G = (int)M->chunks.size();
      // chunk table and partition info (row0, rows, nz rows, rm offset, group, slot offset): one
      // pinned upload
      std::vector<i64> cd(8ULL * std::max(G, 1), 0);
      for (int g = 0; g < G; g++) {
        const hs_chunk& k = M->chunks[g];
        const hs_group& Gr = M->groups[k.part];
        const hs_part& PA = M->parts[Gr.pa];
        i64* d = &cd[8ULL * g];
        d[0] = k.start; d[1] = k.c; d[2] = k.h; d[3] = PA.cp_off; d[4] = PA.nnz_off; d[5] = k.part;
        d[6] = Gr.pb >= 0 ? M->parts[Gr.pb].cp_off : -1;
        d[7] = Gr.pb >= 0 ? M->parts[Gr.pb].nnz_off : 0;
      }
      std::vector<i64> pinfo(6ULL * std::max(nP, 1), 0);
      for (int p = 0; p < nP; p++) {
        const hs_part& P = M->parts[p];
        i64* q = &pinfo[6ULL * p];
        q[0] = P.row0; q[1] = P.rows; q[2] = P.nz_rows; q[3] = P.row0; q[4] = p / srows; q[5] = (p % srows) * s;
      }
      std::vector<i64> poff(2 * (size_t)std::max(nP, 1), 0);  // per partition: CP offset | nonzero offset
      for (int p = 0; p < nP; p++) { poff[p] = M->parts[p].cp_off; poff[nP + p] = M->parts[p].nnz_off; }
      const size_t o_pi = seg(cd.size() * 8), o_po = o_pi + seg(pinfo.size() * 8), meta_bytes = o_po + seg(poff.size() * 8);
      char* up = (char*)t_stage_up.get(meta_bytes);
      std::memcpy(up, cd.data(), cd.size() * 8);
      std::memcpy(up + o_pi, pinfo.data(), pinfo.size() * 8);
      std::memcpy(up + o_po, poff.data(), poff.size() * 8);
      M->d_meta = pmalloc<char>(c, meta_bytes);
      HS_CHECK_HIP(hipMemcpyAsync(M->d_meta, up, meta_bytes, hipMemcpyHostToDevice, st));
      M->d_chunk = (i64*)M->d_meta;
      M->d_pinfo = (i64*)(M->d_meta + o_pi);
      M->d_va = pmalloc<i64>(c, nnz);
      M->d_ci = pmalloc<i32>(c, nnz);
      if (rows && nnz)
        launch_cssc_scatter(row_ptr, col_idx, vals, drank, M->d_cp, (const i64*)(M->d_meta + o_po), (const i64*)(M->d_meta + o_po) + nP,
                            rows, s, M->d_va, M->d_ci, st);
      const int hbad_dummy = 0;
      const int& hbad = nnz ? *hbad_p : hbad_dummy;
      // --- pack + encode (+ encrypt) every chunk; masks
      std::vector<DBuf> hold;
      const bool masks = c->prm.agg_mode == 0;
      if (G && !encrypt_values && !use_split(c)) {
        // plaintexts and masks in one pass each, on the side stream after the structure is final:
        // the encoding overlaps the caller's next work (the vector's encryption); consumers wait
        // for M->ready.  Every buffer it touches belongs to M until hs_matrix_destroy.
        const int np = masks ? 2 * G : G;
        M->d_coef = pmalloc<u64>(c, (size_t)np * N);
        M->d_pt = pmalloc<u64>(c, (size_t)np * c->L * N);
        if (masks) { M->d_mask = M->d_pt + (size_t)G * c->L * N; M->mask_in_pt = true; }
        // the side stream starts once the values are scattered (the event's first record); a
        // malformed CSR is reported at the final synchronisation below, and whatever the encoding
        // then reads stays inside M's buffers (its indices come from the host structure)
        HS_CHECK_HIP(hipEventCreateWithFlags(&M->ready, hipEventDisableTiming));
        HS_CHECK_HIP(hipEventRecord(M->ready, st));
        HS_CHECK_HIP(hipStreamWaitEvent(c->side, M->ready, 0));
        PackArgs pa{};
        pa.va = M->d_va; pa.ci = M->d_ci; pa.v = nullptr; pa.cp = M->d_cp; pa.chunk = M->d_chunk;
        pa.out = M->d_coef; pa.mode = masks ? 3 : 0; pa.nG = G;
        launch_pack_encode(c, pa, np, c->side);
        launch_plain_ntt(c, M->d_coef, M->d_pt, np, c->side);
        HS_CHECK_HIP(hipEventRecord(M->ready, c->side));
      } else if (G) {
        keep.emplace_back(&c->pool, (size_t)G * N * sizeof(u64));
        DBuf& coef = keep.back();
        PackArgs pa{};
        pa.va = M->d_va; pa.ci = M->d_ci; pa.v = nullptr; pa.cp = M->d_cp; pa.chunk = M->d_chunk;
        pa.out = coef.as<u64>(); pa.mode = 0; pa.nG = G;
        pack_encode(c, pa, G, st, hold, use_split(c));
        if (encrypt_values) {
          M->d_pt = pmalloc<u64>(c, (size_t)G * ct_words(c));
          keep.emplace_back(&c->pool, (size_t)G * 3 * N * sizeof(int));
          DBuf& smp = keep.back();
          launch_sample_enc(c, smp.as<int>(), G, seed, P_ENC_U, P_ENC_E0, P_ENC_E1, st);
          encrypt_coefs(c, coef.as<u64>(), smp.as<int>(), ks->pk, M->d_pt, G, st, hold);
        } else {
          M->d_pt = pmalloc<u64>(c, (size_t)G * c->L * N);
          plain_ntt(c, coef.as<u64>(), M->d_pt, G, st, hold);
        }
        if (masks) {
          pa.mode = 2;
          pack_encode(c, pa, G, st, hold, use_split(c));
          M->d_mask = pmalloc<u64>(c, (size_t)G * c->L * N);
          plain_ntt(c, coef.as<u64>(), M->d_mask, G, st, hold);
        }
      }
      HS_CHECK_HIP(hipStreamSynchronize(st));
      HS_REQUIRE(!hbad, HS_EINVAL, "column indices out of range or not strictly ascending within a row");
    } catch (...) {
      (void)hipStreamSynchronize(st);  // nothing in flight may still use the pooled memory
      hs_matrix_destroy(M);
      throw;
    }
    *out = M;
  });
}

void hs_matrix_destroy(hs_matrix* m) {
  if (!m) return;
  // the memory returns to the context's pool, from which work on any stream may take it next:
  // wait for the matrix's own encoding and for the library's asynchronous calls in flight
  if (m->ready) (void)hipEventSynchronize(m->ready);
  drain_async(m->ctx);
  void* ptrs[] = {m->d_struct, m->d_meta, m->d_va, m->d_ci, m->d_pt, m->mask_in_pt ? nullptr : m->d_mask, m->d_coef};
  for (void* p : ptrs) pfree(m->ctx, p);
  if (m->ready) (void)hipEventDestroy(m->ready);
  delete m;
}

int hs_matrix_groups(const hs_matrix* m, int64_t* n_groups) {
  return guarded([&] {
    HS_REQUIRE(m && n_groups, HS_EINVAL, "null argument");
    *n_groups = (int64_t)m->groups.size();
  });
}

int hs_matrix_info(const hs_matrix* m, int64_t* n_parts, int64_t* n_chunks) {
  return guarded([&] {
    HS_REQUIRE(m, HS_EINVAL, "null argument");
    if (n_parts) *n_parts = (int64_t)m->parts.size();
    if (n_chunks) *n_chunks = (int64_t)m->chunks.size();
  });
}

int hs_matrix_chunk(const hs_matrix* m, int64_t k, int64_t out4[4]) {
  return guarded([&] {
    HS_REQUIRE(m && out4, HS_EINVAL, "null argument");
    HS_REQUIRE(k >= 0 && k < (int64_t)m->chunks.size(), HS_EINVAL, "chunk index out of range");
    const hs_chunk& c = m->chunks[k];
    out4[0] = c.part; out4[1] = c.start; out4[2] = c.c; out4[3] = c.h;
  });
}

int hs_matrix_cssc(const hs_matrix* m, int64_t part, int32_t* host_rm, int64_t rm_cap, int64_t* host_cp, int64_t cp_cap,
                   int64_t lens[2]) {
  return guarded([&] {
    HS_REQUIRE(m && lens, HS_EINVAL, "null argument");
    HS_REQUIRE(part >= 0 && part < (i64)m->parts.size(), HS_EINVAL, "partition out of range");
    const hs_part& P = m->parts[part];
    lens[0] = P.rows;
    lens[1] = (i64)P.Lw + 1;
    HS_REQUIRE(host_rm && host_cp && rm_cap >= lens[0] && cp_cap >= lens[1], HS_ECAPACITY, "output too small");
    HS_CHECK_HIP(hipMemcpy(host_rm, m->d_rm + P.row0, P.rows * sizeof(i32), hipMemcpyDeviceToHost));
    for (i64 j = 0; j < lens[1]; j++) host_cp[j] = m->h_cp[P.cp_off + j];
  });
}

int hs_matrix_column_index(const hs_matrix* m, int32_t* host_ci, int64_t cap, int64_t* len) {
  return guarded([&] {
    HS_REQUIRE(m && len, HS_EINVAL, "null argument");
    *len = m->nnz;
    HS_REQUIRE(host_ci && cap >= m->nnz, HS_ECAPACITY, "output too small");
    if (m->nnz) HS_CHECK_HIP(hipMemcpy(host_ci, m->d_ci, m->nnz * sizeof(i32), hipMemcpyDeviceToHost));
  });
}

int hs_matrix_export(const hs_matrix* m, int which, int64_t k, uint64_t* host_out, int64_t cap) {
  return guarded([&] {
    HS_REQUIRE(m && host_out, HS_EINVAL, "null argument");
    HS_REQUIRE(k >= 0 && k < (int64_t)m->chunks.size(), HS_EINVAL, "chunk index out of range");
    const hs_ctx* c = m->ctx;
    const u64* src;
    size_t n;
    if (which == 0) {
      n = m->encrypted ? ct_words(c) : (size_t)c->L * c->N;
      src = m->d_pt + k * n;
    } else {
      HS_REQUIRE(m->d_mask, HS_EINVAL, "no masks (uniform aggregation)");
      n = (size_t)c->L * c->N;
      src = m->d_mask + k * n;
    }
    HS_REQUIRE((size_t)cap >= n, HS_ECAPACITY, "output too small");
    if (m->ready) HS_CHECK_HIP(hipEventSynchronize(m->ready));
    HS_CHECK_HIP(hipMemcpy(host_out, src, n * sizeof(u64), hipMemcpyDeviceToHost));
  });
}

int hs_encrypt(hs_ctx* c, const hs_keyset* ks, const hs_matrix* m, const int64_t* v, int64_t len, uint64_t seed,
               void* stream, hs_ctvec** out) {
  return guarded([&] {
    HS_REQUIRE(c && ks && m && out, HS_EINVAL, "null argument");
    *out = nullptr;
    HS_REQUIRE(ks->ctx == c && m->ctx == c, HS_EKEY, "handles from another context");
    HS_REQUIRE(len == m->C, HS_EINVAL, "vector length must equal the number of matrix columns");
    HS_REQUIRE(len == 0 || v, HS_EINVAL, "null vector");
    hipStream_t st = S(stream);
    const int G = (int)m->chunks.size();
    const size_t N = c->N;
    hs_ctvec* x = new_ctvec(c, G);
    try {
      if (G) {
        std::vector<DBuf> hold;
        DBuf coef(&c->pool, (size_t)G * N * sizeof(u64));
        PackArgs pa{};
        pa.va = m->d_va; pa.ci = m->d_ci; pa.v = v; pa.cp = m->d_cp; pa.chunk = m->d_chunk;
        pa.out = coef.as<u64>(); pa.mode = 1;
        pack_encode(c, pa, G, st, hold, use_split_client(c));
        DBuf smp(&c->pool, (size_t)G * 3 * N * sizeof(int));
        launch_sample_enc(c, smp.as<int>(), G, seed, P_ENC_U, P_ENC_E0, P_ENC_E1, st);
        encrypt_coefs(c, coef.as<u64>(), smp.as<int>(), ks->pk, x->d, G, st, hold);
        HS_CHECK_HIP(hipStreamSynchronize(st));
      }
    } catch (...) {
      (void)hipStreamSynchronize(st);  // nothing in flight may still use the pooled memory
      hs_ctvec_destroy(x);
      throw;
    }
    *out = x;
  });
}

}  // extern "C"

namespace hs {
// Encrypted SpMV of n independent requests (matrix, encrypted vector, key-set): the slot-wise
// products, then every request's chunk programs (totalSum rotations) merged level by level into
// batched rotations, then the masks and per-partition sums.  Results: one vector per request.
// prepare() does all host work, allocation and uploads; enqueue() only launches kernels (no host
// waits, copies or allocations), so it can be recorded into a graph and replayed.
struct BatchWork {
  struct Prod { const u64* x; const u64* pt; u64* out; int G; };
  struct Mask { const u64* const* wp; const u64* mask; const int* pc0; const int* pnc; u64* y; int nP; };
  std::vector<Prod> prods;
  std::vector<const u64*> pa, pb, rk;   // exact ct x ct products (encrypted matrices)
  std::vector<u64*> po, lz;             // lz: destination of an unrelinearised product, or null
  LevelPlan levels;
  LevelPlan relin;                      // lazy relinearisation: one key switch per group
  std::vector<std::pair<u64*, const u64*>> copies;  // lazy mode, groups without one-column chunks
  std::vector<Mask> masks;
  std::vector<DBuf> keep;
  int64_t counters[5] = {0, 0, 0, 0, 0};
  Alloc* al = nullptr;                  // every device buffer of the call (set by prepare)

  // `arena`: take every buffer from this region instead of the context's pool
  void prepare(hs_ctx* c, int n, const hs_keyset* const* ks, const hs_matrix* const* m, const hs_ctvec* const* x, hipStream_t st,
               hs_ctvec** y, Alloc* arena = nullptr) {
    al = arena ? arena : &c->pool;
    const size_t CW = ct_words(c);
    struct Req {
      int G, nP;
      std::vector<std::vector<MicroOp>> progs;
      std::vector<int> wt_base;
      int nwt = 0;
      u64* vbuf = nullptr;
      u64* wtbuf = nullptr;
      std::vector<int> lidx;   // lazy relinearisation: slot of a one-column chunk's product, or -1
      int nlazy = 0;
      u64* d4 = nullptr;       // [nlazy][4][L][N]
    };
    std::vector<Req> rq(n);
    int nlog = 0;
    keep.reserve(2 * (size_t)n + 3 * (size_t)n + 1);
    for (int r = 0; r < n; r++)  // plaintexts still being encoded on the side stream
      if (m[r]->ready) HS_CHECK_HIP(hipStreamWaitEvent(st, m[r]->ready, 0));
    for (int r = 0; r < n; r++) {
      Req& q = rq[r];
      q.G = (int)m[r]->chunks.size();
      q.nP = (int)m[r]->groups.size();
      q.progs.resize(q.G);
      q.wt_base.assign(q.G, -1);
      for (int g = 0; g < q.G; g++) {
        q.progs[g] = total_sum_program(c, ks[r], m[r]->chunks[g].h, m[r]->chunks[g].c, &nlog);
        if (q.progs[g].size() > 1) { q.wt_base[g] = q.nwt; q.nwt += 4; }
      }
      keep.emplace_back(al, (size_t)std::max(q.G, 1) * CW * sizeof(u64));
      q.vbuf = keep.back().as<u64>();
      keep.emplace_back(al, (size_t)std::max(q.nwt, 1) * CW * sizeof(u64));
      q.wtbuf = keep.back().as<u64>();
      q.lidx.assign(q.G, -1);
      for (int g = 0; g < q.G; g++)
        if (lazy_chunk(c, m[r], g)) q.lidx[g] = q.nlazy++;
      if (q.nlazy) {
        keep.emplace_back(al, (size_t)q.nlazy * 2 * CW * sizeof(u64));
        q.d4 = keep.back().as<u64>();
      }
    }
    auto buf = [&](int r, int g, int id) -> u64* {
      Req& q = rq[r];
      return id == 0 ? q.vbuf + (size_t)g * CW : q.wtbuf + (size_t)(q.wt_base[g] + id - 1) * CW;
    };
    // 1. slot-wise products: HE-CMult, or HE-Mult + relinearisation for encrypted matrix values
    for (int r = 0; r < n; r++) {
      if (!rq[r].G) continue;
      if (m[r]->encrypted) {
        for (int g = 0; g < rq[r].G; g++) {
          pa.push_back(m[r]->d_pt + (size_t)g * CW);
          pb.push_back(x[r]->d + (size_t)g * CW);
          po.push_back(rq[r].vbuf + (size_t)g * CW);
          rk.push_back(ks[r]->rk);
          lz.push_back(rq[r].lidx[g] >= 0 ? rq[r].d4 + (size_t)rq[r].lidx[g] * 2 * CW : nullptr);
        }
      } else {
        prods.push_back(Prod{x[r]->d, m[r]->d_pt, rq[r].vbuf, rq[r].G});
        counters[2]++;
      }
      counters[3] += rq[r].G;
    }
    // 2. totalSum of all chunks of all requests, level by level
    size_t nlev = 0;
    for (auto& q : rq)
      for (auto& p : q.progs) nlev = std::max(nlev, p.size() - 1);
    std::vector<std::vector<RotItem>> lv_items(nlev);
    for (size_t lv = 0; lv < nlev; lv++)
      for (int r = 0; r < n; r++)
        for (int g = 0; g < rq[r].G; g++) {
          const auto& prog = rq[r].progs[g];
          if (lv + 1 >= prog.size()) continue;
          const MicroOp& op = prog[lv];
          RotItem it{};
          it.in = buf(r, g, op.in);
          it.out = buf(r, g, op.out);
          it.addend = op.addend >= 0 ? buf(r, g, op.addend) : nullptr;
          it.key = rotation_key(ks[r], op.step);
          it.galois = (u32)galois_step(c, op.step);
          lv_items[lv].push_back(it);
        }
    prepare_levels(c, lv_items, st, levels, *al);
    counters[0] += levels.key_switches;
    counters[2] += levels.launches;
    counters[1] = nlog;
    // 3. masks and the per-partition sums; the argument arrays of every request in one upload:
    //    per request [chunk result pointers (G, at least 1)][first chunk per partition][chunks
    //    per partition], 8-byte words
    //    (lazy relinearisation: the chunk pointers give Y2's operands, and a second pointer
    //    array after the partition words gives LA's)
    std::vector<u64> words;
    std::vector<size_t> at(n, 0), at2(n, 0);
    bool any_lazy = false;
    for (auto& q : rq) any_lazy |= q.nlazy > 0;
    u64* zero = nullptr;
    if (any_lazy) {
      keep.emplace_back(al, CW * sizeof(u64));
      zero = keep.back().as<u64>();
      launch_fill_u64(zero, CW, 0, st);
    }
    for (int r = 0; r < n; r++) {
      Req& q = rq[r];
      at[r] = words.size();
      if (!q.nP) continue;
      for (int g = 0; g < std::max(q.G, 1); g++) {
        const u64* src = g >= q.G ? nullptr
                         : q.lidx[g] >= 0 ? q.d4 + (size_t)q.lidx[g] * 2 * CW + CW   // (0, d1)
                                          : buf(r, g, q.progs[g].back().in);
        words.push_back((u64)(uintptr_t)src);
      }
      std::vector<int> pcn(2 * (size_t)q.nP);
      for (int p = 0; p < q.nP; p++) { pcn[p] = m[r]->groups[p].chunk0; pcn[q.nP + p] = m[r]->groups[p].nchunks; }
      const size_t w0 = words.size();
      words.resize(w0 + (pcn.size() * sizeof(int) + 7) / 8, 0);
      std::memcpy(words.data() + w0, pcn.data(), pcn.size() * sizeof(int));
      at2[r] = words.size();
      if (q.nlazy)
        for (int g = 0; g < q.G; g++)
          words.push_back((u64)(uintptr_t)(q.lidx[g] >= 0 ? q.d4 + (size_t)q.lidx[g] * 2 * CW : zero));   // (d0, d2)
    }
    std::vector<RotItem> relin_items;
    if (!words.empty()) {
      keep.emplace_back(al, words.size() * sizeof(u64));
      u64* dw = keep.back().as<u64>();
      h2d(dw, words.data(), words.size(), st);
      for (int r = 0; r < n; r++) {
        Req& q = rq[r];
        if (!q.nP) continue;
        const u64* const* dwp = (const u64* const*)(dw + at[r]);
        const int* dpc0 = (const int*)(dw + at[r] + std::max(q.G, 1));
        const u64* mask = c->prm.agg_mode == 0 ? m[r]->d_mask : nullptr;
        counters[4] += c->prm.agg_mode == 0 ? q.G : 0;
        if (!q.nlazy) {
          masks.push_back(Mask{dwp, mask, dpc0, dpc0 + q.nP, y[r]->d, q.nP});
          counters[2]++;
          continue;
        }
        keep.emplace_back(al, (size_t)q.nP * 2 * CW * sizeof(u64));
        u64* LA = keep.back().as<u64>();
        u64* Y2 = LA + (size_t)q.nP * CW;
        masks.push_back(Mask{dwp, mask, dpc0, dpc0 + q.nP, Y2, q.nP});
        masks.push_back(Mask{(const u64* const*)(dw + at2[r]), mask, dpc0, dpc0 + q.nP, LA, q.nP});
        counters[2] += 2;
        for (int p = 0; p < q.nP; p++) {
          const hs_group& Gr = m[r]->groups[p];
          bool has = false;
          for (int g = Gr.chunk0; g < Gr.chunk0 + Gr.nchunks; g++) has |= q.lidx[g] >= 0;
          if (!has) { copies.emplace_back(y[r]->d + (size_t)p * CW, Y2 + (size_t)p * CW); continue; }
          RotItem it{};
          it.in = LA + (size_t)p * CW;
          it.addend = Y2 + (size_t)p * CW;
          it.out = y[r]->d + (size_t)p * CW;
          it.key = ks[r]->rk;
          it.galois = 1;
          relin_items.push_back(it);
        }
      }
    }
    if (!relin_items.empty()) {
      prepare_levels(c, {relin_items}, st, relin, *al);
      counters[2] += relin.launches;
    }
  }

  bool capturable() const { return pa.empty(); }

  void enqueue(hs_ctx* c, hipStream_t st) const {
    for (const Prod& p : prods) launch_mul_plain(c, p.x, p.pt, p.out, p.G, c->L, st);
    if (!pa.empty()) mul_ct_batch(c, (int)pa.size(), pa.data(), pb.data(), po.data(), rk.data(), st, lz.data(), al);
    enqueue_levels(c, levels, st);
    for (const Mask& k : masks) launch_mask_acc(c, k.wp, k.mask, k.pc0, k.pnc, k.y, k.nP, st);
    enqueue_levels(c, relin, st);
    copy_pairs(copies, ct_words(c), st);
  }
};

static void spmv_many(hs_ctx* c, int n, const hs_keyset* const* ks, const hs_matrix* const* m, const hs_ctvec* const* x,
                      hipStream_t st, hs_ctvec** y) {
  BatchWork w;
  w.prepare(c, n, ks, m, x, st, y);
  for (int i = 0; i < 5; i++) g_counters[i] = w.counters[i];  // the relinearisations add theirs
  w.enqueue(c, st);
  HS_CHECK_HIP(hipStreamSynchronize(st));
}
}  // namespace hs

extern "C" {

int hs_he_spmv(hs_ctx* c, const hs_keyset* ks, const hs_matrix* m, const hs_ctvec* x, void* stream, hs_ctvec** y) {
  return hs_he_spmv_batch(c, 1, &ks, &m, &x, stream, y);
}

int hs_he_spmv_batch(hs_ctx* c, int n, const hs_keyset* const* ks, const hs_matrix* const* m, const hs_ctvec* const* x,
                     void* stream, hs_ctvec** y) {
  return guarded([&] {
    HS_REQUIRE(c && n >= 0 && (n == 0 || (ks && m && x && y)), HS_EINVAL, "null argument");
    for (int r = 0; r < n; r++) {
      y[r] = nullptr;
      HS_REQUIRE(ks[r] && m[r] && x[r], HS_EINVAL, "null handle in the batch");
      HS_REQUIRE(ks[r]->ctx == c && m[r]->ctx == c && x[r]->ctx == c, HS_EKEY, "handles from another context");
      HS_REQUIRE(x[r]->n == (i64)m[r]->chunks.size(), HS_EINVAL, "the vector must hold one ciphertext per chunk");
    }
    std::vector<hs_ctvec*> out(n, nullptr);
    try {
      for (int r = 0; r < n; r++) out[r] = new_ctvec(c, (i64)m[r]->groups.size());
      spmv_many(c, n, ks, m, x, S(stream), out.data());
    } catch (...) {
      for (hs_ctvec* v : out) hs_ctvec_destroy(v);
      throw;
    }
    for (int r = 0; r < n; r++) y[r] = out[r];
  });
}

}  // extern "C"

int hs_he_spmv_noalloc(hs_ctx* c, const hs_keyset* ks, const hs_matrix* m, const hs_ctvec* x, uint64_t* y, int64_t y_words,
                       void* stream) {
  return guarded([&] {
    HS_REQUIRE(c && ks && m && x && y, HS_EINVAL, "null argument");
    HS_REQUIRE(ks->ctx == c && m->ctx == c && x->ctx == c, HS_EKEY, "handles from another context");
    HS_REQUIRE(x->n == (i64)m->chunks.size(), HS_EINVAL, "the vector must hold one ciphertext per chunk");
    HS_REQUIRE(((uintptr_t)y & 7) == 0, HS_EINVAL, "output pointer not 8-byte aligned");
    const i64 need = (i64)m->groups.size() * (i64)ct_words(c);
    HS_REQUIRE(y_words >= need, HS_ECAPACITY, "output holds " + std::to_string(y_words) + " words; the result needs " + std::to_string(need));
    HS_REQUIRE(c->na_scratch, HS_EDEVICE, "no fixed scratch array on this device");
    hs_ctvec out;
    out.ctx = c;
    out.n = (i64)m->groups.size();
    out.d = (u64*)y;
    out.owned = false;
    hs_ctvec* yp = &out;
    hipStream_t st = S(stream);
    Arena arena(c->na_scratch, c->na_bytes);
    BatchWork w;
    try {
      w.prepare(c, 1, &ks, &m, &x, st, &yp, &arena);
      for (int i = 0; i < 5; i++) g_counters[i] = w.counters[i];
      w.enqueue(c, st);
    } catch (...) {
      (void)hipStreamSynchronize(st);  // no launch of this call may still use the region after it returns
      throw;
    }
    HS_CHECK_HIP(hipStreamSynchronize(st));
  });
}

struct hs_batch_plan {
  hs_ctx* ctx = nullptr;
  std::vector<hs_ctvec*> y;
  hs::BatchWork work;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t last = nullptr;  // stream of the last replay
  bool ran = false;
};

extern "C" {

int hs_ctvec_copy(hs_ctvec* dst, const hs_ctvec* src, void* stream) {
  return guarded([&] {
    HS_REQUIRE(dst && src && dst->ctx == src->ctx, HS_EINVAL, "vectors of one context required");
    HS_REQUIRE(dst->n == src->n, HS_EINVAL, "ciphertext counts differ");
    if (dst->n && dst->d != src->d) {
      HS_CHECK_HIP(hipMemcpyAsync(dst->d, src->d, (size_t)src->n * ct_words(src->ctx) * sizeof(u64), hipMemcpyDeviceToDevice, S(stream)));
      note_async(dst->ctx, S(stream));
    }
  });
}

int hs_autotune(hs_ctx* c, const hs_keyset* ks, void* stream, double* report, int cap, int* len) {
  return guarded([&] {
    HS_REQUIRE(c && ks && ks->ctx == c && !ks->gk.empty(), HS_EINVAL, "autotuning needs a key-set of this context");
    hipStream_t st = S(stream);
    const size_t N = c->N, CW = ct_words(c);
    const int LK = c->L + c->K;
    constexpr int kBmax = 64, kIn = 4;
    // synthetic operands: canonical residues (their values do not affect the timing)
    std::vector<u64> host((size_t)kIn * CW);
    u64 z = 0x9E3779B97F4A7C15ULL;
    for (int i = 0; i < kIn; i++)
      for (int l = 0; l < 2 * c->L; l++)
        for (size_t k = 0; k < N; k++) {
          z ^= z << 13; z ^= z >> 7; z ^= z << 17;
          host[(size_t)i * CW + (size_t)l * N + k] = z % c->mod[l % c->L];
        }
    DBuf in(&c->pool, host.size() * sizeof(u64)), outb(&c->pool, (size_t)kBmax * CW * sizeof(u64));
    h2d(in.as<u64>(), host.data(), host.size(), st);
    std::vector<RotItem> items(kBmax);
    for (int i = 0; i < kBmax; i++) {
      items[i] = RotItem{};
      items[i].in = in.as<u64>() + (size_t)(i % kIn) * CW;
      items[i].out = outb.as<u64>() + (size_t)i * CW;
      items[i].key = ks->gk[0];
      items[i].galois = (u32)galois_step(c, 1);
    }
    DBuf ditems(&c->pool, items.size() * sizeof(RotItem));
    h2d(ditems.as<RotItem>(), items.data(), items.size(), st);
    const bool one_ok = lds_limb_fits(c);
    const KsShape Smax = ks_shape(c, 1);
    DBuf D, ACC, PC;
    if (one_ok) {
      D = DBuf(&c->pool, (size_t)kBmax * c->L * N * sizeof(u64));
      ACC = DBuf(&c->pool, (size_t)kBmax * Smax.ndg * 2 * LK * N * sizeof(double));
      PC = DBuf(&c->pool, (size_t)kBmax * 2 * c->K * N * sizeof(double));
    }
    DBuf T1(&c->pool, (size_t)kBmax * c->L * N * sizeof(double)), E(&c->pool, (size_t)kBmax * c->dnum * LK * N * sizeof(double)),
        ACC2(&c->pool, (size_t)kBmax * 2 * c->L * N * sizeof(double)), T2(&c->pool, (size_t)kBmax * 2 * c->K * N * sizeof(double)),
        F(&c->pool, (size_t)kBmax * 2 * c->L * N * sizeof(double));
    hipEvent_t ea, eb;
    HS_CHECK_HIP(hipEventCreate(&ea));
    HS_CHECK_HIP(hipEventCreate(&eb));
    auto level = [&](bool two, int B) {
      const KsShape Sh = ks_shape(c, B);
      if (two) launch_rotate_batch2(c, ditems.as<RotItem>(), B, Sh, T1.as<double>(), E.as<double>(), ACC2.as<double>(), T2.as<double>(),
                                    F.as<double>(), st);
      else launch_rotate_batch(c, ditems.as<RotItem>(), B, Sh, D.as<u64>(), ACC.as<double>(), PC.as<double>(), st);
    };
    auto time_ms = [&](bool two, int B) {
      level(two, B);  // warm-up
      const int reps = B <= 8 ? 5 : 3;
      HS_CHECK_HIP(hipEventRecord(ea, st));
      for (int r = 0; r < reps; r++) level(two, B);
      HS_CHECK_HIP(hipEventRecord(eb, st));
      HS_CHECK_HIP(hipEventSynchronize(eb));
      float ms = 0;
      HS_CHECK_HIP(hipEventElapsedTime(&ms, ea, eb));
      return (double)ms / reps;
    };
    std::vector<double> rep;
    try {
      // 1. limb-transform variant of the one-workgroup-per-limb kernels, timed on a 32-item level
      double tv[2] = {0, 0};
      const bool has_alt = one_ok && c->logn >= 11;
      if (has_alt) {
        for (int v = 0; v < 2; v++) {
          c->xf_variant = v;
          tv[v] = time_ms(false, 32);
        }
        c->xf_variant = tv[1] < tv[0] ? 1 : 0;
      } else {
        c->xf_variant = 0;
      }
      rep.push_back(c->xf_variant);
      rep.push_back(tv[0]);
      rep.push_back(tv[1]);
      // 1b. the same choice for the plain transform kernels, timed on forward + inverse transforms
      //     of 64 polynomials of L + K limbs
      double tn[2] = {0, 0};
      if (has_alt) {
        const int rows = 64 * LK;
        DBuf lim(&c->pool, (size_t)rows * N * sizeof(u64));
        HS_CHECK_HIP(hipMemcpyAsync(lim.as<u64>(), in.as<u64>(), std::min((size_t)rows * N, (size_t)kIn * CW) * sizeof(u64),
                                    hipMemcpyDeviceToDevice, st));
        if ((size_t)rows * N > (size_t)kIn * CW)  // the rest: valid residues of the first limbs, repeated
          for (size_t o = (size_t)kIn * CW; o < (size_t)rows * N; o += (size_t)kIn * CW)
            HS_CHECK_HIP(hipMemcpyAsync(lim.as<u64>() + o, in.as<u64>(), std::min((size_t)kIn * CW, (size_t)rows * N - o) * sizeof(u64),
                                        hipMemcpyDeviceToDevice, st));
        for (int v = 0; v < 2; v++) {
          c->xf_variant_ntt = v;
          auto pass = [&] {
            launch_ntt(c, lim.as<u64>(), rows, LK, 0, 0, st);
            launch_ntt(c, lim.as<u64>(), rows, LK, 0, 1, st);
          };
          pass();
          HS_CHECK_HIP(hipEventRecord(ea, st));
          for (int r = 0; r < 3; r++) pass();
          HS_CHECK_HIP(hipEventRecord(eb, st));
          HS_CHECK_HIP(hipEventSynchronize(eb));
          float ms = 0;
          HS_CHECK_HIP(hipEventElapsedTime(&ms, ea, eb));
          tn[v] = ms / 3.0;
        }
        c->xf_variant_ntt = tn[1] < tn[0] ? 1 : 0;
      } else {
        c->xf_variant_ntt = 0;
      }
      rep.push_back(c->xf_variant_ntt);
      rep.push_back(tn[0]);
      rep.push_back(tn[1]);
      // 2. key-switch pipeline per batch-size bucket
      double t1_64 = 0.0, t2_64 = 0.0;
      for (int b = 0; b < 7; b++) {
        const int B = 1 << b;
        const double t1 = one_ok ? time_ms(false, B) : 0.0;
        const double t2 = time_ms(true, B);
        c->ks_pick[b] = (!one_ok || t2 <= t1) ? 1 : 0;
        rep.push_back(B);
        rep.push_back(t1);
        rep.push_back(t2);
        t1_64 = t1; t2_64 = t2;
      }
      // levels above 64 items (not timed): the one-workgroup pipeline gains on the two-pass one
      // as levels grow (measured at 128 items: 104 K vs 88 K key switches/s at N = 16384), so the
      // two-pass one keeps them only if it is clearly ahead at 64
      c->ks_pick[7] = (!one_ok || t2_64 < 0.9 * t1_64) ? 1 : 0;
      HS_CHECK_HIP(hipStreamSynchronize(st));
    } catch (...) {
      (void)hipStreamSynchronize(st);
      (void)hipEventDestroy(ea);
      (void)hipEventDestroy(eb);
      throw;
    }
    (void)hipEventDestroy(ea);
    (void)hipEventDestroy(eb);
    if (len) *len = (int)rep.size();
    if (report) {
      HS_REQUIRE(cap >= (int)rep.size(), HS_ECAPACITY, "report buffer too small");
      std::copy(rep.begin(), rep.end(), report);
    }
  });
}

int hs_tuning(const hs_ctx* c, int64_t out[10]) {
  return guarded([&] {
    HS_REQUIRE(c && out, HS_EINVAL, "null argument");
    out[0] = c->xf_variant;
    out[1] = c->xf_variant_ntt;
    for (int b = 0; b < 8; b++) out[2 + b] = c->ks_pick[b];
  });
}

int hs_set_tuning(hs_ctx* c, const int64_t in[10]) {
  return guarded([&] {
    HS_REQUIRE(c && in, HS_EINVAL, "null argument");
    HS_REQUIRE((in[0] == 0 || in[0] == 1) && (in[1] == 0 || in[1] == 1), HS_EINVAL, "transform variants must be 0 or 1");
    for (int b = 0; b < 8; b++) HS_REQUIRE(in[2 + b] >= -1 && in[2 + b] <= 1, HS_EINVAL, "pipeline pick must be -1, 0 or 1");
    c->xf_variant = (int)in[0];
    c->xf_variant_ntt = (int)in[1];
    for (int b = 0; b < 8; b++) c->ks_pick[b] = (signed char)in[2 + b];
  });
}

int hs_batch_plan_create(hs_ctx* c, int n, const hs_keyset* const* ks, const hs_matrix* const* m, const hs_ctvec* const* x,
                         void* stream, hs_batch_plan** out) {
  return guarded([&] {
    HS_REQUIRE(c && out && n >= 1 && ks && m && x, HS_EINVAL, "null argument or empty batch");
    *out = nullptr;
    for (int r = 0; r < n; r++) {
      HS_REQUIRE(ks[r] && m[r] && x[r], HS_EINVAL, "null handle in the batch");
      HS_REQUIRE(ks[r]->ctx == c && m[r]->ctx == c && x[r]->ctx == c, HS_EKEY, "handles from another context");
      HS_REQUIRE(x[r]->n == (i64)m[r]->chunks.size(), HS_EINVAL, "the vector must hold one ciphertext per chunk");
      HS_REQUIRE(!m[r]->encrypted, HS_EINVAL, "graph plans take plaintext matrices");
    }
    hipStream_t st = S(stream);
    hs_batch_plan* P = new hs_batch_plan();
    P->ctx = c;
    hipStream_t cs = nullptr;
    try {
      for (int r = 0; r < n; r++) P->y.push_back(new_ctvec(c, (i64)m[r]->groups.size()));
      P->work.prepare(c, n, ks, m, x, st, P->y.data());
      // one eager pass: the results are valid at once, and every kernel attribute is set before
      // recording (no runtime configuration calls inside the captured region)
      P->work.enqueue(c, st);
      HS_CHECK_HIP(hipStreamSynchronize(st));
      HS_CHECK_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      profile_capturing(true);
      hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        try {
          P->work.enqueue(c, cs);
        } catch (...) {
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(cs, &g);
          if (g) (void)hipGraphDestroy(g);
          throw;
        }
        e = hipStreamEndCapture(cs, &P->graph);
      }
      profile_capturing(false);
      HS_CHECK_HIP(e);
      HS_CHECK_HIP(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0));
      HS_CHECK_HIP(hipStreamDestroy(cs));
      cs = nullptr;
    } catch (...) {
      profile_capturing(false);
      if (cs) (void)hipStreamDestroy(cs);
      (void)hipStreamSynchronize(st);
      hs_batch_plan_destroy(P);
      throw;
    }
    *out = P;
  });
}

int hs_batch_plan_run(hs_batch_plan* P, void* stream) {
  return guarded([&] {
    HS_REQUIRE(P && P->exec, HS_EINVAL, "null plan");
    hipStream_t st = S(stream);
    HS_CHECK_HIP(hipGraphLaunch(P->exec, st));
    note_async(P->ctx, st);
    P->last = st;
    P->ran = true;
  });
}

int hs_batch_plan_output(const hs_batch_plan* P, int i, const hs_ctvec** y) {
  return guarded([&] {
    HS_REQUIRE(P && y && i >= 0 && i < (int)P->y.size(), HS_EINVAL, "bad plan output index");
    *y = P->y[i];
  });
}

void hs_batch_plan_destroy(hs_batch_plan* P) {
  if (!P) return;
  if (P->ran) (void)hipStreamSynchronize(P->last);
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  for (hs_ctvec* v : P->y) hs_ctvec_destroy(v);
  delete P;
}

int hs_decrypt(hs_ctx* c, const hs_keyset* ks, const hs_matrix* m, const hs_ctvec* y, int64_t* out, int64_t rows,
               void* stream) {
  return guarded([&] {
    HS_REQUIRE(c && ks && m && y, HS_EINVAL, "null argument");
    HS_REQUIRE(ks->ctx == c && m->ctx == c && y->ctx == c, HS_EKEY, "handles from another context");
    HS_REQUIRE(rows == m->R, HS_EINVAL, "rows must equal the matrix row count");
    HS_REQUIRE(y->n == (i64)m->groups.size(), HS_EINVAL, "one result ciphertext per partition group expected");
    HS_REQUIRE(rows == 0 || out, HS_EINVAL, "null output");
    hipStream_t st = S(stream);
    const int nP = (int)m->parts.size(), nG = (int)m->groups.size();
    if (!nP) return;
    const size_t N = c->N;
    DBuf X(&c->pool, (size_t)nG * c->L * N * sizeof(u64)), Mc(&c->pool, (size_t)nG * N * sizeof(u64));
    std::vector<DBuf> hold;
    const bool split = use_split_client(c);
    if (split) {
      launch_dec_prep(c, y->d, ks->sk, X.as<u64>(), nG, st);
      ntt_any(c, X.as<u64>(), (i64)nG * c->L, c->L, 0, 1, st, hold);
    } else {
      launch_dec_phase(c, y->d, ks->sk, X.as<u64>(), nG, st);
    }
    launch_dec_round(c, X.as<u64>(), Mc.as<u64>(), nG, st);
    // decode per result ciphertext, scatter per partition (slot row 0 or 1 of its group's ciphertext)
    if (split || nG != nP) {
      ntt_any(c, Mc.as<u64>(), nG, 1, c->n_mod, 0, st, hold);
      launch_slots_scatter(c, Mc.as<u64>(), m->d_rm, m->d_pinfo, nP, out, st);
    } else {
      launch_decode_scatter(c, Mc.as<u64>(), m->d_rm, m->d_pinfo, out, nP, st);
    }
    HS_CHECK_HIP(hipStreamSynchronize(st));
  });
}

int hs_ctvec_count(const hs_ctvec* v, int64_t* n) {
  return guarded([&] {
    HS_REQUIRE(v && n, HS_EINVAL, "null argument");
    *n = v->n;
  });
}

int hs_ct_export(const hs_ctvec* v, int64_t i, uint64_t* host_limbs, int64_t cap) {
  return guarded([&] {
    HS_REQUIRE(v && host_limbs, HS_EINVAL, "null argument");
    HS_REQUIRE(i >= 0 && i < v->n, HS_EINVAL, "ciphertext index out of range");
    const size_t n = ct_words(v->ctx);
    HS_REQUIRE((size_t)cap >= n, HS_ECAPACITY, "output too small");
    HS_CHECK_HIP(hipDeviceSynchronize());
    HS_CHECK_HIP(hipMemcpy(host_limbs, v->d + i * n, n * sizeof(u64), hipMemcpyDeviceToHost));
  });
}

int hs_ct_export_coeff(const hs_ctvec* v, int64_t i, uint64_t* host_limbs, int64_t cap, void* stream) {
  return guarded([&] {
    HS_REQUIRE(v && host_limbs, HS_EINVAL, "null argument");
    HS_REQUIRE(i >= 0 && i < v->n, HS_EINVAL, "ciphertext index out of range");
    hs_ctx* c = v->ctx;
    const size_t n = ct_words(c);
    HS_REQUIRE((size_t)cap >= n, HS_ECAPACITY, "output too small");
    const hipStream_t st = S(stream);
    std::vector<DBuf> hold;
    DBuf tmp(&c->pool, n * sizeof(u64));
    HS_CHECK_HIP(hipMemcpyAsync(tmp.as<u64>(), v->d + i * n, n * sizeof(u64), hipMemcpyDeviceToDevice, st));
    ntt_any(c, tmp.as<u64>(), 2 * c->L, c->L, 0, 1, st, hold);
    HS_CHECK_HIP(hipMemcpyAsync(host_limbs, tmp.as<u64>(), n * sizeof(u64), hipMemcpyDeviceToHost, st));
    HS_CHECK_HIP(hipStreamSynchronize(st));
  });
}

int hs_ctvec_wrap(hs_ctx* c, void* dev, int64_t n, hs_ctvec** out) {
  return guarded([&] {
    HS_REQUIRE(c && dev && out, HS_EINVAL, "null argument");
    HS_REQUIRE(n >= 1, HS_EINVAL, "need at least one ciphertext");
    HS_REQUIRE(((uintptr_t)dev & 7) == 0, HS_EINVAL, "device pointer not 8-byte aligned");
    *out = nullptr;
    hs_ctvec* v = new hs_ctvec();
    v->ctx = c;
    v->n = n;
    v->d = (u64*)dev;
    v->owned = false;
    *out = v;
  });
}

int hs_ctvec_import(hs_ctx* c, const uint64_t* host_limbs, int64_t n, hs_ctvec** out) {
  return guarded([&] {
    HS_REQUIRE(c && out && (n == 0 || host_limbs) && n >= 0, HS_EINVAL, "bad argument");
    *out = nullptr;
    const size_t CW = ct_words(c);
    for (int64_t k = 0; k < n; k++)
      for (int w = 0; w < 2; w++)
        for (int l = 0; l < c->L; l++)
          for (size_t i = 0; i < c->N; i++)
            HS_REQUIRE(host_limbs[k * CW + ((size_t)w * c->L + l) * c->N + i] < c->mod[l], HS_EINVAL, "residue out of range");
    hs_ctvec* v = new_ctvec(c, n);
    if (n) {
      hipError_t e = hipMemcpy(v->d, host_limbs, n * CW * sizeof(u64), hipMemcpyHostToDevice);
      if (e != hipSuccess) { hs_ctvec_destroy(v); throw Error{HS_EDEVICE, hipGetErrorString(e)}; }
    }
    *out = v;
  });
}

void hs_ctvec_destroy(hs_ctvec* v) {
  if (!v) return;
  if (v->d && v->owned) {
    drain_async(v->ctx);  // as for matrices: no asynchronous call in flight may still use the memory
    pfree(v->ctx, v->d);
  }
  delete v;
}

int hs_ntt(hs_ctx* c, uint64_t* d_limbs, int64_t n_polys, int mod0, int n_limbs, int inverse, void* stream) {
  return guarded([&] {
    HS_REQUIRE(c && (n_polys == 0 || d_limbs), HS_EINVAL, "null argument");
    HS_REQUIRE(n_polys >= 0 && n_limbs >= 1, HS_EINVAL, "bad counts");
    int m0 = mod0;
    if (mod0 < 0) {
      HS_REQUIRE(n_limbs == 1, HS_EINVAL, "the plaintext modulus is a single limb");
      m0 = c->n_mod;
    } else {
      HS_REQUIRE(mod0 + n_limbs <= c->n_mod, HS_EINVAL, "modulus index out of range");
    }
    const bool two = (!lds_limb_fits(c) && !ntt15_one_wg(c, (i64)n_polys * n_limbs)) || option(c, HS_OPT_NTT_PATH) == 2;
    if (two) {
      DBuf scratch(&c->pool, (size_t)n_polys * n_limbs * c->N * sizeof(double));
      launch_ntt2(c, d_limbs, scratch.as<double>(), n_polys * n_limbs, n_limbs, m0, inverse, S(stream));
      HS_CHECK_HIP(hipStreamSynchronize(S(stream)));
    } else {
      launch_ntt(c, d_limbs, n_polys * n_limbs, n_limbs, m0, inverse, S(stream));
    }
  });
}

static void check_option(int key, int64_t value) {
  switch (key) {
    case HS_OPT_AUX_PATH:
      HS_REQUIRE(value >= 0 && value <= 2, HS_EINVAL, "path must be 0, 1 or 2");
      break;
    case HS_OPT_KS_PIPELINE:
      HS_REQUIRE(value >= 0 && value <= 2, HS_EINVAL, "pipeline must be 0, 1 or 2");
      break;
    case HS_OPT_NTT_PATH:
      HS_REQUIRE(value >= 0 && value <= 2, HS_EINVAL, "path must be 0, 1 or 2");
      break;
    case HS_OPT_KS_BLOCK:
      HS_REQUIRE(value >= 0 && value <= 3, HS_EINVAL, "key-switch block option must be 0, 1, 2 or 3");
      break;
    case HS_OPT_NTT_PIPE:
      HS_REQUIRE(value == 0 || value == 1, HS_EINVAL, "ntt pipe option must be 0 or 1");
      break;
    case HS_OPT_MODUP_GROUP:
      HS_REQUIRE(value >= 0 && value <= 3, HS_EINVAL, "group must be 0, 1, 2 or 3");
      break;
    case HS_OPT_MODUP_ACC:
      HS_REQUIRE(value >= 0 && value <= 3, HS_EINVAL, "accumulator option must be 0, 1, 2 or 3");
      break;
    case HS_OPT_KS_FUSE:
      HS_REQUIRE(value == 0 || value == 1, HS_EINVAL, "fusion option must be 0 or 1");
      break;
    case HS_OPT_KS_THRESHOLD:
      HS_REQUIRE(value >= 0 && value < (1 << 30), HS_EINVAL, "bad threshold");
      break;
    default:
      throw Error{HS_EINVAL, "unknown option"};
  }
}

int hs_set_option(int key, int64_t value) {
  return guarded([&] {
    check_option(key, value);
    g_opt[key] = (int)value;
  });
}

int hs_ctx_set_option(hs_ctx* c, int key, int64_t value) {
  return guarded([&] {
    HS_REQUIRE(c, HS_EINVAL, "null context");
    if (value != -1) check_option(key, value);
    else HS_REQUIRE(key > 0 && key < 10, HS_EINVAL, "unknown option");
    c->opt[key] = (int)value;
  });
}

int hs_mul_plain(hs_ctx* c, const hs_ctvec* in, const uint64_t* d_pt, void* stream, hs_ctvec** out) {
  return guarded([&] {
    HS_REQUIRE(c && in && d_pt && out, HS_EINVAL, "null argument");
    *out = nullptr;
    hs_ctvec* r = new_ctvec(c, in->n);
    launch_mul_plain(c, in->d, d_pt, r->d, in->n, 0, S(stream));
    note_async(c, S(stream));
    *out = r;
  });
}

int hs_rotate(hs_ctx* c, const hs_keyset* ks, const hs_ctvec* in, int64_t k, void* stream, hs_ctvec** out) {
  return guarded([&] {
    HS_REQUIRE(c && ks && in && out, HS_EINVAL, "null argument");
    *out = nullptr;
    HS_REQUIRE(ks->ctx == c && in->ctx == c, HS_EKEY, "handles from another context");
    hipStream_t st = S(stream);
    const size_t CW = ct_words(c);
    const i64 half = (i64)c->N / 2;
    const i64 kk = ((k % half) + half) % half;
    hs_ctvec* r = new_ctvec(c, in->n);
    try {
      if (in->n) HS_CHECK_HIP(hipMemcpyAsync(r->d, in->d, in->n * CW * sizeof(u64), hipMemcpyDeviceToDevice, st));
      DBuf tmp(&c->pool, std::max<i64>(in->n, 1) * CW * sizeof(u64));
      u64* cur = r->d;
      u64* other = tmp.as<u64>();
      std::vector<std::vector<RotItem>> levels;
      const std::vector<i64> steps = rotation_digits(c, ks, kk);  // one exact-step key switch, or the digits
      for (i64 step : steps) {
        std::vector<RotItem> items;
        for (i64 g = 0; g < in->n; g++) {
          RotItem it{};
          it.in = cur + g * CW; it.out = other + g * CW; it.addend = nullptr;
          it.key = rotation_key(ks, step); it.galois = (u32)galois_step(c, step);
          items.push_back(it);
        }
        levels.push_back(items);
        std::swap(cur, other);
      }
      run_rotation_levels(c, levels, st);
      if (cur != r->d && in->n) HS_CHECK_HIP(hipMemcpyAsync(r->d, cur, in->n * CW * sizeof(u64), hipMemcpyDeviceToDevice, st));
      HS_CHECK_HIP(hipStreamSynchronize(st));
    } catch (...) {
      hs_ctvec_destroy(r);
      throw;
    }
    *out = r;
  });
}

int hs_mul_ct(hs_ctx* c, const hs_keyset* ks, const hs_ctvec* a, const hs_ctvec* b, void* stream, hs_ctvec** out) {
  return guarded([&] {
    HS_REQUIRE(c && ks && a && b && out, HS_EINVAL, "null argument");
    *out = nullptr;
    HS_REQUIRE(ks->ctx == c && a->ctx == c && b->ctx == c, HS_EKEY, "handles from another context");
    HS_REQUIRE(a->n == b->n, HS_EINVAL, "vectors of different lengths");
    const size_t CW = ct_words(c);
    hs_ctvec* r = new_ctvec(c, a->n);
    try {
      std::vector<const u64*> pa, pb, rk;
      std::vector<u64*> po;
      for (i64 i = 0; i < a->n; i++) {
        pa.push_back(a->d + i * CW);
        pb.push_back(b->d + i * CW);
        po.push_back(r->d + i * CW);
        rk.push_back(ks->rk);
      }
      mul_ct_batch(c, (int)a->n, pa.data(), pb.data(), po.data(), rk.data(), S(stream));
    } catch (...) {
      hs_ctvec_destroy(r);
      throw;
    }
    *out = r;
  });
}

// ---------------------------------------------------------------- the diagonal method
// The paper's baseline (Sec. 5, baseline approaches; the diagonal-method figure): square blocks of
// side B = min(N/4, max(R, C)), one plaintext per non-empty generalised block diagonal, the vector
// block encrypted twice over, and per block row the sum of diagonal (.) Rot(x_bj, d).
int hs_diag_pack(hs_ctx* c, int64_t rows, int64_t cols, const int64_t* row_ptr, const int32_t* col_idx, const int64_t* vals,
                 void* stream, hs_diag** out) {
  return guarded([&] {
    HS_REQUIRE(c && out, HS_EINVAL, "null argument");
    *out = nullptr;
    HS_REQUIRE(rows >= 0 && cols >= 0 && rows < (1LL << 31) && cols < (1LL << 31), HS_EINVAL, "bad matrix shape");
    HS_REQUIRE(rows == 0 || row_ptr, HS_EINVAL, "null row_ptr");
    hipStream_t st = S(stream);
    const size_t N = c->N;
    std::vector<i64> rp(rows + 1, 0);
    if (rows) {
      d2h(rp.data(), row_ptr, rows + 1, st);
      HS_CHECK_HIP(hipStreamSynchronize(st));
    }
    HS_REQUIRE(rp[0] == 0, HS_EINVAL, "row_ptr[0] must be 0");
    for (i64 i = 0; i < rows; i++) HS_REQUIRE(rp[i + 1] >= rp[i], HS_EINVAL, "row_ptr must be nondecreasing");
    const i64 nnz = rp[rows];
    HS_REQUIRE(nnz == 0 || (col_idx && vals), HS_EINVAL, "null col_idx/vals");
    hs_diag* D = new hs_diag();
    D->ctx = c; D->R = rows; D->C = cols;
    D->B = std::min<i64>((i64)N / 4, std::max<i64>(std::max<i64>(rows, cols), 1));
    D->nrb = (int)((rows + D->B - 1) / D->B);
    D->ncb = (int)((cols + D->B - 1) / D->B);
    try {
      const i64 B = D->B, nids = (i64)D->nrb * D->ncb * B;
      HS_REQUIRE(nids < (1LL << 31), HS_ECAPACITY, "too many block diagonals for the diagonal method (one flag byte each on host and device)");
      // non-empty diagonals: flagged on the device, listed in ascending id order on the host
      std::vector<i64> ids;
      if (nnz) {
        const size_t fbytes = ((size_t)nids + 255) & ~(size_t)255;
        DBuf flags(&c->pool, fbytes + 256);
        unsigned char* fl = flags.as<unsigned char>();
        int* dbad = (int*)(fl + fbytes);
        HS_CHECK_HIP(hipMemsetAsync(fl, 0, fbytes + 256, st));
        launch_csr_check(row_ptr, col_idx, rows, cols, dbad, st);
        launch_diag_mark(row_ptr, col_idx, rows, cols, B, D->ncb, fl, st);
        std::vector<unsigned char> h(fbytes + 256);
        d2h(h.data(), fl, h.size(), st);
        HS_CHECK_HIP(hipStreamSynchronize(st));
        int bad = 0;
        std::memcpy(&bad, h.data() + fbytes, sizeof(int));
        HS_REQUIRE(!bad, HS_EINVAL, "column indices out of range or not strictly ascending within a row");
        for (i64 id = 0; id < nids; id++)
          if (h[id]) ids.push_back(id);
      }
      const i64 nd = (i64)ids.size();
      HS_REQUIRE(nd < (1LL << 31), HS_ECAPACITY, "too many diagonals");
      D->row0.assign(D->nrb, 0);
      D->rown.assign(D->nrb, 0);
      for (i64 k = 0; k < nd; k++) {
        const i64 bi = ids[k] / ((i64)D->ncb * B), rem = ids[k] % ((i64)D->ncb * B);
        D->key.insert(D->key.end(), {bi, rem / B, rem % B});
        if (!D->rown[bi]) D->row0[bi] = (int)k;
        D->rown[bi]++;
      }
      // identity row map [B] | per block row (row0, rows, rows, 0, block row, 0) | diagonal ids
      std::vector<i32> rm(B);
      std::iota(rm.begin(), rm.end(), 0);
      std::vector<i64> pinfo(6ULL * std::max(D->nrb, 1), 0);
      for (int bi = 0; bi < D->nrb; bi++) {
        i64* q = &pinfo[6ULL * bi];
        q[0] = bi * B; q[1] = std::min(B, rows - bi * B); q[2] = q[1]; q[3] = 0; q[4] = bi; q[5] = 0;
      }
      auto seg = [](size_t bytes) { return (bytes + 255) & ~(size_t)255; };
      const size_t o_rm = 0, o_pi = seg(rm.size() * 4), o_id = o_pi + seg(pinfo.size() * 8), total = o_id + seg(ids.size() * 8 + 8);
      char* up = (char*)t_stage_up.get(total);
      std::memcpy(up + o_rm, rm.data(), rm.size() * 4);
      std::memcpy(up + o_pi, pinfo.data(), pinfo.size() * 8);
      if (nd) std::memcpy(up + o_id, ids.data(), ids.size() * 8);
      D->d_struct = pmalloc<char>(c, total);
      HS_CHECK_HIP(hipMemcpyAsync(D->d_struct, up, total, hipMemcpyHostToDevice, st));
      D->d_rm = (i32*)(D->d_struct + o_rm);
      D->d_pinfo = (i64*)(D->d_struct + o_pi);
      std::vector<DBuf> hold;
      if (nd) {
        DBuf coef(&c->pool, (size_t)nd * N * sizeof(u64));
        HS_CHECK_HIP(hipMemsetAsync(coef.p, 0, coef.bytes, st));
        launch_diag_place(c, row_ptr, col_idx, vals, rows, B, D->ncb, (const i64*)(D->d_struct + o_id), (int)nd, coef.as<u64>(), st);
        ntt_any(c, coef.as<u64>(), nd, 1, c->n_mod, 1, st, hold);
        D->d_pt = pmalloc<u64>(c, (size_t)nd * c->L * N);
        plain_ntt(c, coef.as<u64>(), D->d_pt, (int)nd, st, hold);
        HS_CHECK_HIP(hipStreamSynchronize(st));
      } else {
        HS_CHECK_HIP(hipStreamSynchronize(st));
      }
    } catch (...) {
      (void)hipStreamSynchronize(st);
      hs_diag_destroy(D);
      throw;
    }
    *out = D;
  });
}

void hs_diag_destroy(hs_diag* D) {
  if (!D) return;
  (void)hipDeviceSynchronize();
  pfree(D->ctx, D->d_struct);
  pfree(D->ctx, D->d_pt);
  delete D;
}

int hs_diag_info(const hs_diag* D, int64_t out4[4]) {
  return guarded([&] {
    HS_REQUIRE(D && out4, HS_EINVAL, "null argument");
    out4[0] = D->B; out4[1] = D->nrb; out4[2] = D->ncb; out4[3] = (int64_t)D->key.size() / 3;
  });
}

int hs_diag_keys(const hs_diag* D, int64_t* host_out, int64_t cap) {
  return guarded([&] {
    HS_REQUIRE(D, HS_EINVAL, "null argument");
    HS_REQUIRE(cap >= (int64_t)D->key.size() && (host_out || D->key.empty()), HS_ECAPACITY, "output too small");
    if (!D->key.empty()) std::memcpy(host_out, D->key.data(), D->key.size() * sizeof(i64));
  });
}

int hs_diag_export(const hs_diag* D, int64_t k, uint64_t* host_out, int64_t cap) {
  return guarded([&] {
    HS_REQUIRE(D && host_out, HS_EINVAL, "null argument");
    HS_REQUIRE(k >= 0 && k < (int64_t)D->key.size() / 3, HS_EINVAL, "diagonal index out of range");
    const size_t n = (size_t)D->ctx->L * D->ctx->N;
    HS_REQUIRE((size_t)cap >= n, HS_ECAPACITY, "output too small");
    HS_CHECK_HIP(hipMemcpy(host_out, D->d_pt + k * n, n * sizeof(u64), hipMemcpyDeviceToHost));
  });
}

int hs_diag_rotation_steps(const hs_diag* D, int64_t* out, int64_t cap, int64_t* len) {
  return guarded([&] {
    HS_REQUIRE(D && len, HS_EINVAL, "null argument");
    std::vector<char> used(D->B, 0);
    for (size_t k = 0; k < D->key.size(); k += 3) used[D->key[k + 2]] = 1;
    std::vector<i64> steps;
    for (i64 d = 1; d < D->B; d++)
      if (used[d]) steps.push_back(d);
    *len = (int64_t)steps.size();
    HS_REQUIRE(cap >= *len && (out || steps.empty()), HS_ECAPACITY, "output too small");
    if (!steps.empty()) std::memcpy(out, steps.data(), steps.size() * sizeof(i64));
  });
}

int hs_diag_encrypt(hs_ctx* c, const hs_keyset* ks, const hs_diag* D, const int64_t* v, int64_t len, uint64_t seed, void* stream,
                    hs_ctvec** out) {
  return guarded([&] {
    HS_REQUIRE(c && ks && D && out, HS_EINVAL, "null argument");
    *out = nullptr;
    HS_REQUIRE(ks->ctx == c && D->ctx == c, HS_EKEY, "handles from another context");
    HS_REQUIRE(len == D->C, HS_EINVAL, "vector length must equal the number of matrix columns");
    HS_REQUIRE(len == 0 || v, HS_EINVAL, "null vector");
    hipStream_t st = S(stream);
    const int G = D->ncb;
    const size_t N = c->N;
    hs_ctvec* x = new_ctvec(c, G);
    try {
      if (G) {
        std::vector<DBuf> hold;
        DBuf coef(&c->pool, (size_t)G * N * sizeof(u64));
        launch_diag_vector(c, v, D->C, D->B, G, coef.as<u64>(), st);
        ntt_any(c, coef.as<u64>(), G, 1, c->n_mod, 1, st, hold);
        DBuf smp(&c->pool, (size_t)G * 3 * N * sizeof(int));
        launch_sample_enc(c, smp.as<int>(), G, seed, P_ENC_U, P_ENC_E0, P_ENC_E1, st);
        encrypt_coefs(c, coef.as<u64>(), smp.as<int>(), ks->pk, x->d, G, st, hold);
        HS_CHECK_HIP(hipStreamSynchronize(st));
      }
    } catch (...) {
      (void)hipStreamSynchronize(st);
      hs_ctvec_destroy(x);
      throw;
    }
    *out = x;
  });
}

// Rotations of the vector blocks: Rot(x_bj, d) for every (bj, d) a diagonal needs.  With an
// exact-step key for d, one key switch from x_bj; otherwise the power-of-two digits of d
// (rotation_digits, lowest first: binary, or signed with the right keys), so
// Rot(x_bj, v) = Rot_z(Rot(x_bj, v - z)) for every partial sum v of those digits with z its top
// digit: every such partial rotation is computed once per block column and shared (the low
// digits of a binary expansion or of a non-adjacent form are the expansion of their own sum, so
// the partial rotation of a value is the same whichever offset reaches it).  Level h holds the
// partial rotations whose top digit is +-2^h (the exact-step ones go to level 0); levels are cut
// into batches of at most kDiagBatch key switches.
static constexpr size_t kDiagBatch = 256;
int hs_diag_spmv(hs_ctx* c, const hs_keyset* ks, const hs_diag* D, const hs_ctvec* x, void* stream, hs_ctvec** y) {
  return guarded([&] {
    HS_REQUIRE(c && ks && D && x && y, HS_EINVAL, "null argument");
    *y = nullptr;
    HS_REQUIRE(ks->ctx == c && D->ctx == c && x->ctx == c, HS_EKEY, "handles from another context");
    HS_REQUIRE(x->n == D->ncb, HS_EINVAL, "one encrypted vector block per block column expected");
    hipStream_t st = S(stream);
    const size_t CW = ct_words(c);
    const i64 B = D->B, nd = (i64)D->key.size() / 3;
    hs_ctvec* r = new_ctvec(c, D->nrb);
    try {
      // per block column: slot of each partial (digit) rotation, by its value, and of each
      // exact-step rotation (a step with an exact key may also be a partial rotation of another
      // step's digits: the two are different ciphertexts and both are kept)
      struct Part { int buf; i64 parent, digit; };   // parent 0: the vector block itself
      std::vector<std::map<i64, Part>> tree(D->ncb);
      std::vector<std::vector<int>> direct(D->ncb, std::vector<int>(B, -1));
      std::vector<std::vector<i64>> whole(D->ncb, std::vector<i64>(B, 0));   // d -> its last partial sum
      std::vector<std::vector<char>> seen(D->ncb, std::vector<char>(B, 0));
      int nbuf = 0, nlog = 0;
      for (i64 k = 0; k < nd; k++) {
        const i64 bj = D->key[3 * k + 1], d = D->key[3 * k + 2];
        if (!d || seen[bj][d]) continue;
        seen[bj][d] = 1;
        nlog++;
        if (!is_pow2(d) && ks->step_keys.count(d)) { direct[bj][d] = nbuf++; continue; }
        i64 v = 0;
        for (i64 z : rotation_digits(c, ks, d)) {
          if (!tree[bj].count(v + z)) tree[bj][v + z] = Part{nbuf++, v, z};
          v += z;
        }
        if (v == 0) throw Error{HS_EINVAL, "internal: diagonal offset that rotates by whole rows"};
        whole[bj][d] = v;
      }
      DBuf rot(&c->pool, (size_t)std::max(nbuf, 1) * CW * sizeof(u64));
      auto at = [&](int idx) { return rot.as<u64>() + (size_t)idx * CW; };
      std::vector<std::vector<RotItem>> levels;
      auto push = [&](std::vector<RotItem>& lv, const RotItem& it) {
        lv.push_back(it);
        if (lv.size() == kDiagBatch) { levels.push_back(lv); lv.clear(); }
      };
      for (int h = 0; h < n_pow2(c); h++) {
        std::vector<RotItem> lv;
        for (int bj = 0; bj < D->ncb; bj++) {
          const u64* xb = x->d + (size_t)bj * CW;
          if (h == 0)
            for (i64 d = 1; d < B; d++)
              if (direct[bj][d] >= 0) {
                RotItem it{};
                it.in = xb; it.out = at(direct[bj][d]); it.addend = nullptr;
                it.key = rotation_key(ks, d); it.galois = (u32)galois_step(c, d);
                push(lv, it);
              }
          for (const auto& kv : tree[bj]) {
            const Part& pt = kv.second;
            if ((pt.digit < 0 ? -pt.digit : pt.digit) != (1LL << h)) continue;
            RotItem it{};
            it.in = pt.parent ? at(tree[bj].at(pt.parent).buf) : xb; it.out = at(pt.buf); it.addend = nullptr;
            it.key = rotation_key(ks, pt.digit); it.galois = (u32)galois_step(c, pt.digit);
            push(lv, it);
          }
        }
        if (!lv.empty()) levels.push_back(lv);
      }
      for (int i = 0; i < 5; i++) g_counters[i] = 0;
      run_rotation_levels(c, levels, st);
      g_counters[1] = nlog;
      // per block row: sum over its diagonals of plaintext (.) rotated block (one pass, the
      // masked-sum kernel with the diagonals as masks)
      if (D->nrb) {
        std::vector<u64> words(std::max<i64>(nd, 1), 0);
        for (i64 k = 0; k < nd; k++) {
          const i64 bj = D->key[3 * k + 1], d = D->key[3 * k + 2];
          const u64* src = !d ? x->d + (size_t)bj * CW : at(direct[bj][d] >= 0 ? direct[bj][d] : tree[bj].at(whole[bj][d]).buf);
          words[k] = (u64)(uintptr_t)src;
        }
        const size_t w0 = words.size();
        words.resize(w0 + ((size_t)2 * D->nrb * sizeof(int) + 7) / 8, 0);
        std::memcpy(words.data() + w0, D->row0.data(), D->nrb * sizeof(int));
        std::memcpy((char*)(words.data() + w0) + D->nrb * sizeof(int), D->rown.data(), D->nrb * sizeof(int));
        DBuf dw(&c->pool, words.size() * sizeof(u64));
        h2d(dw.as<u64>(), words.data(), words.size(), st);
        const int* pc0 = (const int*)(dw.as<u64>() + w0);
        launch_mask_acc(c, (const u64* const*)dw.as<u64>(), D->d_pt, pc0, pc0 + D->nrb, r->d, D->nrb, st);
        g_counters[2] += 1;
        HS_CHECK_HIP(hipStreamSynchronize(st));
      }
      g_counters[3] = nd;
    } catch (...) {
      (void)hipStreamSynchronize(st);
      hs_ctvec_destroy(r);
      throw;
    }
    *y = r;
  });
}

int hs_diag_decrypt(hs_ctx* c, const hs_keyset* ks, const hs_diag* D, const hs_ctvec* y, int64_t* out, int64_t rows, void* stream) {
  return guarded([&] {
    HS_REQUIRE(c && ks && D && y, HS_EINVAL, "null argument");
    HS_REQUIRE(ks->ctx == c && D->ctx == c && y->ctx == c, HS_EKEY, "handles from another context");
    HS_REQUIRE(rows == D->R, HS_EINVAL, "rows must equal the matrix row count");
    HS_REQUIRE(y->n == D->nrb, HS_EINVAL, "one result ciphertext per block row expected");
    HS_REQUIRE(rows == 0 || out, HS_EINVAL, "null output");
    const int nb = D->nrb;
    if (!nb) return;
    hipStream_t st = S(stream);
    const size_t N = c->N;
    DBuf X(&c->pool, (size_t)nb * c->L * N * sizeof(u64)), Mc(&c->pool, (size_t)nb * N * sizeof(u64));
    std::vector<DBuf> hold;
    if (use_split_client(c)) {
      launch_dec_prep(c, y->d, ks->sk, X.as<u64>(), nb, st);
      ntt_any(c, X.as<u64>(), (i64)nb * c->L, c->L, 0, 1, st, hold);
    } else {
      launch_dec_phase(c, y->d, ks->sk, X.as<u64>(), nb, st);
    }
    launch_dec_round(c, X.as<u64>(), Mc.as<u64>(), nb, st);
    ntt_any(c, Mc.as<u64>(), nb, 1, c->n_mod, 0, st, hold);
    launch_slots_scatter(c, Mc.as<u64>(), D->d_rm, D->d_pinfo, nb, out, st);
    HS_CHECK_HIP(hipStreamSynchronize(st));
  });
}

int hs_profile(int enable) {
  return guarded([&] { profile_enable(enable != 0); });
}

int hs_profile_summary(char* buf, int64_t cap, int64_t* len) {
  return guarded([&] {
    HS_REQUIRE(len, HS_EINVAL, "null argument");
    const std::string s = profile_summary();
    *len = (int64_t)s.size();
    HS_REQUIRE(buf && cap > (int64_t)s.size(), HS_ECAPACITY, "output too small");
    memcpy(buf, s.c_str(), s.size() + 1);
  });
}

int hs_last_counters(int64_t out[5]) {
  return guarded([&] {
    HS_REQUIRE(out, HS_EINVAL, "null argument");
    for (int i = 0; i < 5; i++) out[i] = g_counters[i];
  });
}

}  // extern "C"

// ====================================================================== continuous-batching server
// Requests (key-set, packed matrix, encrypted vector) are queued by hs_server_submit.  A worker
// thread runs engine ticks: it admits queued requests while their device footprint fits the
// budget, launches the slot-wise products of the newly admitted ones, advances every active
// request's chunk programs by one power-of-two rotation in a single batched rotation level, and
// retires the requests whose programs have finished (mask products and per-partition sums).
// Requests that arrive while others run join at the next tick, so their rotations share launches.
namespace hs {
struct SrvReq {
  i64 id = 0;
  const hs_keyset* ks = nullptr;
  const hs_matrix* m = nullptr;
  const hs_ctvec* x = nullptr;
  hs_ctvec* y = nullptr;
  std::vector<std::vector<MicroOp>> progs;
  std::vector<size_t> pc;
  std::vector<int> wt_base;
  DBuf vbuf, wtbuf;
  std::vector<int> lidx;  // lazy relinearisation: slot of a one-column chunk's product, or -1
  DBuf d4;                // those products, [4][L][N] each
  size_t footprint = 0;
  bool held = false;      // left in the queue by a tick's admission at least once
  double t_submit = 0, t_admit = 0, t_done = 0;
  int status = 0;  // 0 queued, 1 active, 2 done, <0 error code
  std::string err;
};
}  // namespace hs

struct hs_server {
  hs_ctx* ctx = nullptr;
  hipStream_t st = nullptr;
  size_t budget = 0, used = 0;
  int max_active = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<hs::SrvReq>> queue;
  std::vector<std::shared_ptr<hs::SrvReq>> active;
  std::unordered_map<hs::i64, std::shared_ptr<hs::SrvReq>> all;
  hs::i64 next_id = 1;
  bool stop = false;
  std::thread worker;
  std::chrono::steady_clock::time_point t0;
  hs::i64 ticks = 0, max_conc = 0, admitted = 0, completed = 0;
  hs::i64 held_budget = 0, held_slots = 0, waited = 0;  // ticks that left requests queued (budget / max_active); requests held
  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
};

namespace hs {
static size_t request_footprint(const hs_ctx* c, const hs_matrix* m, int* nwt_out) {
  const size_t CW = ct_words(c) * sizeof(u64);
  int nwt = 0;
  for (const hs_chunk& ch : m->chunks)
    if (ch.c > 1) nwt += 4;
  if (nwt_out) *nwt_out = nwt;
  size_t lazy = 0;  // unrelinearised products (two ciphertexts' worth each) and LA, Y2 per group
  for (int g = 0; g < (int)m->chunks.size(); g++) lazy += lazy_chunk(c, m, g) ? 2 : 0;
  if (lazy) lazy += 2 * m->groups.size();
  size_t tensor = 0;  // the exact products of an encrypted matrix: the scratch of its admission tick
  if (m->encrypted) {
    const size_t per = (size_t)(8 * c->L + 7 * c->n_mod) * c->N * sizeof(u64);
    tensor = m->chunks.size() * per * (lds_limb_fits(c) ? 1 : 2);  // two-pass transforms: as much again
  }
  return ((size_t)m->chunks.size() + nwt + m->groups.size() + lazy) * CW + tensor;
}

static void server_tick(hs_server* S) {
  hs_ctx* c = S->ctx;
  const size_t CW = ct_words(c);
  std::vector<std::shared_ptr<SrvReq>> fresh;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    int held = 0;  // 1: the budget, 2: max_active left requests in the queue
    while (!S->queue.empty()) {
      if ((int)S->active.size() >= S->max_active) { held = 2; break; }
      auto& r = S->queue.front();
      if (!S->active.empty() && S->used + r->footprint > S->budget) { held = 1; break; }  // admission by footprint
      S->used += r->footprint;
      r->status = 1;
      r->t_admit = S->now();
      S->active.push_back(r);
      fresh.push_back(r);
      S->queue.pop_front();
      S->admitted++;
    }
    if (held) {
      (held == 1 ? S->held_budget : S->held_slots)++;
      for (auto& q : S->queue)
        if (!q->held) { q->held = true; S->waited++; }
    }
    S->max_conc = std::max<i64>(S->max_conc, (i64)S->active.size());
  }
  // set up and launch the products of the newly admitted requests
  std::vector<const u64*> pa, pb, rk;
  std::vector<u64*> po, lz;
  for (auto& r : fresh) {
    const hs_matrix* m = r->m;
    const int G = (int)m->chunks.size();
    r->progs.resize(G);
    r->pc.assign(G, 0);
    r->wt_base.assign(G, -1);
    int nwt = 0;
    for (int g = 0; g < G; g++) {
      r->progs[g] = total_sum_program(c, r->ks, m->chunks[g].h, m->chunks[g].c, nullptr);
      if (r->progs[g].size() > 1) { r->wt_base[g] = nwt; nwt += 4; }
    }
    r->vbuf = DBuf(&c->pool, (size_t)std::max(G, 1) * CW * sizeof(u64));
    r->wtbuf = DBuf(&c->pool, (size_t)std::max(nwt, 1) * CW * sizeof(u64));
    r->y = new_ctvec(c, (i64)m->groups.size());
    if (!G) continue;
    if (m->ready) HS_CHECK_HIP(hipStreamWaitEvent(S->st, m->ready, 0));
    if (m->encrypted) {
      r->lidx.assign(G, -1);
      int nl = 0;
      for (int g = 0; g < G; g++)
        if (lazy_chunk(c, m, g)) r->lidx[g] = nl++;
      if (nl) r->d4 = DBuf(&c->pool, (size_t)nl * 2 * CW * sizeof(u64));
      for (int g = 0; g < G; g++) {
        pa.push_back(m->d_pt + (size_t)g * CW);
        pb.push_back(r->x->d + (size_t)g * CW);
        po.push_back(r->vbuf.as<u64>() + (size_t)g * CW);
        rk.push_back(r->ks->rk);
        lz.push_back(r->lidx[g] >= 0 ? r->d4.as<u64>() + (size_t)r->lidx[g] * 2 * CW : nullptr);
      }
    } else {
      launch_mul_plain(c, r->x->d, m->d_pt, r->vbuf.as<u64>(), G, c->L, S->st);
    }
  }
  if (!pa.empty()) mul_ct_batch(c, (int)pa.size(), pa.data(), pb.data(), po.data(), rk.data(), S->st, lz.data());
  // rotation levels across every active request: one when requests wait for admission, else as
  // many as every active request still has (at most 4), enqueued without host waits in between, so
  // no request finishes in the middle of a tick and admission stays responsive
  auto buf = [&](SrvReq* r, int g, int id) -> u64* {
    return id == 0 ? r->vbuf.as<u64>() + (size_t)g * CW : r->wtbuf.as<u64>() + (size_t)(r->wt_base[g] + id - 1) * CW;
  };
  int nlev = 1;
  bool waiting;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    waiting = !S->queue.empty();
  }
  if (!waiting) {
    int minrem = 0;
    for (auto& r : S->active) {
      int rem = 0;
      for (size_t g = 0; g < r->progs.size(); g++) rem = std::max(rem, (int)r->progs[g].size() - 1 - (int)r->pc[g]);
      if (rem > 0) minrem = minrem == 0 ? rem : std::min(minrem, rem);
    }
    nlev = std::max(1, std::min(minrem, 4));
  }
  std::vector<std::vector<RotItem>> levels(nlev);
  for (int lv = 0; lv < nlev; lv++)
    for (auto& r : S->active)
      for (size_t g = 0; g < r->progs.size(); g++) {
        auto& prog = r->progs[g];
        if ((size_t)r->pc[g] + 1 >= prog.size()) continue;
        const MicroOp& op = prog[r->pc[g]++];
        RotItem it{};
        it.in = buf(r.get(), (int)g, op.in);
        it.out = buf(r.get(), (int)g, op.out);
        it.addend = op.addend >= 0 ? buf(r.get(), (int)g, op.addend) : nullptr;
        it.key = rotation_key(r->ks, op.step);
        it.galois = (u32)galois_step(c, op.step);
        levels[lv].push_back(it);
      }
  while (!levels.empty() && levels.back().empty()) levels.pop_back();
  if (!levels.empty()) run_rotation_levels(c, levels, S->st);
  // retire finished requests
  std::vector<std::shared_ptr<SrvReq>> done;
  std::vector<DBuf> keep;
  std::vector<RotItem> relin_items;  // lazy relinearisation (see BatchWork): one per group
  std::vector<std::pair<u64*, const u64*>> copies;
  u64* zero = nullptr;
  for (auto& r : S->active) {
    bool fin = true;
    for (size_t g = 0; g < r->progs.size(); g++) fin &= (r->pc[g] + 1 >= r->progs[g].size());
    if (!fin) continue;
    const hs_matrix* m = r->m;
    const int G = (int)m->chunks.size(), nP = (int)m->groups.size();
    if (nP) {
      const bool lazy = r->d4.p != nullptr;
      auto lz_at = [&](int g) { return r->d4.as<u64>() + (size_t)r->lidx[g] * 2 * CW; };
      if (lazy && !zero) {
        keep.emplace_back(&c->pool, CW * sizeof(u64));
        zero = keep.back().as<u64>();
        HS_CHECK_HIP(hipMemsetAsync(zero, 0, CW * sizeof(u64), S->st));
      }
      std::vector<const u64*> wp(std::max(G, 1), nullptr), wa(std::max(G, 1), nullptr);
      for (int g = 0; g < G; g++) {
        const bool lg = lazy && r->lidx[g] >= 0;
        wp[g] = lg ? lz_at(g) + CW : buf(r.get(), g, r->progs[g].back().in);
        wa[g] = lg ? lz_at(g) : zero;
      }
      std::vector<int> pc0(nP), pnc(nP);
      for (int p = 0; p < nP; p++) { pc0[p] = m->groups[p].chunk0; pnc[p] = m->groups[p].nchunks; }
      keep.emplace_back(&c->pool, 2 * wp.size() * sizeof(u64*));
      const u64* const* dw = keep.back().as<const u64*>();
      h2d(keep.back().as<const u64*>(), wp.data(), wp.size(), S->st);
      h2d(keep.back().as<const u64*>() + wp.size(), wa.data(), wa.size(), S->st);
      keep.emplace_back(&c->pool, nP * sizeof(int));
      int* dpc0 = keep.back().as<int>();
      h2d(dpc0, pc0.data(), nP, S->st);
      keep.emplace_back(&c->pool, nP * sizeof(int));
      int* dpnc = keep.back().as<int>();
      h2d(dpnc, pnc.data(), nP, S->st);
      const u64* mask = c->prm.agg_mode == 0 ? m->d_mask : nullptr;
      if (!lazy) {
        launch_mask_acc(c, dw, mask, dpc0, dpnc, r->y->d, nP, S->st);
      } else {
        keep.emplace_back(&c->pool, (size_t)nP * 2 * CW * sizeof(u64));
        u64* LA = keep.back().as<u64>();
        u64* Y2 = LA + (size_t)nP * CW;
        launch_mask_acc(c, dw, mask, dpc0, dpnc, Y2, nP, S->st);
        launch_mask_acc(c, dw + wp.size(), mask, dpc0, dpnc, LA, nP, S->st);
        for (int p = 0; p < nP; p++) {
          const hs_group& Gr = m->groups[p];
          bool has = false;
          for (int g = Gr.chunk0; g < Gr.chunk0 + Gr.nchunks; g++) has |= r->lidx[g] >= 0;
          if (!has) { copies.emplace_back(r->y->d + (size_t)p * CW, Y2 + (size_t)p * CW); continue; }
          RotItem it{};
          it.in = LA + (size_t)p * CW;
          it.addend = Y2 + (size_t)p * CW;
          it.out = r->y->d + (size_t)p * CW;
          it.key = r->ks->rk;
          it.galois = 1;
          relin_items.push_back(it);
        }
      }
    }
    done.push_back(r);
  }
  if (!relin_items.empty()) {
    run_rotation_levels(c, {relin_items}, S->st);
    g_counters[0] -= (int64_t)relin_items.size();   // relinearisations are not rotations
  }
  copy_pairs(copies, CW, S->st);
  HS_CHECK_HIP(hipStreamSynchronize(S->st));
  const double t = S->now();
  std::lock_guard<std::mutex> lk(S->mu);
  for (auto& r : done) {
    r->vbuf.reset();
    r->wtbuf.reset();
    r->d4.reset();
    r->t_done = t;
    r->status = 2;
    S->used -= r->footprint;
    S->completed++;
    S->active.erase(std::find(S->active.begin(), S->active.end(), r));
  }
  S->ticks++;
  if (!done.empty()) S->cv_done.notify_all();
}

static void server_loop(hs_server* S) {
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty() || !S->active.empty(); });
      if (S->stop && S->queue.empty() && S->active.empty()) return;
    }
    try {
      server_tick(S);
    } catch (const Error& e) {
      std::lock_guard<std::mutex> lk(S->mu);
      for (auto& r : S->active) { r->status = e.code; r->err = e.msg; S->used -= r->footprint; }
      for (auto& r : S->queue) { r->status = e.code; r->err = e.msg; }
      S->active.clear();
      S->queue.clear();
      S->cv_done.notify_all();
    }
  }
}
}  // namespace hs

extern "C" {

int hs_server_create(hs_ctx* c, int64_t hbm_budget_bytes, int max_active, void* stream, hs_server** out) {
  return guarded([&] {
    HS_REQUIRE(c && out && hbm_budget_bytes > 0 && max_active > 0, HS_EINVAL, "bad argument");
    *out = nullptr;
    hs_server* srv = new hs_server();
    srv->ctx = c;
    srv->st = (hipStream_t)stream;
    srv->budget = (size_t)hbm_budget_bytes;
    srv->max_active = max_active;
    srv->t0 = std::chrono::steady_clock::now();
    srv->worker = std::thread([srv] {
      (void)hipSetDevice(srv->ctx->device);
      server_loop(srv);
    });
    *out = srv;
  });
}

int hs_server_submit(hs_server* S, const hs_keyset* ks, const hs_matrix* m, const hs_ctvec* x, int64_t* id) {
  return guarded([&] {
    HS_REQUIRE(S && ks && m && x && id, HS_EINVAL, "null argument");
    HS_REQUIRE(ks->ctx == S->ctx && m->ctx == S->ctx && x->ctx == S->ctx, HS_EKEY, "handles from another context");
    HS_REQUIRE(x->n == (i64)m->chunks.size(), HS_EINVAL, "the vector must hold one ciphertext per chunk");
    auto r = std::make_shared<SrvReq>();
    r->ks = ks; r->m = m; r->x = x;
    r->footprint = request_footprint(S->ctx, m, nullptr);
    std::lock_guard<std::mutex> lk(S->mu);
    HS_REQUIRE(!S->stop, HS_EINVAL, "server is shutting down");
    r->id = S->next_id++;
    r->t_submit = S->now();
    S->queue.push_back(r);
    S->all[r->id] = r;
    *id = r->id;
    S->cv_work.notify_one();
  });
}

int hs_server_wait(hs_server* S, int64_t id, hs_ctvec** y, double times[3]) {
  return guarded([&] {
    HS_REQUIRE(S && y, HS_EINVAL, "null argument");
    *y = nullptr;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(id);
    HS_REQUIRE(it != S->all.end(), HS_EINVAL, "unknown request id");
    auto r = it->second;
    S->cv_done.wait(lk, [&] { return r->status == 2 || r->status < 0; });
    S->all.erase(it);
    if (r->status < 0) {
      if (r->y) hs_ctvec_destroy(r->y);
      throw Error{r->status, r->err};
    }
    *y = r->y;
    if (times) { times[0] = r->t_submit; times[1] = r->t_admit; times[2] = r->t_done; }
  });
}

int hs_server_stats(hs_server* S, int64_t out[8], double* now) {
  return guarded([&] {
    HS_REQUIRE(S && out, HS_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    out[0] = S->ticks; out[1] = S->max_conc; out[2] = S->admitted; out[3] = S->completed; out[4] = (int64_t)S->used;
    out[5] = S->held_budget; out[6] = S->held_slots; out[7] = S->waited;
    if (now) *now = S->now();
  });
}

void hs_server_destroy(hs_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->cv_work.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  for (auto& kv : S->all)
    if (kv.second->y) hs_ctvec_destroy(kv.second->y);
  delete S;
}

}  // extern "C"
