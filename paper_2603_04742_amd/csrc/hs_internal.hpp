// Internal host-side structures of the encrypted-SpMV library (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/hespmv.h"

namespace hs {

typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;
typedef int32_t i32;
typedef unsigned __int128 u128;

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
struct Error {
  int code;
  std::string msg;
};
#define HS_CHECK_HIP(expr)                                                              \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      throw ::hs::Error{HS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)}; \
  } while (0)
#define HS_REQUIRE(cond, code, msg) \
  do {                              \
    if (!(cond)) throw ::hs::Error{code, msg}; \
  } while (0)

// ------------------------------------------------------------------ per-modulus device constants
struct ModTab {
  double q, qinv;        // modulus and fl(1/q)
  double2 ninv;          // (N^-1 mod q, quotient)
  const double2* fw;     // forward twiddles (psi^bitrev(i), fl(./q))
  const double2* iv;     // inverse twiddles (psi^-bitrev(i), fl(./q))
  const double* fwc;     // forward twiddles psi^bitrev(i) alone, 8 bytes each (ct_group_c)
};

// pair (w, fl(w/q)) for a constant w in [0, q)
inline double2 make_const(u64 w, u64 q) { return double2{(double)w, (double)w / (double)q}; }

// Source of the device buffers of one call: the context's pool, or a fixed region (Arena).
class Alloc {
 public:
  virtual void* get(size_t bytes) = 0;
  virtual void put(void* p) = 0;

 protected:
  ~Alloc() = default;
};

// Device memory pool: size-bucketed free lists so that steady-state calls do not hipMalloc.
class Pool : public Alloc {
 public:
  void* get(size_t bytes) override;
  void put(void* p) override;
  void release_all();
  ~Pool() { release_all(); }

 private:
  std::mutex mu_;
  std::multimap<size_t, void*> free_;
  std::map<void*, size_t> size_of_;
};

// Slices of a device region that the caller owns, handed out in order (256-byte aligned) and
// never returned: the buffers of one call of the allocation-free entry point.  get() past the end
// throws HS_ENOMEM naming the size needed; put() does nothing.
class Arena : public Alloc {
 public:
  Arena(void* base, size_t cap) : base_((char*)base), cap_(cap) {}
  void* get(size_t bytes) override;
  void put(void*) override {}
  size_t used() const { return used_; }

 private:
  char* base_;
  size_t cap_, used_ = 0;
};

// RAII device buffer from a pool or an arena
struct DBuf {
  Alloc* pool = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() {}
  DBuf(Alloc* pl, size_t b) : pool(pl), p(b ? pl->get(b) : nullptr), bytes(b) {}
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept { *this = std::move(o); }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      reset();
      pool = o.pool; p = o.p; bytes = o.bytes;
      o.p = nullptr; o.bytes = 0;
    }
    return *this;
  }
  void reset() {
    if (p && pool) pool->put(p);
    p = nullptr; bytes = 0;
  }
  ~DBuf() { reset(); }
  template <class T> T* as() const { return (T*)p; }
};

}  // namespace hs

// ------------------------------------------------------------------ opaque handle definitions
struct hs_ctx {
  hs_params prm;
  int logn = 0;
  hs::u64 N = 0, t = 0;
  int L = 0, K = 0, alpha = 0, dnum = 0, n_aux = 0, n_mod = 0;
  int device = 0;
  std::vector<hs::u64> mod;        // [L data][K special][n_aux tensor] ; index n_mod = t (host copy only)
  std::vector<hs::u64> psi;        // smallest primitive 2N-th root per modulus (+ t last)
  hs::ModTab* d_tab = nullptr;     // device [n_mod + 1], entry n_mod = plaintext modulus t
  std::vector<hs::ModTab> h_tab;
  double2* d_tw = nullptr;         // twiddle storage
  double* d_twc = nullptr;         // forward twiddles without quotients
  hs::u32* d_slot_pos = nullptr;   // slot j -> index of the mod-t NTT output
  // encryption: floor(Q/t) mod q_i as (w, w/q), Q mod t
  double2* d_qdt = nullptr;
  hs::u64 q_mod_t = 0;
  // key switching: P mod q_i, P^-1 mod q_i (data primes)
  double2* d_pmod = nullptr;
  double2* d_pinv = nullptr;
  // ModUp basis conversion, digit j with source primes D_j (alpha of them):
  //   d_up_inv[j*alpha + a]             = (Q_j/q_a)^-1 mod q_a
  //   d_up_hat[(j*alpha + a)*(L+K) + m] = (Q_j/q_a) mod mod[m]
  double2* d_up_inv = nullptr;
  double2* d_up_hat = nullptr;
  // ModDown conversion from the K special primes to data prime i
  double2* d_dn_inv = nullptr;     // [K]   (P/p_k)^-1 mod p_k
  double2* d_dn_hat = nullptr;     // [K*L] (P/p_k) mod q_i
  // decryption: Q-hat_i^-1 mod q_i, Q-hat_i as little-endian 64-bit words, Q, 2Q
  int dec_words = 0;
  double2* d_dec_inv = nullptr;
  hs::u64* d_dec_hat = nullptr;    // [L][dec_words]
  hs::u64* d_dec_q = nullptr;      // [dec_words] Q
  // exact ciphertext product over the tensor basis (all n_mod moduli)
  bool has_tensor = false;
  int tq_words = 0, tm_words = 0, td_words = 0, tmu_words = 0, ta_words = 0, t_kw = 0;
  hs::u64* d_t_halfq = nullptr;
  double2* d_t_mhat_inv = nullptr;
  hs::u64* d_t_mhat = nullptr;
  hs::u64* d_t_m = nullptr;
  hs::u64* d_t_halfm = nullptr;
  hs::u64* d_t_d = nullptr;
  hs::u64* d_t_mu = nullptr;
  double2* d_t_r32 = nullptr;
  hs::Pool pool;
  // stream of the matrix plaintext encoding, which runs after hs_cssc_pack returns (default
  // priority, non-blocking); each matrix records an event on it when its plaintexts are ready
  hipStream_t side = nullptr;
  // launch choices set by hs_autotune (results do not depend on them):
  //   xf_variant 0: compile-time / half-limb transforms, 1: runtime radix-8 / whole-limb, for the
  //   key-switch kernels; xf_variant_ntt the same for the plain transform kernels (NTT, plaintext
  //   encoding, decryption phase);
  //   ks_pick[b]: key-switch pipeline for levels of 2^(b-1) < B <= 2^b items (b = 7: larger),
  //   1 two-pass, 0 one workgroup per limb, -1 the fixed threshold rule.
  int xf_variant = 0;
  int xf_variant_ntt = 0;
  signed char ks_pick[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
  // execution options of this context (hs_ctx_set_option), by HS_OPT_* key; -1 = the process-wide
  // default (hs_set_option)
  int opt[10] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
  // events of the asynchronous calls still in flight (see note_async), guarded by async_mu
  std::mutex async_mu;
  std::vector<hipEvent_t> async_ev;
  // device address and size of the fixed scratch array on this context's device (allocation-free
  // entry point), looked up when the context is created
  void* na_scratch = nullptr;
  size_t na_bytes = 0;
};

struct hs_keyset {
  hs_ctx* ctx = nullptr;
  hs::u64 seed = 0;
  hs::u64* sk = nullptr;        // [n_mod][N] NTT form, canonical
  hs::u64* pk = nullptr;        // [2][L][N]
  std::vector<hs::u64*> gk;     // rotation keys [2][dnum][L+K][N]: left by 2^i at i < log2 N - 1, then the optional right ones
  std::map<hs::i64, hs::u64*> step_keys;  // exact-step rotation keys by step k, same layout
  hs::u64* rk = nullptr;        // relinearisation key, same layout
  size_t ksk_words = 0;
};

struct hs_chunk {
  int part;        // group (result ciphertext): a row partition, or a pair with two slot rows
  int start, c;    // first CSSC column, number of columns
  hs::i64 h;       // height (rows); slot k <-> (block k / h, sorted row k % h)
};

struct hs_part {
  hs::i64 row0, rows;   // original rows [row0, row0 + rows)
  int Lw;               // CSSC columns (max nonzeros in a row)
  hs::i64 nnz_off;      // offset of this partition's VA/CI in the matrix arrays
  hs::i64 cp_off;       // offset of this partition's CP in the matrix CP array
  hs::i64 nz_rows;      // rows with at least one nonzero (= NNZ of CSSC column 0)
};

// One result ciphertext: partition pa in slot row 0 and, with two slot rows, partition pb (or -1)
// in slot row 1; its chunks are chunks[chunk0, chunk0 + nchunks).
struct hs_group {
  int pa, pb;
  int chunk0, nchunks;
};

struct hs_matrix {
  hs_ctx* ctx = nullptr;
  hs::i64 R = 0, C = 0, nnz = 0;
  int encrypted = 0;
  std::vector<hs_part> parts;
  std::vector<hs_group> groups;
  std::vector<hs_chunk> chunks;
  std::vector<hs::i64> h_cp;     // all partitions' CP arrays, concatenated (a copy of d_cp)
  char* d_struct = nullptr;      // one allocation: d_cp, d_rm
  char* d_meta = nullptr;        // one allocation: d_chunk, d_pinfo
  hs::i64* d_cp = nullptr;
  hs::i32* d_rm = nullptr;
  hs::i64* d_pinfo = nullptr;    // per partition: (row0, rows, nonzero rows, row-map offset, group, slot offset)
  hs::i64* d_va = nullptr;       // CSSC values (nnz)
  hs::i32* d_ci = nullptr;       // CSSC column indices (nnz)
  hs::i64* d_chunk = nullptr;    // per chunk: (start, c, h, cp_off) for device kernels
  hs::u64* d_pt = nullptr;       // per chunk: plaintext [L][N] or ciphertext [2][L][N]
  hs::u64* d_mask = nullptr;     // per chunk: mask plaintext [L][N] (paper aggregation)
  bool mask_in_pt = false;       // d_mask points into the d_pt allocation
  hs::u64* d_coef = nullptr;     // mod-t coefficients of the deferred encoding (kept until destroy)
  hipEvent_t ready = nullptr;    // recorded on the context's side stream when d_pt/d_mask are final
};

// The diagonal method (the paper's baseline): square blocks of side B; per block its non-empty
// generalised diagonals, each one NTT-form plaintext, sorted by (block row, block column, d).
struct hs_diag {
  hs_ctx* ctx = nullptr;
  hs::i64 R = 0, C = 0, B = 0;
  int nrb = 0, ncb = 0;              // block rows, block columns
  std::vector<hs::i64> key;          // per diagonal: (bi, bj, d)
  std::vector<int> row0, rown;       // per block row: first diagonal, number of diagonals
  char* d_struct = nullptr;          // identity row map [B] (i32) | per block row 6-word scatter info
  hs::i32* d_rm = nullptr;
  hs::i64* d_pinfo = nullptr;
  hs::u64* d_pt = nullptr;           // [n diagonals][L][N]
};

struct hs_ctvec {
  hs_ctx* ctx = nullptr;
  hs::i64 n = 0;                 // ciphertexts
  hs::u64* d = nullptr;          // [n][2][L][N] NTT form, canonical
  bool owned = true;
};

namespace hs {
// host math (params.cpp)
bool is_prime_u64(u64 n);
std::vector<u64> primes_1_mod_2n(u64 N, int bits, int count);
u64 smallest_root_2n(u64 q, u64 N);
u64 pow_mod(u64 b, u64 e, u64 m);
u64 mul_mod(u64 a, u64 b, u64 m);
u64 inv_mod(u64 a, u64 q);
void build_ctx(hs_ctx* c);
// value of execution option `key` (HS_OPT_*) for context c: its own setting, else the process-wide one
int option(const hs_ctx* c, int key);
void free_ctx(hs_ctx* c);
size_t ct_words(const hs_ctx* c);
}  // namespace hs
