// Kernel argument structures and host launchers of the encrypted-SpMV library.
#pragma once
#include <string>

#include "hs_internal.hpp"

namespace hs {

// One power-of-two rotation of a batched key switch.
struct RotItem {
  const u64* in;      // ciphertext [2][L][N] (NTT form)
  u64* out;           // result [2][L][N]; must not alias `in`
  const u64* addend;  // optional ciphertext added to the result (may alias `out`), else nullptr
  const u64* key;     // key-switching key [2][dnum][L+K][N] for sigma_g(s) -> s
  u32 galois;         // Galois element g
  u32 next;           // two-pass levels: 1 + index, in the next level, of the item whose input is
                      // this item's output and whose first key-switch step (Galois gather +
                      // inverse low pass of c1) this item's last kernel performs; 0 = none
};

struct KsShape {
  int L, K, alpha, dnum;
  int ndg;   // digit groups (one partial accumulator each)
  int dpg;   // digits per group
};

struct KskArgs {
  u64* b; u64* a;            // outputs [N]
  const int* e_coef;         // Gaussian coefficients [N]
  const u64* sk;             // secret key limb (NTT form) of this modulus
  int mod_index;
  u64 seed; u32 purpose_a; u64 idx_a;
  int sprime_mode; u32 galois; double2 pfac;  // s' mode: 0 none, 1 sigma_g(s), 2 s^2; pfac = P mod q or 0
  double2 r64;               // 2^64 mod q as (w, w/q)
};

struct PackArgs {
  const i64* va; const int* ci; const i64* v;
  const i64* cp;             // CSSC column pointers of the whole matrix
  const i64* chunk;          // per chunk 8 words: (start, c, h, cp_off, nnz_off, part, 0, 0)
  u64* out;                  // [nchunks][N] coefficients mod t
  int mode;                  // 0 matrix values, 1 reorganised vector, 2 mask,
                             // 3 matrix values for plaintexts g < nG, mask of chunk g - nG after
  int nG;                    // chunks (mode 3)
};

// Constants of the exact ciphertext product (tensor.hip); device pointers.
struct TensorConst {
  const double2* qhat_inv;  // [L]  (Q/q_i)^-1 mod q_i
  const u64* qhat;          // [L][WQ] Q/q_i
  const u64* Q;             // [WQ]
  const u64* halfQ;         // [WQ] floor(Q/2)
  int WQ;
  const double2* mhat_inv;  // [T]  (M/m)^-1 mod m
  const u64* mhat;          // [T][WM] M/m
  const u64* M;             // [WM + 1]
  const u64* halfM;         // [WM] floor(M/2)
  int WM;
  const u64* D;             // [WD] 2Q
  int WD;
  const u64* mu;            // [WMU + 1] floor(2^(64 kw) / 2Q)
  int WMU, WA;
  const double2* r32;       // [T] 2^32 mod m
  int T, L;
  u64 t;
  int kw;                   // word capacity of the kernels (8, 16 or 24); mu = floor(2^(64 kw) / 2Q)
};

// HIP-event timing of kernel launches (profiler.cpp)
class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t st);
  ~ProfScope();
 private:
  const char* name_;
  hipStream_t st_;
  hipEvent_t a_ = nullptr;
  bool active_ = false;
};
// The launches the calling thread makes while it lives process `n` units of work each (key
// switches of a rotation level), summed per kernel in the profile summary.
class ProfUnits {
 public:
  explicit ProfUnits(long n);
  ~ProfUnits();
 private:
  long prev_;
};
void profile_enable(bool on);
void profile_capturing(bool on);  // calling thread is recording a graph: no timing events
std::string profile_summary();

void upload_cdt(const u64* tab20);
// fixed scratch region of the allocation-free entry point on the current device (noalloc.hip)
int noalloc_scratch(void** ptr, size_t* bytes);
void launch_fill_u64(u64* p, size_t n, u64 v, hipStream_t st);
// Where each row (limb) of a batched N = 2^15 transform is read and written: mode 0 in place at
// data + r N; mode 1 (gather) row r of item i = r / per reads limb q = r % per of opA[i] (q < split)
// or limb q - split of opB[i] and writes data + r N; mode 2 (scatter) reads data + r N and writes
// limb q of out[i] when out[i] is set, else in place.  At most kNttRowItems items per launch.
static constexpr int kNttRowItems = 32;
struct NttRows {
  int mode = 0, per = 0, split = 0;
  const u64* opA[kNttRowItems] = {};
  const u64* opB[kNttRowItems] = {};
  u64* out[kNttRowItems] = {};
};
void launch_ntt15_rows(const hs_ctx* c, u64* data, i64 nblocks, int nl, int mod0, int inverse, const NttRows& rows, hipStream_t st);
// n device-to-device copies of words[j] u64 words (src[j] -> dst[j]; host arrays of device
// pointers), batched into launches of up to 32 (one launch instead of one copy call each)
void launch_copy_batch(const u64* const* src, u64* const* dst, const size_t* words, int n, hipStream_t st);
void launch_ntt(const hs_ctx* c, u64* data, i64 nblocks, int nl, int mod0, int inverse, hipStream_t st);
void launch_sample_small(const hs_ctx* c, int* out, int nobj, i64 obj_stride, u64 seed, u32 purpose, u64 index0, u64 index_step,
                         int kind, hipStream_t st);
void launch_sk_ntt(const hs_ctx* c, u64* sk, const int* s_coef, hipStream_t st);
void launch_ksk_limbs(const hs_ctx* c, const KskArgs* d_args, int count, hipStream_t st);
void launch_pack_encode(const hs_ctx* c, const PackArgs& a, int nchunks, hipStream_t st);
void launch_plain_ntt(const hs_ctx* c, const u64* coef, u64* out, int n_plain, hipStream_t st);
void launch_encrypt(const hs_ctx* c, const u64* mcoef, const int* samples, const u64* pk, u64* out, int n_ct, hipStream_t st);
void launch_mul_plain(const hs_ctx* c, const u64* x, const u64* pt, u64* out, i64 n_ct, int pt_stride_ct, hipStream_t st);
void launch_mask_acc(const hs_ctx* c, const u64* const* w, const u64* mask, const int* part_chunk0, const int* part_nchunks,
                     u64* res, int nparts, hipStream_t st);
void launch_rotate_batch(const hs_ctx* c, const RotItem* d_items, int B, const KsShape& S, u64* D, double* ACC, double* PC, hipStream_t st);
// two-pass (multi-workgroup) transforms and key switching (ks2.hip)
void launch_ntt2(const hs_ctx* c, u64* data, double* scratch, i64 rows, int nl, int mod0, int inverse, hipStream_t st);
// Items [0, B1) get the first step (K1) here; the others had it from the previous level's last
// kernel.  d_next: the next level's items when some items here have `next` set, else nullptr.
void launch_rotate_batch2(const hs_ctx* c, const RotItem* d_items, int B, const KsShape& S, double* T1, double* E, double* ACC, double* T2,
                          double* F, hipStream_t st, int B1 = -1, const RotItem* d_next = nullptr);

// split path (aux2.hip): elementwise prologues / epilogues around batched transforms
void launch_ints_to_limbs(const hs_ctx* c, const int* src, i64 src_stride, int nobj, u64* out, int nl, int mod0, hipStream_t st);
void launch_ksk_combine(const hs_ctx* c, const KskArgs* d_args, const u64* e_ntt, int count, hipStream_t st);
void launch_pack_slots(const hs_ctx* c, const PackArgs& a, int nchunks, hipStream_t st);
void launch_lift_plain(const hs_ctx* c, const u64* coef, int n_plain, u64* out, hipStream_t st);
void launch_enc_prep(const hs_ctx* c, const u64* mcoef, const int* samples, int n_ct, u64* out, hipStream_t st);
void launch_enc_combine(const hs_ctx* c, const u64* prep, const u64* pk, u64* out, int n_ct, hipStream_t st);
void launch_dec_prep(const hs_ctx* c, const u64* ct, const u64* sk, u64* X, int n_ct, hipStream_t st);
void launch_slots_scatter(const hs_ctx* c, const u64* Mntt, const int* rm, const i64* pinfo, int nparts, i64* y, hipStream_t st);
// exact ciphertext product (tensor.hip)
void launch_crt_lift(const hs_ctx* c, const TensorConst& C, const u64* x, u64* out, int rows, hipStream_t st);
void launch_tensor(const hs_ctx* c, const u64* lift, u64* prod, int items, int T, hipStream_t st);
void launch_scale_round(const hs_ctx* c, const TensorConst& C, const u64* prod, u64* out, int items, hipStream_t st);

void launch_dec_phase(const hs_ctx* c, const u64* ct, const u64* sk, u64* X, int n_ct, hipStream_t st);
void launch_dec_round(const hs_ctx* c, const u64* X, u64* M, int n_ct, hipStream_t st);
void launch_decode_scatter(const hs_ctx* c, const u64* M, const int* rm, const i64* pinfo, i64* y, int nparts, hipStream_t st);
void launch_cssc_scatter(const i64* row_ptr, const int* col, const i64* val, const int* rank, const i64* cp, const i64* part_cp_off,
                         const i64* part_nnz_off, i64 R, i64 s, i64* va, int* ci, hipStream_t st);
void launch_csr_check(const i64* row_ptr, const int* col, i64 R, i64 C, int* bad, hipStream_t st);
// CSR -> CSSC structure on the device (cssc.hip)
void launch_csr_rows(const i64* row_ptr, i64 R, i64 s, int* cnt, unsigned long long* stat, hipStream_t st);
int cssc_sort_block(i64 s);
void launch_cssc_one_pass(const i64* row_ptr, i64 R, i64 s, int* dig, int* bh, int* bflag, i64* hdr, i64* cp, int* rm, int* rank,
                          hipStream_t st);
const u32* launch_cssc_order(const int* cnt, const unsigned long long* stat, i64 R, i64 s, int passes, u32* keyA, u32* keyB, int* idxA,
                             int* idxB, int* bh, int* rm, int* rank, hipStream_t st);
void launch_cssc_cp(const u32* key_sorted, const unsigned long long* stat, i64 R, i64 s, const i64* cp_off, const i64* cp_len, i64* cp,
                    hipStream_t st);

}  // namespace hs
