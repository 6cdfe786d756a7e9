/*
 * hespmv.h -- C ABI of an MI355X (gfx950) library for encrypted sparse matrix-vector
 * multiplication over the Compressed Sparse Sorted Column (CSSC) format, arXiv 2603.04742.
 *
 * The calls follow the paper's three-party protocol (Sec. 3.2; Sec. 4.4, Alg. "Sparse
 * Matrix-Vector Multiplication"):
 *   Client A   hs_cssc_pack        CSR -> CSSC (App. B), row partitions (Sec. 4.7), chunks
 *                                  (Alg. generateChunk), slot packing and encoding/encryption
 *              hs_matrix_column_index   the plaintext column-index array sent to Client B
 *   Client B   hs_encrypt          reorganised vector (Alg. reorgVector), encoded and encrypted
 *   Cloud      hs_he_spmv          slot-wise products (HE-CMult, or HE-Mult when the matrix values
 *                                  are encrypted) and Alg. Aggregation (totalSum rotations, masks)
 *   Key holder hs_decrypt          decryption and the row-map scatter
 * plus hs_keygen (secret, public, power-of-two rotation and relinearisation keys).
 *
 * Scheme: BFV-style RLWE over Z_q[X]/(X^N + 1), RNS with L data primes and K special primes (all
 * NTT-friendly, < 2^50), plaintext modulus t prime with t = 1 mod 2N, ternary secret, discrete
 * Gaussian errors (sigma 3.2).  Conventions (prime choice, slot order, NTT order, sampling, key
 * switching, ct x ct) are pinned so that every ciphertext limb is reproducible bit for bit.
 *
 * Conventions of the ABI:
 *  - Every function returns HS_OK (0) or a negative HS_E* code; hs_last_error() then returns a
 *    thread-local message.  On error no output handle is created.
 *  - Handles are opaque and library-owned; each has a matching *_destroy.  Device memory held by a
 *    handle is allocated on the device that was current at hs_ctx_create.
 *  - Pointers documented as "device" are HBM addresses on that device (e.g. torch tensor
 *    data_ptr()); "host" pointers are ordinary CPU memory.  Input arrays are read during the call
 *    (device inputs: in stream order) and not retained.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued on it; calls that
 *    return host data synchronise it.  Two calls that share no output handle may run on different
 *    streams concurrently; an hs_ctx and an hs_keyset are read-only after creation.
 *  - Ciphertexts are stored limb-major, [2][L][N] u64 residues in [0, q_i), NTT form, where the
 *    NTT order is A[k] = a(psi_i^(2 bitrev(k) + 1)), psi_i the smallest primitive 2N-th root of
 *    unity mod q_i.
 */
#ifndef HESPMV_H
#define HESPMV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status codes */
#define HS_OK 0
#define HS_EINVAL (-1)     /* bad argument or malformed CSR (unsorted row pointers, index out of range) */
#define HS_EPARAM (-2)     /* unsupported parameters: N not a power of two in [2^3, 2^15], t prime below 2^26 with
                              t = 1 mod 2N required, not enough NTT-friendly primes, prime width above 50 bits;
                              also hs_mul_ct and encrypted matrices on a ring whose NTT-friendly primes cannot
                              form a basis above 4 N Q^2 for the exact ciphertext product */
#define HS_ECAPACITY (-3)  /* a size exceeds what the handle or parameter set can hold */
#define HS_EKEY (-4)       /* keys missing or from another context */
#define HS_ENOMEM (-5)     /* host or device allocation failed */
#define HS_EDEVICE (-6)    /* HIP runtime error (message names the call) */

/* Thread-local description of the last error of a failed call on this thread. */
const char* hs_last_error(void);

/* ---------------------------------------------------------------- parameters and context */
typedef struct hs_params {
  uint32_t log_n;    /* ring degree N = 2^log_n, 3 <= log_n <= 15 */
  uint32_t n_q;      /* L: number of data primes */
  uint32_t q_bits;   /* bit width of data and special primes (<= 50) */
  uint32_t n_p;      /* K: number of special (key-switching) primes, >= 1; also the digit size */
  uint32_t p_bits;   /* must equal q_bits */
  uint64_t t;        /* plaintext modulus, prime, t = 1 mod 2N, t < 2^26 (65537 for N <= 32768) */
  double sigma;      /* error width; only 3.2 is supported */
  uint32_t agg_mode; /* 0 = paper aggregation: chunk heights NNZ[start] and masks (Alg. Aggregation);
                        1 = uniform heights NNZ[0] in a partition and no masks (one fewer ct x pt,
                            needed when Q/t leaves too little noise room for the mask product) */
  uint32_t slot_rows; /* 0 or 1 = the paper's layout: a partition's chunks in slot row 0, row 1 zero;
                         2 = two row partitions per ciphertext: partition 2g in slot row 0 and
                             2g + 1 in slot row 1, chunks generated on the joint column heights
                             max(NNZ_2g[j], NNZ_2g+1[j]) so that one rotation schedule serves both
                             rows (a rotation turns each slot row on its own); half the chunks,
                             products and rotations for matrices of two or more partitions, one
                             result ciphertext per pair.  Decrypted results are the same. */
  uint32_t relin_mode; /* matrices with encrypted values: 0 = relinearise after every ct x ct product
                            (the paper's placement); 1 = lazy: a one-column chunk (no totalSum
                            rotation) keeps its unrelinearised product (d0, d1, d2), which is masked
                            and summed component by component, and each result ciphertext is
                            relinearised once.  Decrypted results are the same; limbs differ. */
} hs_params;

typedef struct hs_ctx hs_ctx;
typedef struct hs_keyset hs_keyset;
typedef struct hs_matrix hs_matrix;
typedef struct hs_ctvec hs_ctvec;
typedef struct hs_diag hs_diag;

/* Create a context: prime selection (the largest primes q < 2^q_bits with q = 1 mod 2N, first K
   special, next L data primes, then tensor primes for exact ct x ct), NTT tables, constants.
   Uses the current HIP device.  HS_EPARAM for unsupported parameter sets. */
int hs_ctx_create(const hs_params* params, hs_ctx** out);
void hs_ctx_destroy(hs_ctx* ctx);
/* Moduli in chain order (L data, K special, then tensor primes) into host `out` (capacity
   `cap`); *n receives the total count.  HS_ECAPACITY if cap is too small. */
int hs_ctx_moduli(const hs_ctx* ctx, uint64_t* out, int cap, int* n);
/* Word widths (64-bit words) of the exact ciphertext product's multiword values, into host
   out[7]: [tensor moduli T, Q, M (product of the T moduli), 2Q, the Barrett reciprocal of 2Q,
   2 t |X| + Q, word capacity of the kernels]; all 0 when the ring has no exact product. */
int hs_ctx_tensor_widths(const hs_ctx* ctx, int64_t out[7]);

/* The 20 thresholds of the discrete Gaussian sampler, T[k] = floor(2^63 P(|e| <= k)) for sigma = 3.2
   truncated at |e| <= 19, computed by the library in 128-bit fixed point (host `out`). */
int hs_cdt_table(uint64_t out[20]);

/* ---------------------------------------------------------------- keys (Sec. 5 setup: one
   relinearisation key set plus power-of-two rotation keys) */
/* Generate a key-set from a 64-bit seed (ChaCha20 streams, RFC 8439): ternary secret s, public
   key (-a s + e, a), rotation keys index i = 0 .. log_n - 2 for left rotations by 2^i (Galois
   elements 3^(2^i) mod 2N), and a relinearisation key for s^2.  Key-switching keys use the hybrid form with
   digits of K data primes and special modulus P.  The key-set holds the secret key too: it plays
   both the key holder and the evaluation-key owner of the protocol. */
int hs_keygen(hs_ctx* ctx, uint64_t seed, void* stream, hs_keyset** out);
void hs_keyset_destroy(hs_keyset* ks);
/* Copy key material to host memory, for verification.  which: 0 = secret key, NTT form
   [n_moduli][N]; 1 = public key [2][L][N]; 2 = rotation key `index` (0 .. log_n - 2 as in
   hs_keygen; log_n - 1 .. 2 log_n - 3 for the right keys when added) [2][dnum][L+K][N] (b then a); 3 = relinearisation key, same layout; 4 = exact-step rotation key for the step
   `index` (HS_EKEY if the key-set holds none).  cap in u64 words; HS_ECAPACITY if short. */
int hs_keyset_export(const hs_keyset* ks, int which, int index, uint64_t* host_out, int64_t cap);
/* Add rotation keys for left rotations by exactly steps[i] slots (Sec. 2.1, HE-Rot with Galois
   element 3^k mod 2N; each step taken mod N/2).  Steps that are 0 or a power of two, and steps
   the key-set already holds, are skipped.  Afterwards every rotation by a held step -- in
   hs_rotate and in the totalSum of hs_he_spmv, its batched forms and the server -- is one key
   switch instead of one per power-of-two digit: the decrypted results are the same, the ciphertext
   limbs (their noise) differ.  Keys are [2][dnum][L+K][N] each (10.5 MiB at N = 16384 with
   6 + 1 primes), sampled from the key-set's seed with a stream id of their own.  Must not run
   concurrently with other calls that use the key-set; batch plans keep the keys they were
   recorded with.  Synchronises `stream`. */
int hs_keyset_add_rotation_keys(hs_ctx* ctx, hs_keyset* ks, const int64_t* host_steps, int64_t n,
                                void* stream);
/* Add rotation keys for right rotations by 2^i, i = 0 .. log_n - 2 (key index log_n - 1 + i,
   Galois element 3^(-2^i) = 3^(N/2 - 2^i) mod 2N, sampling id 64 + i); nothing if held.  Not the
   paper's reading of its power-of-two keys (left powers, binary digits), but the default of common
   BFV libraries: afterwards a rotation by k without an exact-step key -- in hs_rotate, the totalSum
   of hs_he_spmv, its batched forms, the server and the diagonal method -- applies the signed digits
   +-2^i of the non-adjacent form of k mod N/2 (no two adjacent digits nonzero: the fewest
   power-of-two key switches), lowest first, a digit of N/2 left out.  The decrypted results are the
   same; the limbs differ.  Keys as for hs_keyset_add_rotation_keys (13 more of 10.5 MiB at N =
   16384).  Must not run concurrently with other calls that use the key-set.  Synchronises
   `stream`. */
int hs_keyset_add_right_rotation_keys(hs_ctx* ctx, hs_keyset* ks, void* stream);

/* ---------------------------------------------------------------- Client A: matrix */
/* Pack an R x C integer matrix given in CSR form (device arrays: row_ptr int64[R+1] with
   row_ptr[0] = 0 and nondecreasing, col_idx int32[nnz] in [0, C) ascending within each row,
   vals int64[nnz], any magnitude; values are taken mod t).  Rows are split into partitions of
   N/2 rows (Sec. 4.7); each partition is converted to CSSC (rows sorted by descending nonzero
   count, stable, App. B), cut into chunks (Alg. generateChunk: column i joins the chunk started at
   column `start` while h * (i - start + 1) <= N/2), and each chunk's values are packed into the
   first slot row (slot k <-> column block k / h, sorted row k % h) and batch-encoded
   (encrypt_values = 0) or encrypted under `ks` with `seed` (encrypt_values = 1, both-encrypted
   variant).  Masks 1^h || 0 are encoded per chunk when agg_mode = 0.  Synchronises `stream`
   for the structure (CSSC arrays, chunks, column index); the plaintext and mask encoding of the
   plain path may still be running on the context's internal stream when the call returns, so it
   overlaps the caller's next work: every call that reads the plaintexts (hs_he_spmv, its batched,
   graph and server forms, hs_matrix_export) waits for it first.  HS_EPARAM for encrypt_values = 1
   on parameters whose tensor basis cannot hold the exact ciphertext product (hs_mul_ct). */
int hs_cssc_pack(hs_ctx* ctx, int64_t rows, int64_t cols, const int64_t* row_ptr,
                 const int32_t* col_idx, const int64_t* vals, int encrypt_values,
                 const hs_keyset* ks, uint64_t seed, void* stream, hs_matrix** out);
/* Matrices and ciphertext vectors take their device memory from the context's pool.  Every call
   that uses them synchronises its stream before returning except hs_mul_plain, hs_ctvec_copy and
   hs_batch_plan_run (and a matrix's plaintext encoding on the context's internal stream); their
   destroy functions wait for that work -- not for the whole device -- before handing the memory
   back.  A handle must not be destroyed while a call that uses it runs on another thread, while a
   server request holding it is not yet waited for, or while a batch plan borrows it; destroy
   before the context's hs_ctx_destroy. */
void hs_matrix_destroy(hs_matrix* m);
int hs_matrix_info(const hs_matrix* m, int64_t* n_parts, int64_t* n_chunks);
/* Result ciphertexts of hs_he_spmv for this matrix: the row partitions (slot_rows <= 1) or pairs of
   them (slot_rows = 2). */
int hs_matrix_groups(const hs_matrix* m, int64_t* n_groups);
/* Chunk k (global numbering over groups): out4 = (group = result ciphertext, first CSSC column,
   columns c, height h); a group is a row partition unless slot_rows = 2. */
int hs_matrix_chunk(const hs_matrix* m, int64_t k, int64_t out4[4]);
/* The CSSC column-index array (all partitions, concatenated) that Client A sends to Client B
   (Alg. "Sparse Matrix-Vector Multiplication"), into host memory. *len receives nnz. */
int hs_matrix_column_index(const hs_matrix* m, int32_t* host_ci, int64_t cap, int64_t* len);
/* The CSSC structure of row partition `part` (App. B; built on the device): the row map RM (the
   partition's local row indices ordered by descending nonzero count, equal counts in ascending
   row order; host int32[rows of the partition]) and the column pointers CP[0..Lw] (host
   int64[Lw + 1], Lw = the partition's longest row; CP[j + 1] - CP[j] = rows with more than j
   nonzeros).  lens[0], lens[1] receive the two lengths; HS_ECAPACITY if a capacity is short,
   HS_EINVAL for a partition out of range.  Synchronises the device. */
int hs_matrix_cssc(const hs_matrix* m, int64_t part, int32_t* host_rm, int64_t rm_cap, int64_t* host_cp,
                   int64_t cp_cap, int64_t lens[2]);
/* The distinct rotation steps (mod N/2, ascending) of the totalSum of every chunk of the matrix
   (Alg. Aggregation: e r and r for the chunk height r), into host memory; *len receives the count
   (HS_ECAPACITY if cap is short).  The layout is public, so a key holder can add exactly these
   keys with hs_keyset_add_rotation_keys. */
int hs_matrix_rotation_steps(const hs_matrix* m, int64_t* host_steps, int64_t cap, int64_t* len);
/* Encoded (NTT-form [L][N]) or encrypted ([2][L][N]) chunk k, or its mask (which = 1), to host. */
int hs_matrix_export(const hs_matrix* m, int which, int64_t k, uint64_t* host_out, int64_t cap);

/* ---------------------------------------------------------------- Client B: vector */
/* Reorganise the dense vector v (device int64[len], len = cols) per chunk (slot k = v[CI[k]], 0 for
   padding; Alg. reorgVector), batch-encode and encrypt under the public key of `ks` with `seed`:
   one ciphertext per chunk, ciphertext index = global chunk number. */
int hs_encrypt(hs_ctx* ctx, const hs_keyset* ks, const hs_matrix* m, const int64_t* v,
               int64_t len, uint64_t seed, void* stream, hs_ctvec** out);

/* ---------------------------------------------------------------- Cloud */
/* Encrypted SpMV: for each chunk the slot-wise product with the encrypted vector (HE-CMult, or
   HE-Mult + relinearisation for an encrypted matrix), the intra-chunk totalSum by rotations of
   e*h slots (Alg. Aggregation; each rotation applied as its power-of-two digits as in hs_rotate,
   one key switch per digit, or as one key switch with an exact-step key), the mask product
   (agg_mode 0), and the sum over the chunks of each group.  *y receives one ciphertext per group
   (hs_matrix_groups: a row partition, or a pair of them with slot_rows = 2). */
int hs_he_spmv(hs_ctx* ctx, const hs_keyset* ks, const hs_matrix* m, const hs_ctvec* x,
               void* stream, hs_ctvec** y);

/* Batched form: n independent encrypted SpMVs (request r: key-set ks[r], matrix m[r], vector
   x[r]; the same context) in one call.  The totalSum rotations of all requests are merged level by
   level into batched key switches, so small requests share launches and key reads; every result
   is identical to the request's own hs_he_spmv.  y[r] receives request r's result. */
int hs_he_spmv_batch(hs_ctx* ctx, int n, const hs_keyset* const* ks, const hs_matrix* const* m,
                     const hs_ctvec* const* x, void* stream, hs_ctvec** y);

/* Allocation-free form of hs_he_spmv, for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  The same arithmetic
   and result as hs_he_spmv, written to caller-owned device memory y (u64[y_words], 8-byte
   aligned, on the context's device): hs_matrix_groups(m) ciphertexts [2][L][N] in NTT form, one
   after another; wrap it with hs_ctvec_wrap to decrypt or export it.  Every intermediate buffer
   (slot products, totalSum ciphertexts, key-switch scratch, item arrays) is a slice of one fixed
   device array of 256 MiB that the library holds on each GPU it runs on until the process ends;
   the call makes no device allocation and no free.  Errors: HS_ECAPACITY if y_words is below the
   result's size; HS_ENOMEM (message: the size needed) if the call's intermediates exceed the
   fixed array -- the single 16384 x 16384 Zipf SpMV at N = 16384 with 6 + 1 primes fits, an
   encrypted-matrix SpMV at N = 32768 does not.  Every call on a GPU (any context, any thread)
   shares that GPU's array and leaves its last contents there: calls that overlap in time on one
   GPU race and must be serialised by the caller.  Returns after `stream` has drained. */
int hs_he_spmv_noalloc(hs_ctx* ctx, const hs_keyset* ks, const hs_matrix* m, const hs_ctvec* x,
                       uint64_t* y, int64_t y_words, void* stream);

/* Batched form recorded as a HIP graph, for a batch that is run repeatedly with new vector
   contents (same handles): hs_batch_plan_create does all host work of hs_he_spmv_batch once (chunk
   programs, rotation levels, item arrays, scratch and the result vectors), runs the batch once,
   then records its kernel sequence into a graph; hs_batch_plan_run replays it on `stream`
   (asynchronous; it reads the vectors x[r] as they are at replay time and overwrites the results).
   Results equal hs_he_spmv_batch's.  The plan borrows ks, m and x (they must outlive it) and owns
   its results: hs_batch_plan_output gives a borrowed handle, valid until the plan is destroyed
   (do not destroy it).  Plaintext matrices only (HS_EINVAL for encrypted values).
   hs_batch_plan_destroy waits for the plan's last replay. */
/* Copy the ciphertexts of src into dst (same context and count), asynchronously on `stream`:
   the way to give a graph plan new input vectors. */
int hs_ctvec_copy(hs_ctvec* dst, const hs_ctvec* src, void* stream);
typedef struct hs_batch_plan hs_batch_plan;
int hs_batch_plan_create(hs_ctx* ctx, int n, const hs_keyset* const* ks, const hs_matrix* const* m,
                         const hs_ctvec* const* x, void* stream, hs_batch_plan** out);
int hs_batch_plan_run(hs_batch_plan* plan, void* stream);
int hs_batch_plan_output(const hs_batch_plan* plan, int i, const hs_ctvec** y);
void hs_batch_plan_destroy(hs_batch_plan* plan);

/* ---------------------------------------------------------------- serving (continuous batching) */
typedef struct hs_server hs_server;
/* Start a server on `stream` (its own worker thread).  Engine ticks admit queued requests while
   the device footprint of the active ones (product, accumulator and rotation buffers, results)
   stays within hbm_budget_bytes (one request is always admitted) and at most max_active run; each
   tick advances every active request by one key switch of its totalSum, all in one batched level, so
   requests that arrive while others run share their launches.  Every result is identical to the
   request's own hs_he_spmv. */
int hs_server_create(hs_ctx* ctx, int64_t hbm_budget_bytes, int max_active, void* stream, hs_server** out);
/* Queue one request; the handles must stay alive until hs_server_wait returns for it.  *id
   receives the request id. */
int hs_server_submit(hs_server* s, const hs_keyset* ks, const hs_matrix* m, const hs_ctvec* x, int64_t* id);
/* Block until request `id` is done; *y receives its result (caller owns it).  times (optional,
   host): submit, admission and completion time in seconds since the server started. */
int hs_server_wait(hs_server* s, int64_t id, hs_ctvec** y, double times[3]);
/* out = [ticks, most requests active at once, admitted, completed, bytes in use, ticks whose
   admission left requests queued because the next one did not fit the budget, ticks that left
   requests queued because max_active were running, requests that stayed queued through at least
   one tick]; *now (optional) = seconds since the server started.  A request's footprint counts
   its chunk products, totalSum buffers and results, and for an encrypted matrix the exact-product
   scratch of the tick that admits it. */
int hs_server_stats(hs_server* s, int64_t out[8], double* now);
/* Drain the queue, stop the worker and free the server (results not yet collected are freed). */
void hs_server_destroy(hs_server* s);

/* ---------------------------------------------------------------- key holder */
/* Decrypt the per-group results and scatter each partition's slot row with its row map: out
   (device int64[rows]) receives y = A v reduced into (-t/2, t/2]; rows without nonzeros receive
   0. */
int hs_decrypt(hs_ctx* ctx, const hs_keyset* ks, const hs_matrix* m, const hs_ctvec* y,
               int64_t* out, int64_t rows, void* stream);

/* ---------------------------------------------------------------- the diagonal method
   The paper's baseline (Sec. 5, baseline approaches, and its diagonal-method figure), run on the
   same primitives so that the two methods are compared on one GPU.  The matrix is cut into square
   blocks of side B = min(N/4, max(rows, cols)), zero padded at the right and bottom edges.  Block
   (bi, bj) keeps each generalised diagonal d (0 <= d < B) that holds a stored entry:
   diag[i] = A[bi B + i][bj B + (i + d) mod B], encoded into slots [0, B) of slot row 0 as one
   NTT-form plaintext.  Diagonals are ordered by (bi, bj, d).  The vector block bj is encrypted
   twice over (slots j and B + j hold v[bj B + j]), so a left rotation by d puts
   v[bj B + (i + d) mod B] in slot i.  Result block bi = sum over its diagonals of
   diag (.) Rot(x_bj, d); its slots [0, B) hold rows bi B .. bi B + B - 1 of A v mod t. */
/* Client A: CSR (device row_ptr int64[rows+1], col_idx int32[nnz], vals int64[nnz], columns
   strictly ascending within a row) -> the diagonal plaintexts.  HS_EINVAL for malformed CSR;
   HS_ECAPACITY when block rows x block columns x B reaches 2^31 (one flag byte per possible
   diagonal is kept on host and device while packing). */
int hs_diag_pack(hs_ctx* ctx, int64_t rows, int64_t cols, const int64_t* row_ptr,
                 const int32_t* col_idx, const int64_t* vals, void* stream, hs_diag** out);
void hs_diag_destroy(hs_diag* d);
/* out4 = (B, block rows, block columns, diagonals). */
int hs_diag_info(const hs_diag* d, int64_t out4[4]);
/* The diagonals' (bi, bj, d) triples in their order, into host int64[3 * diagonals]. */
int hs_diag_keys(const hs_diag* d, int64_t* host_out, int64_t cap);
/* Diagonal k's plaintext, [L][N] NTT form, into host memory. */
int hs_diag_export(const hs_diag* d, int64_t k, uint64_t* host_out, int64_t cap);
/* The distinct non-zero rotation steps d of the diagonals, ascending (for
   hs_keyset_add_rotation_keys); *len receives the count, HS_ECAPACITY if cap is smaller. */
int hs_diag_rotation_steps(const hs_diag* d, int64_t* host_steps, int64_t cap, int64_t* len);
/* Client B: the vector (device int64[len], len = cols) as one ciphertext per block column, each
   x_bj || x_bj, encrypted with the sampling index bj. */
int hs_diag_encrypt(hs_ctx* ctx, const hs_keyset* ks, const hs_diag* d, const int64_t* v,
                    int64_t len, uint64_t seed, void* stream, hs_ctvec** out);
/* Cloud: one result ciphertext per block row.  Rot(x_bj, d) uses one exact-step key switch when
   the key-set holds a key for d, else the power-of-two digits of d as in hs_rotate (each partial
   rotation, a partial sum of those digits, computed once per block column).  hs_last_counters then reports [0] key switches,
   [1] distinct rotated blocks, [2] kernel launches, [3] diagonal products. */
int hs_diag_spmv(hs_ctx* ctx, const hs_keyset* ks, const hs_diag* d, const hs_ctvec* x,
                 void* stream, hs_ctvec** y);
/* Key holder: out (device int64[rows]) = A v reduced into (-t/2, t/2]. */
int hs_diag_decrypt(hs_ctx* ctx, const hs_keyset* ks, const hs_diag* d, const hs_ctvec* y,
                    int64_t* out, int64_t rows, void* stream);

/* ---------------------------------------------------------------- ciphertext vectors */
int hs_ctvec_count(const hs_ctvec* v, int64_t* n);
/* Ciphertext i as [2][L][N] NTT-form residues, into host memory (synchronises the device). */
int hs_ct_export(const hs_ctvec* v, int64_t i, uint64_t* host_limbs, int64_t cap);
/* Ciphertext i in the canonical coefficient form: [2][L][N] residues in [0, q_i) of the
   polynomials c0, c1 (coefficient k of limb i is c_p(X) mod q_i at X^k), into host memory.  The
   inverse NTT runs on the device (its own scratch, on `stream`, which is then synchronised);
   `v` is not modified.  cap in u64 words (HS_ECAPACITY if short); HS_EINVAL for i out of range. */
int hs_ct_export_coeff(const hs_ctvec* v, int64_t i, uint64_t* host_limbs, int64_t cap, void* stream);
/* Build a vector of n ciphertexts from host limbs [n][2][L][N] (NTT form, residues < q_i). */
int hs_ctvec_import(hs_ctx* ctx, const uint64_t* host_limbs, int64_t n, hs_ctvec** out);
/* Wrap caller-owned device memory (e.g. a torch tensor's data_ptr()) holding n ciphertexts
   [n][2][L][N] u64, NTT form, residues < q_i, as a vector handle without copying: every call that
   takes an hs_ctvec reads it (hs_he_spmv's x, hs_ctvec_copy's dst ...) in place.  `dev` must be
   8-byte aligned on the context's device and stay allocated until hs_ctvec_destroy, which frees
   the handle only, never the memory.  HS_EINVAL for a null pointer, n < 1 or misalignment. */
int hs_ctvec_wrap(hs_ctx* ctx, void* dev, int64_t n, hs_ctvec** out);
void hs_ctvec_destroy(hs_ctvec* v);

/* ---------------------------------------------------------------- primitive operations
   (the building blocks of the protocol, exposed for verification and composition; device
   pointers, enqueued on `stream`) */
/* In-place negacyclic NTT (inverse = 0) or inverse NTT (inverse = 1) of n_polys polynomials of
   n_limbs limbs each, limb l reduced modulo chain modulus mod0 + l (mod0 = -1: the plaintext
   modulus t, n_limbs = 1).  d_limbs: device u64 [n_polys][n_limbs][N], residues < modulus. */
int hs_ntt(hs_ctx* ctx, uint64_t* d_limbs, int64_t n_polys, int mod0, int n_limbs, int inverse,
           void* stream);
/* Slot-wise product of every ciphertext of `in` with the NTT-form plaintext pt (device u64
   [L][N]) (HE-CMult). */
int hs_mul_plain(hs_ctx* ctx, const hs_ctvec* in, const uint64_t* d_pt, void* stream, hs_ctvec** out);
/* Left rotation of every ciphertext of `in` by k slots within each slot row (HE-Rot): one Galois
   automorphism 3^k plus a key switch when the key-set holds an exact-step key for k mod N/2, else
   the binary digits of k mod N/2 in ascending order (with the right keys of
   hs_keyset_add_right_rotation_keys: the signed digits +-2^i of its non-adjacent form), each a
   Galois automorphism 3^(+-2^i) plus a key switch. */
int hs_rotate(hs_ctx* ctx, const hs_keyset* ks, const hs_ctvec* in, int64_t k, void* stream,
              hs_ctvec** out);
/* Slot-wise product of two ciphertexts (HE-Mult): exact scaled tensor round(t/Q * (a (x) b)) of the
   centered lifts, then relinearisation.  Vectors of equal length, element by element. */
int hs_mul_ct(hs_ctx* ctx, const hs_keyset* ks, const hs_ctvec* a, const hs_ctvec* b,
              void* stream, hs_ctvec** out);

/* Execution options (they never change results, only which kernels compute them).  Each context
   holds its own setting of every option (hs_ctx_set_option; value -1 = unset); an unset option
   takes the process-wide default set by hs_set_option, read at each call.  The process-wide
   defaults are the one piece of global mutable state of the library: they exist so that a test or
   benchmark can switch kernels for every context at once.  Setting an option must not race with
   calls that use it (on the context, or on any context for a process-wide default).  Keys:
   HS_OPT_KS_PIPELINE  key switching of a rotation level: 0 = automatic, 1 = one workgroup per limb
                       transform (least HBM traffic; large batches), 2 = two-pass transforms over
                       N/2048 workgroups per limb (lowest latency; small batches; always used for
                       N = 32768, whose limb does not fit in LDS)
   HS_OPT_NTT_PATH     hs_ntt and the library's batched transforms: 0 = automatic (N = 2^15: one
                       workgroup per limb on half-limb LDS from 256 limbs on, else two-pass),
                       1 = one workgroup per limb, 2 = two-pass
   HS_OPT_KS_THRESHOLD automatic choice: two-pass when (L + K) x items of a level is below this
                       value; 0 = default (192 at N = 2^14 with the register accumulators of
                       HS_OPT_MODUP_ACC, else 512)
   HS_OPT_AUX_PATH     keygen, encoding, encryption, decryption: 0 = automatic, 1 = fused kernels
                       with the limb in LDS, 2 = elementwise kernels around batched transforms
                       (always used for N = 32768)
   HS_OPT_MODUP_GROUP  two-pass ModUp: targets per workgroup, 0 = automatic (by level size and block
                       geometry), 1 = one
                       (the digit's inverse pass repeated per target), 2 or 3 = one inverse pass
                       shared by that many targets
   HS_OPT_NTT_PIPE     forward transforms of many N = 2^14 limbs (hs_ntt, encryption): 0 = automatic
                       (a persistent grid of two workgroups per CU that reads each workgroup's next
                       limb while it finishes the current one, used from two limbs per workgroup
                       on), 1 = one workgroup per limb
   HS_OPT_KS_BLOCK     two-pass key switching at N = 2^14, elements per workgroup block: 1 = 2048
                       (the inner product on 1024), 2 = 1024 throughout, 3 = 512 for the single-pass
                       kernels and 1024 for ModUp and the key inner product (more, shorter
                       workgroups for latency-bound small levels), 0 = automatic (3 up to 8 items
                       per level, else 1)
   HS_OPT_MODUP_ACC    one-workgroup-per-limb key switching at N = 2^14, ModUp + key inner product:
                       0 = automatic (3 from 64 items per level on, else 2), 1 = one workgroup per
                       (target modulus, item) with the accumulators read and written in memory
                       for every digit, 2 = one workgroup of 512 threads per (half of the target
                       limb, item) with the accumulators in registers across the digits (written
                       once), 3 = the same with one workgroup of 1024 threads per whole limb
   HS_OPT_KS_FUSE      consecutive two-pass rotation levels: 0 = automatic (the last kernel of a
                       level also runs the first step of the next level's key switch for each
                       item whose input is an output of this level), 1 = every level runs its own
                       first step
   HS_EINVAL for an unknown key or value. */
#define HS_OPT_KS_PIPELINE 1
#define HS_OPT_NTT_PATH 2
#define HS_OPT_KS_THRESHOLD 3
#define HS_OPT_AUX_PATH 4
#define HS_OPT_MODUP_GROUP 5
#define HS_OPT_NTT_PIPE 6
#define HS_OPT_KS_BLOCK 7
#define HS_OPT_MODUP_ACC 8
#define HS_OPT_KS_FUSE 9
int hs_set_option(int key, int64_t value);
int hs_ctx_set_option(hs_ctx* ctx, int key, int64_t value);

/* Autotuner.  Times, on synthetic operands and the key-switching key of `ks`, (1) the two variants
   of the one-workgroup-per-limb transforms (N = 2^14: half-limb LDS with 512 threads vs whole limb
   with 1024; N = 2^11..2^13: compile-time radix-16 rounds vs runtime radix-8 rounds), once inside
   the key-switch kernels on a 32-item rotation level and once in the plain transform kernels on
   64 polynomials of L + K limbs (forward + inverse), and (2) the two key-switch pipelines
   (two-pass vs one workgroup per limb) on levels of B = 1, 2, 4, ..., 64 items, and stores the
   faster choices in the context; later calls use them (results never depend on these choices;
   HS_OPT_KS_PIPELINE still forces a pipeline).  Report (host `report`, capacity `cap` doubles;
   *len receives the count, 27): [key-switch variant, ms variant 0, ms variant 1, transform variant,
   ms variant 0, ms variant 1], then per B: [B, ms one workgroup per limb, ms two-pass] (0 where a
   variant does not exist for the ring).  Not thread-safe against concurrent calls on the context. */
int hs_autotune(hs_ctx* ctx, const hs_keyset* ks, void* stream, double* report, int cap, int* len);
/* The context's launch choices: out[0] key-switch transform variant, out[1] plain transform
   variant (0/1 as above), out[2 + b] key-switch pipeline for levels of 2^(b-1) < B <= 2^b items
   (b = 7: larger): 1 two-pass, 0 one workgroup per limb, -1 the fixed threshold rule
   (HS_OPT_KS_THRESHOLD).  hs_set_tuning installs such a table. */
int hs_tuning(const hs_ctx* ctx, int64_t out[10]);
int hs_set_tuning(hs_ctx* ctx, const int64_t in[10]);

/* Kernel timing: hs_profile(1) clears the records and brackets every subsequent kernel launch with
   two HIP events on its stream; hs_profile(0) stops.  hs_profile_summary waits for the recorded
   events and writes one text line per kernel, "name launches total_ms units", NUL-terminated, into
   host `buf` (capacity `cap` bytes; *len receives the length; HS_ECAPACITY if it does not fit);
   units = the work the launches processed: rotation items (key switches) for the key-switch
   kernels, limbs for the one-workgroup N = 2^15 transform, 0 for the others. */
int hs_profile(int enable);
int hs_profile_summary(char* buf, int64_t cap, int64_t* len);

/* Counters of the calling thread's last hs_he_spmv / hs_he_spmv_batch: [0] key switches,
   [1] logical rotations, [2] kernel launches, [3] slot-wise products, [4] mask products. */
int hs_last_counters(int64_t out[5]);

#ifdef __cplusplus
}
#endif
#endif /* HESPMV_H */
