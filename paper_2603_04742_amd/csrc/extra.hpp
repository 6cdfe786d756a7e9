// Launchers beside those of kernels.hpp: the diagonal method's packing kernels (aux2.hip), the
// encryption samples in one launch, encryption's transforms with the prologue in their input,
// the switch of the pipelined forward transform (kernels.hip),
// the block size of the two-pass key switch (ks2.hip).
#pragma once
#include "hs_internal.hpp"

namespace hs {
void launch_diag_mark(const i64* row_ptr, const int* col, i64 R, i64 C, i64 B, i64 ncb, unsigned char* flags, hipStream_t st);
void launch_diag_place(const hs_ctx* c, const i64* row_ptr, const int* col, const i64* val, i64 R, i64 B, i64 ncb, const i64* ids, int nd,
                       u64* out, hipStream_t st);
void launch_diag_vector(const hs_ctx* c, const i64* v, i64 C, i64 B, int ncb, u64* out, hipStream_t st);
void launch_sample_enc(const hs_ctx* c, int* out, int nobj, u64 seed, u32 pu, u32 pe0, u32 pe1, hipStream_t st);
void launch_enc_ntt(const hs_ctx* c, const u64* mcoef, const int* samples, int n_ct, u64* prep, hipStream_t st);
}  // namespace hs
