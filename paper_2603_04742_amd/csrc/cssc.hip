// CSR -> CSSC on the device (App. B, conversion from CSR to CSSC), per row partition of s rows
// (Sec. 4.7): the nonzero count of every row, the rows ordered by descending count -- stable, so
// equal counts keep ascending row order -- the row map RM and each row's rank in that order, and
// the column pointers CP[j] = sum_{j' < j} #{rows with count > j'} (j = 0 .. Lw, Lw the longest
// row).  The order is a least-significant-digit radix sort, 8 bits per pass, of the key
// Lw_p - count over blocks of rows that never straddle a partition; a pass is a per-block digit
// histogram, a per-partition scan of the histograms (digit-major, then block) and a stable
// scatter (the rank of an element among the block's elements of its digit that precede it).
#include <hip/hip_runtime.h>

#include <mutex>

#include "kernels.hpp"

namespace hs {

int cssc_sort_block(i64 s) { return (int)std::min<i64>(256, s); }

// Per row: its count (clamped to [0, 2^30 + 1]); stat[0] |= 1 when row_ptr[0] != 0, a count is
// negative or above 2^30; stat[1] = row_ptr[R]; per partition p: stat[2 + 2p] = its longest row,
// stat[3 + 2p] = row_ptr[p s].  Reads row_ptr only (no other address comes from it).
__global__ void k_csr_rows(const i64* __restrict__ rp, i64 R, i64 s, int* __restrict__ cnt, unsigned long long* stat) {
  const i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x;
  if (i >= R) return;
  const i64 a = rp[i], b = rp[i + 1];
  const i64 c = b - a;
  const i64 cmax = (i64)1 << 30;
  if ((i == 0 && a != 0) || c < 0 || c > cmax) atomicOr(&stat[0], 1ull);
  const i64 cc = c < 0 ? 0 : (c > cmax ? cmax + 1 : c);
  cnt[i] = (int)cc;
  const i64 p = i / s;
  atomicMax(&stat[2 + 2 * p], (unsigned long long)cc);
  if (i == p * s) stat[3 + 2 * p] = (unsigned long long)a;
  if (i == R - 1) stat[1] = (unsigned long long)b;
}

// Sort keys Lw_p - count and the identity order.
__global__ void k_sort_init(const int* __restrict__ cnt, const unsigned long long* __restrict__ stat, i64 R, i64 s, u32* key, int* idx) {
  const i64 i = blockIdx.x * (i64)blockDim.x + threadIdx.x;
  if (i >= R) return;
  const i64 lw = (i64)stat[2 + 2 * (i / s)];
  key[i] = (u32)(lw - cnt[i]);
  idx[i] = (int)i;
}

// Digit histogram of each block of BR positions: bh[b][d].
__global__ void k_sort_hist(const u32* __restrict__ key, i64 R, int BR, int sh, int* bh) {
  __shared__ int h[256];
  const int b = blockIdx.x;
  for (int d = threadIdx.x; d < 256; d += blockDim.x) h[d] = 0;
  __syncthreads();
  const i64 pos = (i64)b * BR + threadIdx.x;
  if (threadIdx.x < BR && pos < R) atomicAdd(&h[(key[pos] >> sh) & 255], 1);
  __syncthreads();
  for (int d = threadIdx.x; d < 256; d += blockDim.x) bh[(size_t)b * 256 + d] = h[d];
}

// One workgroup (256 threads) per partition: bh[b][d] becomes the first destination position of
// digit d of block b -- the partition's first row + the elements of smaller digits in the
// partition + the elements of digit d in earlier blocks of the partition.
__global__ void k_sort_scan(int* bh, i64 R, i64 s, int BR) {
  __shared__ int tot[256];
  const int p = blockIdx.x, d = threadIdx.x;
  const i64 nblk = (R + BR - 1) / BR;
  const i64 b0 = p * (s / BR), b1 = std::min<i64>(nblk, (p + 1) * (s / BR));
  int t = 0;
  for (i64 b = b0; b < b1; b++) t += bh[(size_t)b * 256 + d];
  tot[d] = t;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {   // inclusive scan over the digits, then exclusive
    const int w = d >= o ? tot[d - o] : 0;
    __syncthreads();
    tot[d] += w;
    __syncthreads();
  }
  const int excl = tot[d] - t;
  int run = (int)(p * s) + excl;
  for (i64 b = b0; b < b1; b++) {
    const int v = bh[(size_t)b * 256 + d];
    bh[(size_t)b * 256 + d] = run;
    run += v;
  }
}

// Stable scatter of one pass: blockDim = BR; the element at position b BR + t goes to the first
// position of its digit in this block + the number of the block's earlier elements with that digit.
__global__ void k_sort_scatter(const u32* __restrict__ kin, const int* __restrict__ iin, u32* kout, int* iout, const int* __restrict__ off,
                               i64 R, int BR, int sh) {
  __shared__ int dg[256];
  const int b = blockIdx.x, t = threadIdx.x;
  const i64 pos = (i64)b * BR + t;
  const bool ok = pos < R;
  const u32 k = ok ? kin[pos] : 0u;
  const int v = ok ? iin[pos] : 0;
  const int d = ok ? (int)((k >> sh) & 255) : -1;
  dg[t] = d;
  __syncthreads();
  if (!ok) return;
  int rank = 0;
  for (int u = 0; u < t; u++) rank += dg[u] == d;
  const int dst = off[(size_t)b * 256 + d] + rank;
  kout[dst] = k;
  iout[dst] = v;
}

// RM[pos] = local row at sorted position pos; rank[row] = its local sorted position.
__global__ void k_sort_finish(const int* __restrict__ idx, i64 R, i64 s, int* rm, int* rank) {
  const i64 pos = blockIdx.x * (i64)blockDim.x + threadIdx.x;
  if (pos >= R) return;
  const i64 base = (pos / s) * s;
  const int row = idx[pos];
  rm[pos] = (int)(row - base);
  rank[row] = (int)(pos - base);
}

// One workgroup of 256 threads per partition: CP of the partition at cp + cp_off[p], Lw + 1
// entries, then padded with its last value up to cp_len[p] entries.  From the sorted keys: the
// rows with count > j are the first k + 1 sorted rows for every j in [count(k + 1), count(k)), so
// each j < Lw is written once; CP is the running sum of those numbers.
__global__ void k_cssc_cp(const u32* __restrict__ key, const unsigned long long* __restrict__ stat, i64 R, i64 s,
                          const i64* __restrict__ cp_off, const i64* __restrict__ cp_len, i64* cp) {
  __shared__ i64 sc[256];
  __shared__ i64 carry;
  const int p = blockIdx.x, t = threadIdx.x;
  const i64 lw = (i64)stat[2 + 2 * p];
  const i64 base = (i64)p * s, rows = std::min<i64>(s, R - base);
  i64* out = cp + cp_off[p];
  for (i64 k = t; k < rows; k += blockDim.x) {
    const i64 c = lw - key[base + k];
    const i64 cn = k + 1 < rows ? lw - key[base + k + 1] : 0;
    for (i64 j = cn; j < c; j++) out[1 + j] = k + 1;
  }
  if (t == 0) { out[0] = 0; carry = 0; }
  __syncthreads();
  for (i64 j0 = 0; j0 < lw; j0 += blockDim.x) {
    const i64 j = j0 + t;
    i64 v = j < lw ? out[1 + j] : 0;
    sc[t] = v;
    __syncthreads();
    for (int o = 1; o < (int)blockDim.x; o <<= 1) {
      const i64 w = t >= o ? sc[t - o] : 0;
      __syncthreads();
      sc[t] += w;
      __syncthreads();
    }
    if (j < lw) out[1 + j] = carry + sc[t];
    __syncthreads();
    if (t == (int)blockDim.x - 1) carry += sc[t];
    __syncthreads();
  }
  const i64 last = out[lw];
  for (i64 j = lw + 1 + t; j < cp_len[p]; j += blockDim.x) out[j] = last;
}

// ---- one-pass form, for partitions whose rows hold at most 255 nonzeros (the common case): the
// key 255 - count fits one 8-bit digit, so one histogram / scan / scatter orders the rows, and
// CP follows from the partition's histogram; the host reads the statistics and CP in one copy.
// hdr (i64): [0] row_ptr[R], then per partition p: [1 + 3p] longest row, [2 + 3p] flags (1: a
// malformed row pointer, 2: a row longer than 255), [3 + 3p] row_ptr[p s].  cp: 256 entries per
// partition (CP[0..Lw], then its last value repeated).

// Blocks of BR rows (one partition each): the digit of every row, the block's digit histogram
// and flags, row_ptr at the partition starts and at R.
__global__ void k_cssc_rows1(const i64* __restrict__ rp, i64 R, i64 s, int BR, int* __restrict__ dig, int* __restrict__ bh,
                             int* __restrict__ bflag, i64* __restrict__ hdr) {
  __shared__ int h[256];
  __shared__ int fl;
  const int b = blockIdx.x, t = threadIdx.x;
  for (int d = t; d < 256; d += blockDim.x) h[d] = 0;
  if (t == 0) fl = 0;
  __syncthreads();
  const i64 i = (i64)b * BR + t;
  if (i < R) {
    const i64 a = rp[i], e = rp[i + 1];
    const i64 c = e - a;
    int f = ((i == 0 && a != 0) || c < 0 || c > ((i64)1 << 30)) ? 1 : 0;
    if (c > 255) f |= 2;
    if (f) atomicOr(&fl, f);
    const int d = 255 - (int)(c < 0 ? 0 : (c > 255 ? 255 : c));
    dig[i] = d;
    atomicAdd(&h[d], 1);
    const i64 p = i / s;
    if (i == p * s) hdr[3 + 3 * p] = a;
    if (i == R - 1) hdr[0] = e;
  }
  __syncthreads();
  for (int d = t; d < 256; d += blockDim.x) bh[(size_t)b * 256 + d] = h[d];
  if (t == 0) bflag[b] = fl;
}

// Inclusive prefix sum over the 256 threads of a workgroup: within each 64-lane wave by shuffles,
// then the totals of the earlier waves (ws: 4 values of LDS; two barriers).
template <class T>
__device__ __forceinline__ T scan256_incl(T v, T* ws) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  if (lane == 63) ws[wv] = v;
  __syncthreads();
  T add = 0;
  for (int i = 0; i < wv; i++) add += ws[i];
  __syncthreads();
  return v + add;
}

// One workgroup of 256 threads per partition: the partition's histogram tot[d] and flags; bh[b][d]
// becomes the first destination of digit d of block b (as k_sort_scan); CP[j + 1] - CP[j] = rows
// with count > j = rows with digit < 255 - j = the exclusive prefix of tot at 255 - j.  The
// partition's block histograms (at most N / 512 blocks) are staged in LDS with coalesced loads,
// so the per-digit running sums over the blocks read LDS, not global memory.
__global__ void k_cssc_scan1(int* bh, const int* __restrict__ bflag, i64 R, i64 s, int BR, i64* hdr, i64* cp) {
  extern __shared__ int sh[];            // [nb][256] block histograms of the partition
  __shared__ int base[256];              // exclusive prefix of the partition histogram over digits
  __shared__ i64 ws[4];                  // wave totals of the scans
  __shared__ int fl, dmin;
  const int p = blockIdx.x, d = threadIdx.x;
  const i64 nblk = (R + BR - 1) / BR;
  const i64 b0 = p * (s / BR), b1 = std::min<i64>(nblk, (p + 1) * (s / BR));
  const int nb = (int)(b1 - b0);
  if (d == 0) { fl = 0; dmin = 255; }
  for (int i = d; i < nb * 256; i += 256) sh[i] = bh[(size_t)b0 * 256 + i];
  int f = 0;
  for (int b = d; b < nb; b += 256) f |= bflag[b0 + b];
  __syncthreads();
  if (f) atomicOr(&fl, f);
  int t = 0;
  for (int b = 0; b < nb; b++) t += sh[b * 256 + d];
  if (t && d < 255) atomicMin(&dmin, d);   // the smallest digit present: the longest row (else 255)
  // exclusive scan of the histogram over the digits
  const int incl = (int)scan256_incl<i64>(t, ws);
  base[d] = incl - t;
  __syncthreads();
  // CP[j + 1] = sum_{i <= j} base[255 - i] for j < Lw, then the last value repeated
  const i64 lw = 255 - dmin;
  const i64 cpi = scan256_incl<i64>(d < lw ? (i64)base[255 - d] : 0, ws);
  i64* out = cp + (size_t)p * 256;
  if (d < 255) out[d + 1] = cpi;   // entries past Lw add zero, so the sum stays at CP[Lw]
  if (d == 0) out[0] = 0;
  if (d == 0) {
    hdr[1 + 3 * p] = lw;
    hdr[2 + 3 * p] = fl;
  }
  // destinations: digit d of block b starts after the partition's rows of smaller digits and
  // the rows of digit d in earlier blocks
  int run = (int)(p * s) + base[d];
  for (int b = 0; b < nb; b++) {
    const int v = sh[b * 256 + d];
    sh[b * 256 + d] = run;
    run += v;
  }
  __syncthreads();
  for (int i = d; i < nb * 256; i += 256) bh[(size_t)b0 * 256 + i] = sh[i];
}

// The scatter of the one pass (rows in their original order): RM and each row's rank.  A row's
// rank among the block's rows of its digit = the rows of that digit in earlier waves (per-wave
// histograms in LDS) + the earlier lanes of its wave with the same digit (eight ballots give the
// lanes whose digit equals this lane's).
__global__ void k_cssc_scatter1(const int* __restrict__ dig, const int* __restrict__ off, i64 R, i64 s, int BR, int* rm, int* rank) {
  __shared__ int wh[4][256];   // BR <= 256: at most four waves
  const int b = blockIdx.x, t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6, nw = ((int)blockDim.x + 63) >> 6;
  for (int x = t; x < nw * 256; x += blockDim.x) wh[x >> 8][x & 255] = 0;
  __syncthreads();
  const i64 i = (i64)b * BR + t;
  const bool ok = i < R;
  const int d = ok ? dig[i] : 0;
  int r = 0;
  if (ok) {
    unsigned long long same = __ballot(1);
#pragma unroll
    for (int bit = 0; bit < 8; bit++) {
      const unsigned long long m = __ballot((d >> bit) & 1);
      same &= ((d >> bit) & 1) ? m : ~m;
    }
    r = __popcll(same & ((1ull << lane) - 1));
    if ((same >> lane) == 1ull) wh[wv][d] = __popcll(same);   // the wave's last lane of this digit
  }
  __syncthreads();
  if (!ok) return;
  for (int u = 0; u < wv; u++) r += wh[u][d];
  const i64 dst = off[(size_t)b * 256 + d] + r;
  const i64 base = (i / s) * s;
  rm[dst] = (int)(i - base);
  rank[i] = (int)(dst - base);
}

static unsigned grid_of(i64 n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_cssc_one_pass(const i64* row_ptr, i64 R, i64 s, int* dig, int* bh, int* bflag, i64* hdr, i64* cp, int* rm, int* rank,
                          hipStream_t st) {
  if (R <= 0) return;
  const int BR = cssc_sort_block(s);
  const i64 nblk = (R + BR - 1) / BR;
  const int nP = (int)((R + s - 1) / s);
  ProfScope _prof("k_cssc_one_pass", st);
  hipLaunchKernelGGL(k_cssc_rows1, dim3((unsigned)nblk), dim3(BR), 0, st, row_ptr, R, s, BR, dig, bh, bflag, hdr);
  const size_t lds = (size_t)(s / BR) * 256 * sizeof(int);   // one partition's block histograms
  static std::once_flag attr;   // up to 64 KiB (N = 32768) beside the static arrays
  std::call_once(attr, [] {
    (void)hipFuncSetAttribute((const void*)k_cssc_scan1, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024);
  });
  hipLaunchKernelGGL(k_cssc_scan1, dim3((unsigned)nP), dim3(256), lds, st, bh, bflag, R, s, BR, hdr, cp);
  hipLaunchKernelGGL(k_cssc_scatter1, dim3((unsigned)nblk), dim3(BR), 0, st, dig, bh, R, s, BR, rm, rank);
  HS_CHECK_HIP(hipGetLastError());
}

void launch_csr_rows(const i64* row_ptr, i64 R, i64 s, int* cnt, unsigned long long* stat, hipStream_t st) {
  if (R <= 0) return;
  ProfScope _prof("k_csr_rows", st);
  hipLaunchKernelGGL(k_csr_rows, dim3(grid_of(R, 256)), dim3(256), 0, st, row_ptr, R, s, cnt, stat);
  HS_CHECK_HIP(hipGetLastError());
}

// Returns the buffer (keyA or keyB) that holds the sorted keys.
const u32* launch_cssc_order(const int* cnt, const unsigned long long* stat, i64 R, i64 s, int passes, u32* keyA, u32* keyB, int* idxA,
                             int* idxB, int* bh, int* rm, int* rank, hipStream_t st) {
  if (R <= 0) return keyA;
  const int BR = cssc_sort_block(s);
  const i64 nblk = (R + BR - 1) / BR;
  const int nP = (int)((R + s - 1) / s);
  ProfScope _prof("k_cssc_order", st);
  hipLaunchKernelGGL(k_sort_init, dim3(grid_of(R, 256)), dim3(256), 0, st, cnt, stat, R, s, keyA, idxA);
  for (int ps = 0; ps < passes; ps++) {
    hipLaunchKernelGGL(k_sort_hist, dim3((unsigned)nblk), dim3(BR), 0, st, keyA, R, BR, 8 * ps, bh);
    hipLaunchKernelGGL(k_sort_scan, dim3((unsigned)nP), dim3(256), 0, st, bh, R, s, BR);
    hipLaunchKernelGGL(k_sort_scatter, dim3((unsigned)nblk), dim3(BR), 0, st, keyA, idxA, keyB, idxB, bh, R, BR, 8 * ps);
    std::swap(keyA, keyB);
    std::swap(idxA, idxB);
  }
  hipLaunchKernelGGL(k_sort_finish, dim3(grid_of(R, 256)), dim3(256), 0, st, idxA, R, s, rm, rank);
  HS_CHECK_HIP(hipGetLastError());
  return keyA;
}

void launch_cssc_cp(const u32* key_sorted, const unsigned long long* stat, i64 R, i64 s, const i64* cp_off, const i64* cp_len, i64* cp,
                    hipStream_t st) {
  if (R <= 0) return;
  const int nP = (int)((R + s - 1) / s);
  ProfScope _prof("k_cssc_cp", st);
  hipLaunchKernelGGL(k_cssc_cp, dim3((unsigned)nP), dim3(256), 0, st, key_sorted, stat, R, s, cp_off, cp_len, cp);
  HS_CHECK_HIP(hipGetLastError());
}

}  // namespace hs
