// Fixed device scratch of the allocation-free encrypted SpMV (hs_he_spmv_noalloc): every buffer of
// such a call (slot products, totalSum ping-pong ciphertexts, key-switch intermediates, item and
// argument arrays) is a slice of one file-scope device array.  Each GPU the library runs on holds
// its own copy of the array until the process ends; all calls on one GPU share it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "hs_internal.hpp"
#include "kernels.hpp"

namespace hs {
// 256 MiB: the single 16384 x 16384 Zipf SpMV (N = 16384, 6 + 1 primes) needs about 200 MiB
constexpr size_t kNoAllocScratchBytes = (size_t)256 << 20;
}  // namespace hs

static __device__ __align__(256) unsigned char scratch[hs::kNoAllocScratchBytes];

namespace hs {

// Device address of `scratch` on the current device, looked up once per device with that device
// current (the host-side name of the array is not a device address).
int noalloc_scratch(void** ptr, size_t* bytes) {
  static std::mutex mu;
  static std::vector<void*> addr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return HS_EDEVICE;
  std::lock_guard<std::mutex> g(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return HS_EDEVICE;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  *bytes = kNoAllocScratchBytes;
  return HS_OK;
}

__global__ void k_fill_u64(u64* p, size_t n, u64 v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// p[0, n) = v with a kernel (a memset node recorded into a graph is avoided)
void launch_fill_u64(u64* p, size_t n, u64 v, hipStream_t st) {
  if (!n) return;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 2048);
  k_fill_u64<<<(unsigned)blocks, 256, 0, st>>>(p, n, v);
  HS_CHECK_HIP(hipGetLastError());
}

// Up to kCopyJobs device-to-device copies of u64 words in one launch (grid y = the job), the
// pointers in the kernel arguments; 16-byte words when every pointer is 16-byte aligned.
static constexpr int kCopyJobs = 32;
struct CopyBatch {
  const u64* src[kCopyJobs];
  u64* dst[kCopyJobs];
  size_t words[kCopyJobs];
};
template <bool VEC>
__global__ void k_copy_batch(CopyBatch cb) {
  const int j = blockIdx.y;
  const u64* s = cb.src[j];
  u64* d = cb.dst[j];
  const size_t w = cb.words[j];
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (VEC) {
    const ulonglong2* s2 = (const ulonglong2*)s;
    ulonglong2* d2 = (ulonglong2*)d;
    for (; i < w / 2; i += stride) d2[i] = s2[i];
  } else {
    for (; i < w; i += stride) d[i] = s[i];
  }
}

void launch_copy_batch(const u64* const* src, u64* const* dst, const size_t* words, int n, hipStream_t st) {
  for (int j0 = 0; j0 < n; j0 += kCopyJobs) {
    const int m = std::min(kCopyJobs, n - j0);
    CopyBatch cb{};
    bool vec = true;
    size_t most = 0;
    for (int j = 0; j < m; j++) {
      cb.src[j] = src[j0 + j];
      cb.dst[j] = dst[j0 + j];
      cb.words[j] = words[j0 + j];
      vec &= ((uintptr_t)cb.src[j] % 16 == 0) && ((uintptr_t)cb.dst[j] % 16 == 0) && cb.words[j] % 2 == 0;
      most = std::max(most, cb.words[j]);
    }
    if (!most) continue;
    const size_t per = vec ? most / 2 : most;
    const unsigned bx = (unsigned)std::min<size_t>((per + 1023) / 1024, 1024);
    ProfScope _prof("k_copy_batch", st);
    if (vec) hipLaunchKernelGGL(k_copy_batch<true>, dim3(bx, m), dim3(256), 0, st, cb);
    else hipLaunchKernelGGL(k_copy_batch<false>, dim3(bx, m), dim3(256), 0, st, cb);
    HS_CHECK_HIP(hipGetLastError());
  }
}

}  // namespace hs
