// Fixed device scratch of the allocation-free encrypted SpMV (hs_he_spmv_noalloc): every buffer of
// such a call (slot products, totalSum ping-pong ciphertexts, key-switch intermediates, item and
// argument arrays) is a slice of one file-scope device array.  Each GPU the library runs on holds
// its own copy of the array until the process ends; all calls on one GPU share it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "hs_internal.hpp"

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

}  // namespace hs
