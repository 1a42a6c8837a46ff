// Workspace binding kernels: relocation of a plan's item image into a device binding and the
// fill of the binding's ranges that must read as zero (or, for diagnostics, as NaN); the static
// workspace of the allocation-free solve.
//
// The item image holds workspace addresses as kVBase + offset; a binding at device address B
// holds the same image with every such word moved by (B - kVBase).  The image is copied by the
// host (a device-to-device copy) and the listed words are patched here, so binding needs no host
// staging and no allocation.
#include <mutex>

#include "plan.hpp"

namespace lgf {

namespace {

// Workspace of the allocation-free solve (lgf_solve_noalloc): a static device array, one copy per
// GPU the library runs on, held until the process ends.  Host code never uses the array's name
// as an address (on the host it is only a stand-in for the symbol): scratch_binding looks up
// each device's copy with hipGetSymbolAddress and hands out that pointer.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
Binding g_scratch[kMaxDevices];

__global__ __launch_bounds__(256) void relocate_kernel(uint64_t* img, const uint32_t* __restrict__ idx, int64_t n,
                                                       uint64_t delta) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const gview<uint64_t> q = gl(img);
  q[idx[i]] += delta;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// one row of workgroups per range; 16-byte stores, ranges are 16-byte multiples
__global__ __launch_bounds__(256) void fill_kernel(uint8_t* base, FillRanges r, uint32_t pattern) {
  const int k = blockIdx.y;
  if (k >= r.n) return;
  const gview<u32x4> q = gl((u32x4*)(base + r.off[k]));
  const int64_t words = r.bytes[k] / 16;
  const u32x4 v = {pattern, pattern, pattern, pattern};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
    q[i] = v;
}

}  // namespace

hipError_t scratch_binding(Binding** out) {
  int dev = 0;
  LGF_HIP_CHECK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  Binding& b = g_scratch[dev];
  if (!b.base) {
    void* ptr = nullptr;
    LGF_HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr || (uintptr_t)ptr % 256) return hipErrorInvalidSymbol;
    b.base = (uint8_t*)ptr;
    b.bytes = kScratchBytes;
    b.plan = nullptr;
    b.owned = false;
  }
  *out = &b;
  return hipSuccess;
}

hipError_t launch_relocate(uint64_t* img, const uint32_t* idx, int64_t n, uint64_t delta, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(relocate_kernel, dim3((unsigned)blocks), dim3(256), 0, st, img, idx, n, delta);
  return hipGetLastError();
}

hipError_t launch_fill(uint8_t* base, const FillRanges& r, uint32_t pattern, hipStream_t st) {
  if (r.n <= 0) return hipSuccess;
  int64_t most = 0;
  for (int k = 0; k < r.n; ++k) {
    if (r.off[k] % 16 || r.bytes[k] % 16) return hipErrorInvalidValue;
    most = std::max<int64_t>(most, r.bytes[k] / 16);
  }
  const int64_t gx = std::min<int64_t>(2048, (most + 255) / 256);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)std::max<int64_t>(gx, 1), (unsigned)r.n), dim3(256), 0, st, base, r,
                     pattern);
  return hipGetLastError();
}

}  // namespace lgf
