// Scratch for the no-allocation entry point haf_batch_noalloc, and the kernel that builds its plan.
//
// The scratch is a file-scope device array: each GPU the library runs on holds its own copy for the
// life of the process. Host code never uses the array's name as an address; it takes the device
// address once per device with hipGetSymbolAddress (that device current) and passes that pointer.
#include <hip/hip_runtime.h>

#include <mutex>

#include "gbs_internal.h"

namespace gbs {

constexpr size_t kNoallocScratchBytes = size_t(32) << 20;  // 32 MiB per device

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

size_t noalloc_scratch_bytes() { return kNoallocScratchBytes; }

void* noalloc_scratch(int device, hipError_t* err) {
  *err = hipSuccess;
  if (device < 0 || device >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return g_scratch_ptr[device];
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) prev = -1;
  if (prev != device) {
    *err = hipSetDevice(device);
    if (*err != hipSuccess) return nullptr;
  }
  void* p = nullptr;
  *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
  if (*err != hipSuccess) return nullptr;
  g_scratch_ptr[device] = p;
  return p;
}

// One thread per item (and per pattern for the per-pattern arrays).
__global__ void noalloc_plan_kernel(NoallocPlanArgs a) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < a.total_items; i += stride) {
    int g = 0;
    while (g + 1 < a.n_groups && i >= a.g[g + 1].first) ++g;
    const NoallocGroup G = a.g[g];
    const int64_t r = i - G.first;
    const int64_t p = r / G.count;
    const int64_t j = r - p * G.count;
    WorkItem w;
    w.lo = G.a + j * G.chunk;
    w.hi = w.lo + G.chunk < G.b ? w.lo + G.chunk : G.b;
    w.pattern = (int32_t)p;
    w.partial = (int32_t)(p * a.ipp + G.local_base + j);
    a.items[i] = w;
  }
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p <= a.batch; p += stride) {
    a.part_off[p] = p * a.ipp;
    if (p < a.batch) {
      PatternDesc d;
      d.src = p * a.stride;
      d.n = a.n;
      d.pad = 0;
      a.pats[p] = d;
      a.nvec[p] = a.n;
      a.sfact[p] = 1.0;
    }
  }
}

void launch_noalloc_plan(const NoallocPlanArgs& a, hipStream_t s) {
  const int64_t work = a.total_items > a.batch + 1 ? a.total_items : a.batch + 1;
  int64_t blocks = (work + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(noalloc_plan_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
}

}  // namespace gbs
