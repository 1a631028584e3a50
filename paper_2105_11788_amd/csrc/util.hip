// The library's device allocator (stream-ordered memory, or a caller's
// region for the allocation-free entry point) and a measurement helper: a
// plain streaming copy, used to measure the bandwidth the device actually
// sustains and to calibrate memory-traffic counters.
#include "internal.h"

namespace bisim {

static thread_local ArenaScope* g_arena = nullptr;

ArenaScope::ArenaScope(char* base, size_t capacity) : base_(base), cap_(capacity), outer_(g_arena) {
  g_arena = this;
}
ArenaScope::~ArenaScope() { g_arena = outer_; }
bool arena_active() { return g_arena != nullptr; }

hipError_t dev_alloc(void** p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  if (bytes == 0) bytes = 1;
  ArenaScope* a = g_arena;
  if (!a) return hipMallocAsync(p, bytes, s);
  const size_t at = (a->used_ + 255) & ~(size_t)255;
  if (at > a->cap_ || bytes > a->cap_ - at) return hipErrorOutOfMemory;
  *p = a->base_ + at;
  a->used_ = at + bytes;
  return hipSuccess;
}

hipError_t dev_free(void* p, hipStream_t s) {
  if (!p) return hipSuccess;
  for (ArenaScope* a = g_arena; a; a = a->outer_)
    if ((char*)p >= a->base_ && (char*)p < a->base_ + a->cap_) return hipSuccess;
  return hipFreeAsync(p, s);
}

namespace {
__global__ void __launch_bounds__(256) k_copy16(const uint4* __restrict__ src,
                                                uint4* __restrict__ dst, uint64_t n16) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    dst[i] = src[i];
}
}  // namespace
}  // namespace bisim

using namespace bisim;

extern "C" bisim_status bisim_device_copy(void* dst, const void* src, int64_t bytes,
                                          void* hip_stream, double* ms_out) {
  if (!dst || !src || bytes < 0 || (bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15)) {
    set_error("bisim_device_copy: 16-byte aligned pointers and a multiple of 16 bytes");
    return BISIM_E_INVALID;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  int dev = 0, cu = 0;
  BISIM_TRY_HIP(hipGetDevice(&dev));
  BISIM_TRY_HIP(hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev));
  const uint64_t n16 = (uint64_t)bytes / 16;
  uint64_t g = (n16 + 255) / 256;
  if (g > (uint64_t)cu * 32) g = (uint64_t)cu * 32;
  if (g < 1) g = 1;
  hipEvent_t e0, e1;
  BISIM_TRY_HIP(hipEventCreate(&e0));
  BISIM_TRY_HIP(hipEventCreate(&e1));
  BISIM_TRY_HIP(hipEventRecord(e0, s));
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)g), dim3(256), 0, s, (const uint4*)src, (uint4*)dst,
                     n16);
  BISIM_TRY_HIP(hipGetLastError());
  BISIM_TRY_HIP(hipEventRecord(e1, s));
  BISIM_TRY_HIP(hipEventSynchronize(e1));
  float ms = 0;
  BISIM_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (ms_out) *ms_out = ms;
  return BISIM_OK;
}
