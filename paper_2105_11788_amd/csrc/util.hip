// Measurement helper: a plain streaming copy, used to measure the bandwidth
// the device actually sustains and to calibrate memory-traffic counters.
#include "internal.h"

namespace bisim {
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
