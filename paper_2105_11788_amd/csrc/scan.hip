// Exclusive prefix sum over uint32 (used for offset arrays during loading):
// a tile pass (256 threads x 8 items, wave64 shuffles + LDS for the
// cross-wave carry), a recursive scan of the tile totals, and an add pass.
#include "internal.h"

namespace bisim {

namespace {
constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;

__global__ void __launch_bounds__(kThreads) k_scan_tiles(const uint32_t* __restrict__ in,
                                                          uint32_t* __restrict__ out,
                                                          uint32_t* __restrict__ tile_sums,
                                                          int64_t count) {
  __shared__ uint32_t wsum[kThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
  uint32_t v[kItems];
  uint32_t acc = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    int64_t i = base + j;
    v[j] = i < count ? in[i] : 0u;
    acc += v[j];
  }
  const uint32_t incl = wave_incl_scan_u32(acc);
  const int w = threadIdx.x / kWave;
  if (lane() == kWave - 1) wsum[w] = incl;
  __syncthreads();
  uint32_t before = 0, total = 0;
#pragma unroll
  for (int q = 0; q < kThreads / kWave; ++q) {
    if (q < w) before += wsum[q];
    total += wsum[q];
  }
  uint32_t run = before + incl - acc;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    int64_t i = base + j;
    if (i < count) out[i] = run;
    run += v[j];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kThreads) k_scan_add(uint32_t* __restrict__ out,
                                                        const uint32_t* __restrict__ tile_off,
                                                        int64_t count) {
  const uint32_t add = tile_off[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    int64_t i = base + j;
    if (i < count) out[i] += add;
  }
}
}  // namespace

size_t exclusive_scan_scratch_bytes(int64_t count) {
  size_t total = 0;
  for (int64_t c = count; c > kTile;) {  // c needs two tiles or more
    const int64_t tiles = (c + kTile - 1) / kTile;
    total += (sizeof(uint32_t) * (size_t)tiles + 255) / 256 * 256;
    total += (sizeof(uint32_t) * (size_t)(tiles + 1) + 255) / 256 * 256;
    c = tiles;
  }
  return total;
}

bisim_status exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t count,
                                hipStream_t stream) {
  if (count <= 0) {
    BISIM_TRY_HIP(hipMemsetAsync(out, 0, sizeof(uint32_t), stream));
    return BISIM_OK;
  }
  const int64_t tiles = (count + kTile - 1) / kTile;
  if (tiles == 1) {
    // one tile: its total is the grand total; nothing left to carry
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(kThreads), 0, stream, in, out, out + count,
                       count);
    BISIM_TRY_HIP(hipGetLastError());
    return BISIM_OK;
  }
  // tiles >= 2: the recursion below runs on ceil(count / kTile) < count values
  uint32_t* sums = nullptr;
  uint32_t* offs = nullptr;
  BISIM_TRY_HIP(dev_alloc((void**)&sums, sizeof(uint32_t) * tiles, stream));
  BISIM_TRY_HIP(dev_alloc((void**)&offs, sizeof(uint32_t) * (tiles + 1), stream));
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)tiles), dim3(kThreads), 0, stream, in, out, sums,
                     count);
  BISIM_TRY_HIP(hipGetLastError());
  bisim_status st = exclusive_scan_u32(sums, offs, tiles, stream);
  if (st != BISIM_OK) return st;
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)tiles), dim3(kThreads), 0, stream, out, offs,
                     count);
  BISIM_TRY_HIP(hipGetLastError());
  BISIM_TRY_HIP(hipMemcpyAsync(out + count, offs + tiles, sizeof(uint32_t),
                               hipMemcpyDeviceToDevice, stream));
  BISIM_TRY_HIP(dev_free(sums, stream));
  BISIM_TRY_HIP(dev_free(offs, stream));
  return BISIM_OK;
}

}  // namespace bisim
