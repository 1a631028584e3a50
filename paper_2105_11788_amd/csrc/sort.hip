// Stable least-significant-digit radix sort of 64-bit keys (optionally with
// 32-bit values) and an inclusive max-scan, for the signature baseline's
// regrouping rounds.
//
// A pass sorts by one 8-bit digit.  The input is cut into tiles of kSortTile
// elements.  A histogram kernel counts each tile's digits into a digit-major
// table (count[digit * tiles + tile]); one exclusive scan of that table gives
// every (digit, tile) pair its first output position; a scatter kernel sorts
// its tile by the digit in LDS and writes it out.  In the scatter kernel each
// wave owns a contiguous quarter of the tile: it walks its part in rounds
// of 64 elements, the lanes holding one digit find each other with eight
// ballots, and a per-wave, per-digit running count gives every element its
// rank among the equal digits before it in the wave.  The waves' counts are
// then combined in wave order and the tile's digit starts taken by one block
// scan, so an element's place in the tile is (digit start) + (earlier waves)
// + (its rank): input order is kept among equal digits.  The sorted tile goes
// out with consecutive threads on consecutive positions of one digit's run,
// so the writes coalesce.  Equal digits of different tiles keep the tiles'
// order through the table.  Up to kFuseTiles tiles the scatter kernel reads
// its positions off the table itself and the scan is skipped; inputs of at
// most kSmallMax elements take one single-workgroup launch for all passes.
#include "internal.h"

namespace bisim {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kDigits = 256;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr int kDigitWaves = kDigits / kWave;  // the waves whose threads own a digit each
constexpr uint32_t kFuseTiles = 64;  // up to this many tiles, no separate offset scan
static_assert(kSortThreads >= kDigits, "a thread per digit");

__device__ __forceinline__ uint32_t digit_of(uint64_t k, int shift) {
  return (uint32_t)(k >> shift) & (kDigits - 1);
}

// exclusive scan of one value per digit over threads t < kDigits (all threads
// of the workgroup call it; `sum` holds kDigitWaves words of LDS)
__device__ __forceinline__ uint32_t digit_excl_scan(uint32_t x, uint32_t* sum) {
  const uint32_t t = threadIdx.x, w = t / kWave;
  uint32_t incl = 0;
  if (t < kDigits) {
    incl = wave_incl_scan_u32(x);
    if (lane() == kWave - 1) sum[w] = incl;
  }
  __syncthreads();
  uint32_t before = 0;
  if (t < kDigits) {
#pragma unroll
    for (int q = 0; q < kDigitWaves; ++q)
      if (q < (int)w) before += sum[q];
  }
  return before + incl - x;
}

__global__ void __launch_bounds__(kSortThreads) k_rs_hist(const uint64_t* __restrict__ keys,
                                                          int64_t count, int shift,
                                                          uint32_t* __restrict__ table,
                                                          uint32_t tiles) {
  __shared__ uint32_t h[2][kDigits];  // one per half of the workgroup
  const uint32_t t = threadIdx.x;
  for (uint32_t c = t; c < 2u * kDigits; c += kSortThreads) (&h[0][0])[c] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  uint32_t* hh = h[t < kSortThreads / 2 ? 0 : 1];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + (int64_t)r * kSortThreads + t;
    if (i < count) atomicAdd(&hh[digit_of(keys[i], shift)], 1u);
  }
  __syncthreads();
  if (t < kDigits) table[(size_t)t * tiles + blockIdx.x] = h[0][t] + h[1][t];
}

template <bool kVals>
__global__ void __launch_bounds__(kSortThreads) k_rs_scatter(
    const uint64_t* __restrict__ keys, const uint32_t* __restrict__ vals, int64_t count,
    int shift, const uint32_t* __restrict__ offsets, const uint32_t* __restrict__ table,
    uint32_t tiles, uint64_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out) {
  __shared__ uint64_t sk[kSortTile];
  __shared__ uint32_t sv[kVals ? kSortTile : 1];
  __shared__ uint32_t wcnt[kSortWaves][kDigits];  // per wave and digit: count, then start
  __shared__ uint32_t lstart[kDigits];            // digit's first place in the sorted tile
  __shared__ uint32_t goff[kDigits];              // digit's first output position
  __shared__ uint32_t wsum[kDigitWaves];
  const uint32_t t = threadIdx.x, w = t / kWave, ln = lane();
  for (uint32_t c = t; c < (uint32_t)(kSortWaves * kDigits); c += kSortThreads)
    (&wcnt[0][0])[c] = 0;
  if (offsets) {
    if (t < kDigits) goff[t] = offsets[(size_t)t * tiles + blockIdx.x];
  } else {
    // few tiles: take the position from the histogram table directly (the
    // digits before t over all tiles, then digit t over the tiles before)
    uint32_t tot = 0, mine = 0;
    if (t < kDigits) {
      for (uint32_t u = 0; u < tiles; ++u) {
        const uint32_t c = table[(size_t)t * tiles + u];
        mine += u < blockIdx.x ? c : 0u;
        tot += c;
      }
    }
    const uint32_t ex = digit_excl_scan(tot, wsum);
    if (t < kDigits) goff[t] = ex + mine;
  }
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const int64_t wbase = base + (int64_t)w * (kSortItems * kWave);
  const uint64_t lt = (1ull << ln) - 1ull;
  uint64_t k[kSortItems];
  uint32_t v[kSortItems], rk[kSortItems];
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = wbase + (int64_t)r * kWave + ln;
    const bool valid = i < count;
    k[r] = valid ? keys[i] : 0ull;
    v[r] = (kVals && valid) ? vals[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const bool valid = wbase + (int64_t)r * kWave + ln < count;
    const uint32_t d = digit_of(k[r], shift);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? bal : ~bal;
    }
    const uint32_t below = (uint32_t)__popcll(peers & lt);
    // the wave's own row: every lane reads its digit's count, then the first
    // lane of each digit group adds the group (the add depends on the read)
    const uint32_t prior = wcnt[w][d];
    rk[r] = prior + below;
    if (valid && below == 0) wcnt[w][d] = prior + (uint32_t)__popcll(peers);
  }
  __syncthreads();
  // thread t < kDigits owns digit t: the starts of each wave's run, the tile's total
  uint32_t tot = 0;
  if (t < kDigits) {
#pragma unroll
    for (int q = 0; q < kSortWaves; ++q) {
      const uint32_t c = wcnt[q][t];
      wcnt[q][t] = tot;
      tot += c;
    }
  }
  const uint32_t ex = digit_excl_scan(tot, wsum);
  if (t < kDigits) lstart[t] = ex;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = wbase + (int64_t)r * kWave + ln;
    if (i < count) {
      const uint32_t d = digit_of(k[r], shift);
      const uint32_t lp = lstart[d] + wcnt[w][d] + rk[r];
      sk[lp] = k[r];
      if (kVals) sv[lp] = v[r];
    }
  }
  __syncthreads();
  const int64_t left = count - base;
  const uint32_t nt = left < kSortTile ? (uint32_t)left : (uint32_t)kSortTile;
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const uint32_t j = (uint32_t)r * kSortThreads + t;
    if (j < nt) {
      const uint64_t key = sk[j];
      const uint32_t d = digit_of(key, shift);
      const uint32_t pos = goff[d] + (j - lstart[d]);
      keys_out[pos] = key;
      if (kVals) vals_out[pos] = sv[j];
    }
  }
}

// Inputs of at most kSmallMax elements are sorted by one workgroup in one
// launch (a chain of launches per digit costs more than the work).  Every
// wave owns a contiguous stretch of the input, held in registers during a
// pass; it ranks its elements round by round with a per-wave, per-digit count
// as the multi-workgroup scatter does, the counts of all waves are then
// combined in wave order and scanned over the digits (the whole input is one
// tile, so no histogram pass is needed), and the elements go straight to
// their places.  The passes hand their output on through global memory; the
// workgroup barrier orders those writes before the next pass reads them.
// The per-wave counts alternate between two buffers, one cleared while the
// other is in use.  Up to kSmallLdsMax elements the passes between the first
// and the last read and write LDS instead (every element sits in registers
// between its read and its write, and barriers separate the two).
constexpr int kSmallThreads = 1024;
constexpr int kSmallWaves = kSmallThreads / kWave;
constexpr int kSmallRounds = 16;
constexpr int64_t kSmallMax = (int64_t)kSmallThreads * kSmallRounds;
constexpr int kSmallLdsMax = 10240;  // up to this many elements the passes stay in LDS

template <bool kVals, bool kLds>
__global__ void __launch_bounds__(kSmallThreads) k_rs_small(
    const uint64_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, int32_t count,
    int begin_bit, int passes, uint64_t* keys_out, uint32_t* vals_out, uint64_t* ktmp,
    uint32_t* vtmp) {
  __shared__ uint32_t wcnt[2][kSmallWaves][kDigits];
  __shared__ uint32_t dstart[kDigits];  // digit's first output position
  __shared__ uint32_t wsum[kDigits / kWave];
  // kLds: the passes between the first and the last keep the data in LDS
  __shared__ uint64_t lk[kLds ? kSmallLdsMax : 1];
  __shared__ uint32_t lv[kLds && kVals ? kSmallLdsMax : 1];
  const uint32_t t = threadIdx.x, w = t / kWave, ln = lane();
  const uint64_t lt = (1ull << ln) - 1ull;
  for (uint32_t c = t; c < (uint32_t)(2 * kSmallWaves * kDigits); c += kSmallThreads)
    (&wcnt[0][0][0])[c] = 0;
  __syncthreads();
  // elements per wave: a multiple of the wave size, at most kSmallRounds waves' worth
  const int32_t per = ((count + kSmallWaves - 1) / kSmallWaves + kWave - 1) / kWave * kWave;
  const int rounds = per / kWave;
  const int32_t wbase = (int32_t)w * per;
  const uint64_t* ks = keys_in;
  const uint32_t* vs = vals_in;
  for (int p = 0; p < passes; ++p) {
    uint32_t(*cnt)[kDigits] = wcnt[p & 1];
    const bool to_out = ((passes - p) & 1) == 1;  // the last pass writes keys_out
    uint64_t* kd = to_out ? keys_out : ktmp;
    uint32_t* vd = to_out ? vals_out : vtmp;
    const int shift = begin_bit + 8 * p;
    uint64_t k[kSmallRounds];
    uint32_t v[kSmallRounds], rk[kSmallRounds];
#pragma unroll
    for (int r = 0; r < kSmallRounds; ++r) {
      const int32_t i = wbase + r * kWave + (int32_t)ln;
      const bool valid = r < rounds && i < count;
      if (kLds && p > 0) {
        k[r] = valid ? lk[i] : 0ull;
        v[r] = (kVals && valid) ? lv[i] : 0u;
      } else {
        k[r] = valid ? ks[i] : 0ull;
        v[r] = (kVals && valid) ? vs[i] : 0u;
      }
    }
#pragma unroll
    for (int r = 0; r < kSmallRounds; ++r) {
      if (r < rounds) {  // uniform over the workgroup
        const bool valid = wbase + r * kWave + (int32_t)ln < count;
        const uint32_t d = digit_of(k[r], shift);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const uint64_t bal = __ballot((d >> b) & 1u);
          peers &= ((d >> b) & 1u) ? bal : ~bal;
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt);
        const uint32_t prior = cnt[w][d];  // the wave's own row; the add depends on the read
        rk[r] = prior + below;
        if (valid && below == 0) cnt[w][d] = prior + (uint32_t)__popcll(peers);
      }
    }
    __syncthreads();
    uint32_t tot = 0, incl = 0;
    if (t < kDigits) {
#pragma unroll
      for (int q = 0; q < kSmallWaves; ++q) {
        const uint32_t c = cnt[q][t];
        cnt[q][t] = tot;
        tot += c;
        wcnt[(p & 1) ^ 1][q][t] = 0;
      }
      incl = wave_incl_scan_u32(tot);
      if (ln == kWave - 1) wsum[w] = incl;
    }
    __syncthreads();
    if (t < kDigits) {
      uint32_t before = 0;
#pragma unroll
      for (int q = 0; q < kDigits / kWave; ++q)
        if (q < (int)w) before += wsum[q];
      dstart[t] = before + incl - tot;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSmallRounds; ++r) {
      if (r < rounds && wbase + r * kWave + (int32_t)ln < count) {
        const uint32_t d = digit_of(k[r], shift);
        const uint32_t pos = dstart[d] + cnt[w][d] + rk[r];
        if (kLds && p + 1 < passes) {
          lk[pos] = k[r];
          if (kVals) lv[pos] = v[r];
        } else {
          kd[pos] = k[r];
          if (kVals) vd[pos] = v[r];
        }
      }
    }
    __syncthreads();
    ks = kd;
    vs = vd;
  }
}

// inclusive max-scan: per tile, then the tiles' maxima, then the carry
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ uint32_t wave_incl_max_u32(uint32_t v) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t u = (uint32_t)__shfl_up((int)v, d, kWave);
    if ((int)lane() >= d) v = max(v, u);
  }
  return v;
}

__global__ void __launch_bounds__(kScanThreads) k_maxscan_tiles(const uint32_t* __restrict__ in,
                                                                uint32_t* __restrict__ out,
                                                                uint32_t* __restrict__ tile_max,
                                                                int64_t count) {
  __shared__ uint32_t wmax[kScanThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  uint32_t v[kScanItems];
  uint32_t acc = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int64_t i = base + j;
    v[j] = i < count ? in[i] : 0u;
    acc = max(acc, v[j]);
  }
  const uint32_t incl = wave_incl_max_u32(acc);
  const uint32_t excl = (uint32_t)__shfl_up((int)incl, 1, kWave);
  const int w = threadIdx.x / kWave;
  if (lane() == kWave - 1) wmax[w] = incl;
  __syncthreads();
  uint32_t before = 0, total = 0;
#pragma unroll
  for (int q = 0; q < kScanThreads / kWave; ++q) {
    if (q < w) before = max(before, wmax[q]);
    total = max(total, wmax[q]);
  }
  uint32_t m = max(before, lane() > 0 ? excl : 0u);
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int64_t i = base + j;
    m = max(m, v[j]);
    if (i < count) out[i] = m;
  }
  if (threadIdx.x == 0) tile_max[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanThreads) k_maxscan_carry(uint32_t* __restrict__ out,
                                                                const uint32_t* __restrict__ tmax,
                                                                int64_t count) {
  if (blockIdx.x == 0) return;
  const uint32_t c = tmax[blockIdx.x - 1];  // inclusive max of the tiles before
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const int64_t i = base + j;
    if (i < count) out[i] = max(out[i], c);
  }
}

// one workgroup over at most kSmallMax values, in chunks with a carry
__global__ void __launch_bounds__(kSmallThreads) k_maxscan_small(const uint32_t* __restrict__ in,
                                                                 uint32_t* __restrict__ out,
                                                                 int32_t count) {
  __shared__ uint32_t wmax[kSmallWaves];
  const uint32_t t = threadIdx.x, w = t / kWave;
  uint32_t carry = 0;
  for (int32_t base = 0; base < count; base += kSmallThreads) {
    const int32_t i = base + (int32_t)t;
    const uint32_t x = i < count ? in[i] : 0u;
    const uint32_t incl = wave_incl_max_u32(x);
    if (lane() == kWave - 1) wmax[w] = incl;
    __syncthreads();
    uint32_t before = carry, total = carry;
#pragma unroll
    for (int q = 0; q < kSmallWaves; ++q) {
      if (q < (int)w) before = max(before, wmax[q]);
      total = max(total, wmax[q]);
    }
    if (i < count) out[i] = max(before, incl);
    carry = total;
    __syncthreads();
  }
}

}  // namespace

static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

size_t radix_sort_temp_bytes(int64_t count, bool with_values) {
  if (count <= 0) return 0;
  const size_t tiles = (size_t)((count + kSortTile - 1) / kSortTile);
  const size_t cells = (size_t)kDigits * tiles;
  size_t b = round256(sizeof(uint32_t) * cells) + round256(sizeof(uint32_t) * (cells + 1)) +
             round256(sizeof(uint64_t) * (size_t)count);
  if (with_values) b += round256(sizeof(uint32_t) * (size_t)count);
  return b;
}

bisim_status radix_sort_u64(void* temp, size_t temp_bytes, const uint64_t* keys_in,
                            uint64_t* keys_out, const uint32_t* vals_in, uint32_t* vals_out,
                            int64_t count, int begin_bit, int end_bit, hipStream_t st) {
  if (count <= 0) return BISIM_OK;
  if (count > (int64_t)0xFFFFFFFFll || begin_bit < 0 || end_bit > 64) {
    set_error("radix sort: more than 2^32 - 1 elements or a bit range outside [0, 64)");
    return BISIM_E_UNSUPPORTED;
  }
  const bool with_values = vals_in != nullptr;
  if (temp_bytes < radix_sort_temp_bytes(count, with_values)) {
    set_error("radix sort: %zu bytes of workspace, %zu needed", temp_bytes,
              radix_sort_temp_bytes(count, with_values));
    return BISIM_E_INVALID;
  }
  const int passes = (end_bit - begin_bit + 7) / 8;
  if (passes <= 0) {
    BISIM_TRY_HIP(hipMemcpyAsync(keys_out, keys_in, sizeof(uint64_t) * (size_t)count,
                                 hipMemcpyDeviceToDevice, st));
    if (with_values)
      BISIM_TRY_HIP(hipMemcpyAsync(vals_out, vals_in, sizeof(uint32_t) * (size_t)count,
                                   hipMemcpyDeviceToDevice, st));
    return BISIM_OK;
  }
  const uint32_t tiles = (uint32_t)((count + kSortTile - 1) / kSortTile);
  const size_t cells = (size_t)kDigits * tiles;
  char* p = (char*)temp;
  if (count <= kSmallMax) {
    uint64_t* kt = (uint64_t*)(p + round256(sizeof(uint32_t) * cells) +
                               round256(sizeof(uint32_t) * (cells + 1)));
    uint32_t* vt = (uint32_t*)((char*)kt + round256(sizeof(uint64_t) * (size_t)count));
    const bool lds = count <= kSmallLdsMax;
    if (with_values && lds)
      hipLaunchKernelGGL((k_rs_small<true, true>), dim3(1), dim3(kSmallThreads), 0, st, keys_in,
                         vals_in, (int32_t)count, begin_bit, passes, keys_out, vals_out, kt, vt);
    else if (with_values)
      hipLaunchKernelGGL((k_rs_small<true, false>), dim3(1), dim3(kSmallThreads), 0, st, keys_in,
                         vals_in, (int32_t)count, begin_bit, passes, keys_out, vals_out, kt, vt);
    else if (lds)
      hipLaunchKernelGGL((k_rs_small<false, true>), dim3(1), dim3(kSmallThreads), 0, st, keys_in,
                         (const uint32_t*)nullptr, (int32_t)count, begin_bit, passes, keys_out,
                         (uint32_t*)nullptr, kt, (uint32_t*)nullptr);
    else
      hipLaunchKernelGGL((k_rs_small<false, false>), dim3(1), dim3(kSmallThreads), 0, st, keys_in,
                         (const uint32_t*)nullptr, (int32_t)count, begin_bit, passes, keys_out,
                         (uint32_t*)nullptr, kt, (uint32_t*)nullptr);
    BISIM_TRY_HIP(hipGetLastError());
    return BISIM_OK;
  }
  uint32_t* table = (uint32_t*)p;
  p += round256(sizeof(uint32_t) * cells);
  uint32_t* offs = (uint32_t*)p;
  p += round256(sizeof(uint32_t) * (cells + 1));
  uint64_t* ktmp = (uint64_t*)p;
  p += round256(sizeof(uint64_t) * (size_t)count);
  uint32_t* vtmp = with_values ? (uint32_t*)p : nullptr;
  // ping-pong ending in keys_out: an odd number of passes starts there
  const uint64_t* ksrc = keys_in;
  const uint32_t* vsrc = vals_in;
  for (int q = 0; q < passes; ++q) {
    const bool to_out = ((passes - q) & 1) == 1;
    uint64_t* kdst = to_out ? keys_out : ktmp;
    uint32_t* vdst = with_values ? (to_out ? vals_out : vtmp) : nullptr;
    const int shift = begin_bit + 8 * q;
    hipLaunchKernelGGL(k_rs_hist, dim3(tiles), dim3(kSortThreads), 0, st, ksrc, count, shift,
                       table, tiles);
    BISIM_TRY_HIP(hipGetLastError());
    const uint32_t* o = nullptr;  // few tiles: the scatter reads the table itself
    if (tiles > kFuseTiles) {
      BISIM_TRY(exclusive_scan_u32(table, offs, (int64_t)cells, st));
      o = offs;
    }
    if (with_values)
      hipLaunchKernelGGL(k_rs_scatter<true>, dim3(tiles), dim3(kSortThreads), 0, st, ksrc, vsrc,
                         count, shift, o, table, tiles, kdst, vdst);
    else
      hipLaunchKernelGGL(k_rs_scatter<false>, dim3(tiles), dim3(kSortThreads), 0, st, ksrc,
                         (const uint32_t*)nullptr, count, shift, o, table, tiles, kdst,
                         (uint32_t*)nullptr);
    BISIM_TRY_HIP(hipGetLastError());
    ksrc = kdst;
    vsrc = vdst;
  }
  return BISIM_OK;
}

bisim_status inclusive_max_scan_u32(const uint32_t* in, uint32_t* out, int64_t count,
                                    hipStream_t st) {
  if (count <= 0) return BISIM_OK;
  if (count <= kSmallMax) {
    hipLaunchKernelGGL(k_maxscan_small, dim3(1), dim3(kSmallThreads), 0, st, in, out,
                       (int32_t)count);
    BISIM_TRY_HIP(hipGetLastError());
    return BISIM_OK;
  }
  const int64_t tiles = (count + kScanTile - 1) / kScanTile;
  uint32_t* tmax = nullptr;
  BISIM_TRY_HIP(dev_alloc((void**)&tmax, sizeof(uint32_t) * (size_t)tiles, st));
  hipLaunchKernelGGL(k_maxscan_tiles, dim3((unsigned)tiles), dim3(kScanThreads), 0, st, in, out,
                     tmax, count);
  BISIM_TRY_HIP(hipGetLastError());
  bisim_status rc = BISIM_OK;
  if (tiles > 1) {
    uint32_t* tmax2 = nullptr;
    BISIM_TRY_HIP(dev_alloc((void**)&tmax2, sizeof(uint32_t) * (size_t)tiles, st));
    rc = inclusive_max_scan_u32(tmax, tmax2, tiles, st);
    if (rc == BISIM_OK) {
      hipLaunchKernelGGL(k_maxscan_carry, dim3((unsigned)tiles), dim3(kScanThreads), 0, st, out,
                         tmax2, count);
      if (hipGetLastError() != hipSuccess) rc = BISIM_E_DEVICE;
    }
    (void)dev_free(tmax2, st);
  }
  (void)dev_free(tmax, st);
  return rc;
}

}  // namespace bisim
