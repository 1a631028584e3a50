// Multi-way signature refinement: the signature-based splitting used by the
// GPU systems the paper compares against in section 5 (there: Wijs' Wms),
// built here as an in-house baseline beside the paper's method.  It is not
// part of the paper's algorithms.
//
// From pi_pre (section 4.1), every round gives each state s the signature
// sig(s) = {(a, block(t)) : s -a-> t} and regroups the states by
// (block(s), sig(s)); a new block is named by its smallest state.  The round
// that changes nothing ends the run.  A round on the GPU:
//   1. key[e] = (source << 32) | (rank * n + block(target)) for every
//      transition (rank: the action's rank among the source's actions; within
//      a block of pi_pre, and so of every later partition, ranks name the same
//      actions, so (rank, block) pairs stand for (action, block) pairs);
//   2. radix sort of the keys, so equal (s, a, block) triples are adjacent;
//   3. sig(s) = sum over the distinct triples of a 64-bit hash of (rank,
//      block) (a set hash: duplicates count once), reduced per wave over the
//      sorted segments;
//   4. radix sort of the states by a hash of (block(s), sig(s)), stable in
//      the state index, so each run of equal hashes starts at its smallest
//      state; a max-scan of the run heads names every state's new block.
// Hashing can only merge states with different signatures, never separate
// equal ones, so the fixpoint is at least as coarse as the coarsest stable
// partition.  At the fixpoint every state's signature is hashed again with an
// independent seed and compared with its block leader's (and the pi_pre block
// with the leader's): if all agree the partition is stable and refines pi_0,
// hence it is the coarsest one; if not, the run is repeated with new seeds.
//
// The hybrid run (the combination of multi-way splitting with the linear
// bound that section 6 leaves open) stops the rounds after two consecutive
// ones that each add fewer than kHybridStall blocks, and continues with
// Algorithm 3 from the partition reached, every block unstable.  That
// partition refines pi_pre (checked) and is at least as coarse as the
// coarsest stable one, so Algorithm 3 ends in the same result.
#include <hipcub/hipcub.hpp>

#include "internal.h"

namespace bisim {
namespace {

constexpr int kT = 256;

// SplitMix64's output function (Steele, Lea and Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

#define SSTRIDE(i, count)                                                        \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (count); \
       i += (int64_t)gridDim.x * blockDim.x)

__global__ void k_targets(int32_t n, const uint32_t* __restrict__ in_ptr,
                          int32_t* __restrict__ tgt) {
  SSTRIDE(t, (int64_t)n) {
    for (uint32_t e = in_ptr[t]; e < in_ptr[t + 1]; ++e) tgt[e] = (int32_t)t;
  }
}

__global__ void k_keys(int64_t m, uint32_t n, const int32_t* __restrict__ in_src,
                       const int32_t* __restrict__ in_ord, const int32_t* __restrict__ tgt,
                       const int32_t* __restrict__ blk, uint64_t* __restrict__ key) {
  SSTRIDE(e, m) {
    key[e] = ((uint64_t)(uint32_t)in_src[e] << 32) |
             (uint32_t)((uint32_t)in_ord[e] * n + (uint32_t)blk[tgt[e]]);
  }
}

// sig[s] += hash(rank, block) over the distinct sorted keys of source s; one
// atomic per segment piece within a wave (all lanes of a wave reach the
// shuffles).
__global__ void __launch_bounds__(kT) k_sig_sum(int64_t m, const uint64_t* __restrict__ key,
                                                uint64_t seed, uint64_t* __restrict__ sig) {
  const int64_t waves = (int64_t)gridDim.x * (kT / kWave);
  const int64_t gw = (int64_t)blockIdx.x * (kT / kWave) + threadIdx.x / kWave;
  const int l = (int)lane();
  for (int64_t base = gw * kWave; base < m; base += waves * kWave) {
    const int64_t e = base + l;
    const bool valid = e < m;
    const uint64_t k = valid ? key[e] : ~0ull;
    const uint64_t kp = (valid && e > 0) ? key[e - 1] : ~0ull;
    const bool distinct = valid && (e == 0 || k != kp);
    const uint32_t s = (uint32_t)(k >> 32);
    uint64_t v = distinct ? mix64((k & 0xFFFFFFFFull) + seed) : 0ull;
    const uint32_t s_next = (uint32_t)__shfl_down((int)s, 1, kWave);
    const bool tail = valid && (l == kWave - 1 || !(e + 1 < m) || s_next != s);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {  // inclusive prefix sum (mod 2^64)
      const uint64_t t = (uint64_t)__shfl_up((unsigned long long)v, d, kWave);
      if (l >= d) v += t;
    }
    const uint64_t tails = __ballot(tail);
    const uint64_t below = tails & ((1ull << l) - 1ull);
    const int prev = below ? 63 - __clzll((long long)below) : -1;
    const uint64_t pv = (uint64_t)__shfl((unsigned long long)v, prev < 0 ? 0 : prev, kWave);
    if (tail) atomicAdd((unsigned long long*)&sig[s], (unsigned long long)(v - (prev < 0 ? 0ull : pv)));
  }
}

__global__ void k_state_keys(int32_t n, const int32_t* __restrict__ blk,
                             const uint64_t* __restrict__ sig, uint64_t* __restrict__ hk,
                             int32_t* __restrict__ idx) {
  SSTRIDE(s, (int64_t)n) {
    hk[s] = mix64(sig[s] ^ mix64((uint64_t)(uint32_t)blk[s] + 0x9E3779B97F4A7C15ull));
    idx[s] = (int32_t)s;
  }
}

__global__ void __launch_bounds__(kT) k_heads(int32_t n, const uint64_t* __restrict__ hs,
                                              int32_t* __restrict__ hp,
                                              unsigned long long* __restrict__ count) {
  uint32_t c = 0;
  SSTRIDE(i, (int64_t)n) {
    const bool head = i == 0 || hs[i] != hs[i - 1];
    hp[i] = head ? (int32_t)i : 0;
    c += head;
  }
  atomicAdd(count, (unsigned long long)c);
}

__global__ void k_assign(int32_t n, const int32_t* __restrict__ idxs,
                         const int32_t* __restrict__ hp, int32_t* __restrict__ nb) {
  SSTRIDE(i, (int64_t)n) { nb[idxs[i]] = idxs[hp[i]]; }
}

// bad += states whose block leader is not its own leader, lies in another
// block of pi_pre, or (stable) has another signature hash
__global__ void __launch_bounds__(kT) k_check(int32_t n, const int32_t* __restrict__ blk,
                                              const int32_t* __restrict__ pre,
                                              const uint64_t* __restrict__ sig2, int stable,
                                              unsigned long long* __restrict__ bad) {
  uint32_t c = 0;
  SSTRIDE(s, (int64_t)n) {
    const int32_t l = blk[s];
    c += (stable && sig2[s] != sig2[l]) || (pre[s] != pre[l]) || (blk[l] != l);
  }
  if (c) atomicAdd(bad, (unsigned long long)c);
}

unsigned grid_of(int64_t work, int cu) {
  const int64_t g = (work + kT - 1) / kT;
  const int64_t cap = (int64_t)cu * 16;
  return (unsigned)(g < 1 ? 1 : (g > cap ? cap : g));
}

// device buffers of one run, freed on every exit
struct Bufs {
  hipStream_t st;
  void* p[16] = {};
  int k = 0;
  ~Bufs() {
    for (int i = 0; i < k; ++i) (void)hipFreeAsync(p[i], st);
  }
  template <class T>
  bisim_status get(T** out, size_t count) {
    void* q = nullptr;
    if (count == 0) count = 1;
    if (k == 16) {
      set_error("signature refinement: too many buffers");
      return BISIM_E_INVALID;
    }
    if (hipMallocAsync(&q, sizeof(T) * count, st) != hipSuccess) {
      set_error("signature refinement: out of device memory (%zu bytes)", sizeof(T) * count);
      return BISIM_E_NOMEM;
    }
    p[k++] = q;
    *out = (T*)q;
    return BISIM_OK;
  }
};

}  // namespace

constexpr int64_t kHybridStall = 64;

// Signature rounds from pi_pre into out (device int32[n]): to the fixpoint
// (stall = 0), or until two consecutive rounds each add fewer than stall
// blocks.  Reports the rounds run, the blocks reached, whether the last round
// changed nothing, and the time (ms).  Needs n > 0.
bisim_status signature_core(bisim_lts* h, int64_t stall, int32_t* out, int64_t* rounds_out,
                            int64_t* blocks_out, bool* fixpoint_out, double* ms_out) {
  hipStream_t st = h->stream;
  const int32_t n = h->n;
  const int64_t m = h->m;
  if (m >= (1ll << 31) || (uint64_t)h->max_ranks * (uint64_t)n > 0xFFFFFFFFull) {
    set_error("signature refinement: needs m < 2^31 and (actions per state) * n < 2^32");
    return BISIM_E_UNSUPPORTED;
  }
  const int cu = h->num_cu;
  Bufs b{st};
  int32_t *tgt, *blk, *nb, *idx, *idxs, *hp, *hp2;
  uint64_t *key, *keys, *sig, *hk, *hks;
  unsigned long long* cnt;
  BISIM_TRY(b.get(&tgt, (size_t)m));
  BISIM_TRY(b.get(&key, (size_t)m));
  BISIM_TRY(b.get(&keys, (size_t)m));
  BISIM_TRY(b.get(&blk, (size_t)n));
  BISIM_TRY(b.get(&nb, (size_t)n));
  BISIM_TRY(b.get(&idx, (size_t)n));
  BISIM_TRY(b.get(&idxs, (size_t)n));
  BISIM_TRY(b.get(&hp, (size_t)n));
  BISIM_TRY(b.get(&hp2, (size_t)n));
  BISIM_TRY(b.get(&sig, (size_t)n));
  BISIM_TRY(b.get(&hk, 2 * (size_t)n));
  BISIM_TRY(b.get(&cnt, 2));
  hks = hk + n;

  int kbits = 1;  // bits of the source index in the key's high half
  while (kbits < 31 && (1ll << kbits) < n) ++kbits;
  size_t t1 = 0, t2 = 0, t3 = 0;
  BISIM_TRY_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, t1, key, keys, (int)m, 0, 32 + kbits, st));
  BISIM_TRY_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, t2, hk, hks, idx, idxs, n, 0, 64, st));
  BISIM_TRY_HIP(hipcub::DeviceScan::InclusiveScan(nullptr, t3, hp, hp2, hipcub::Max(), n, st));
  size_t tb = t1 > t2 ? t1 : t2;
  if (t3 > tb) tb = t3;
  uint8_t* temp;
  BISIM_TRY(b.get(&temp, tb));

  if (m > 0) hipLaunchKernelGGL(k_targets, dim3(grid_of(n, cu)), dim3(kT), 0, st, n, h->in_ptr, tgt);
  BISIM_TRY_HIP(hipGetLastError());
  BISIM_TRY_HIP(hipEventRecord(h->ev0, st));
  int64_t rounds = 0;
  unsigned long long blocks = (unsigned long long)h->pre_blocks;
  bool fixpoint = false;
  uint64_t seed = 0x2545F4914F6CDD1Dull;
  for (int attempt = 0;; ++attempt) {
    BISIM_TRY_HIP(hipMemcpyAsync(blk, h->pre_block, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
    blocks = (unsigned long long)h->pre_blocks;
    rounds = 0;
    bool prev_few = false;
    for (;;) {
      ++rounds;
      size_t tb1 = tb;
      if (m > 0) {
        hipLaunchKernelGGL(k_keys, dim3(grid_of(m, cu)), dim3(kT), 0, st, m, (uint32_t)n,
                           h->in_src, h->in_ord, tgt, blk, key);
        BISIM_TRY_HIP(hipcub::DeviceRadixSort::SortKeys(temp, tb1, key, keys, (int)m, 0,
                                                       32 + kbits, st));
      }
      BISIM_TRY_HIP(hipMemsetAsync(sig, 0, sizeof(uint64_t) * n, st));
      if (m > 0)
        hipLaunchKernelGGL(k_sig_sum, dim3(grid_of(m, cu)), dim3(kT), 0, st, m, keys, seed, sig);
      hipLaunchKernelGGL(k_state_keys, dim3(grid_of(n, cu)), dim3(kT), 0, st, n, blk, sig, hk, idx);
      tb1 = tb;
      BISIM_TRY_HIP(hipcub::DeviceRadixSort::SortPairs(temp, tb1, hk, hks, idx, idxs, n, 0, 64, st));
      BISIM_TRY_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), st));
      hipLaunchKernelGGL(k_heads, dim3(grid_of(n, cu)), dim3(kT), 0, st, n, hks, hp, cnt);
      tb1 = tb;
      BISIM_TRY_HIP(hipcub::DeviceScan::InclusiveScan(temp, tb1, hp, hp2, hipcub::Max(), n, st));
      hipLaunchKernelGGL(k_assign, dim3(grid_of(n, cu)), dim3(kT), 0, st, n, idxs, hp2, nb);
      BISIM_TRY_HIP(hipGetLastError());
      unsigned long long c = 0;
      BISIM_TRY_HIP(hipMemcpyAsync(&c, cnt, sizeof(c), hipMemcpyDeviceToHost, st));
      BISIM_TRY_HIP(hipStreamSynchronize(st));
      int32_t* t = blk;
      blk = nb;
      nb = t;
      if (c == blocks) {  // new refines old: same count, same partition
        fixpoint = true;
        break;
      }
      const bool few = (int64_t)(c - blocks) < stall;
      blocks = c;
      if (stall > 0 && few && prev_few) {
        fixpoint = false;
        break;
      }
      prev_few = few;
      if (rounds > (int64_t)n + 1) {
        set_error("signature refinement: no fixpoint after %lld rounds", (long long)rounds);
        return BISIM_E_DEVICE;
      }
    }
    // check with an independent hash (at the fixpoint the keys still hold the
    // final partition's), or, after a stall, only that pi_pre is refined
    BISIM_TRY_HIP(hipMemsetAsync(sig, 0, sizeof(uint64_t) * n, st));
    BISIM_TRY_HIP(hipMemsetAsync(cnt + 1, 0, sizeof(unsigned long long), st));
    if (m > 0 && fixpoint)
      hipLaunchKernelGGL(k_sig_sum, dim3(grid_of(m, cu)), dim3(kT), 0, st, m, keys,
                         seed ^ 0xD1B54A32D192ED03ull, sig);
    hipLaunchKernelGGL(k_check, dim3(grid_of(n, cu)), dim3(kT), 0, st, n, blk, h->pre_block, sig,
                       fixpoint ? 1 : 0, cnt + 1);
    BISIM_TRY_HIP(hipGetLastError());
    unsigned long long bad = 0;
    BISIM_TRY_HIP(hipMemcpyAsync(&bad, cnt + 1, sizeof(bad), hipMemcpyDeviceToHost, st));
    BISIM_TRY_HIP(hipStreamSynchronize(st));
    if (bad == 0) break;
    if (attempt == 2) {
      set_error("signature refinement: hash check failed three times");
      return BISIM_E_DEVICE;
    }
    seed = seed * 6364136223846793005ull + 1442695040888963407ull;
  }
  BISIM_TRY_HIP(hipEventRecord(h->ev1, st));
  BISIM_TRY_HIP(hipMemcpyAsync(out, blk, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
  BISIM_TRY_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  BISIM_TRY_HIP(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  *ms_out = ms;
  *rounds_out = rounds;
  *blocks_out = (int64_t)blocks;
  *fixpoint_out = fixpoint;
  return BISIM_OK;
}

bisim_status signature_run(bisim_lts* h, int32_t* block_id, bool hybrid) {
  h->run_pre_blocks = h->pre_blocks;
  h->last_iters = 0;
  h->last_blocks = h->pre_blocks;
  h->t_alg_ms = 0.0;
  if ((h->policy == 1 && h->policy_w) || h->trace_cap > 0) {
    set_error("signature refinement has no splitter: no splitter policy or trace");
    return BISIM_E_UNSUPPORTED;
  }
  if (h->n == 0) return BISIM_OK;
  int64_t rounds = 0, blocks = 0;
  bool fixpoint = false;
  double ms = 0.0;
  BISIM_TRY(signature_core(h, hybrid ? kHybridStall : 0, block_id, &rounds, &blocks, &fixpoint,
                           &ms));
  if (!fixpoint) {  // continue with Algorithm 3 from the partition in block_id
    h->start_override = block_id;
    h->start_override_blocks = blocks;
    const bisim_status rc = refine_run(h, block_id);
    h->start_override = nullptr;
    h->start_override_blocks = 0;
    h->run_pre_blocks = h->pre_blocks;
    BISIM_TRY(rc);
    h->last_iters += rounds;
    h->t_alg_ms += ms;
    return BISIM_OK;
  }
  h->t_alg_ms = ms;
  h->last_iters = rounds;
  h->last_blocks = blocks;
  return BISIM_OK;
}

}  // namespace bisim
