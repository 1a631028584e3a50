// Loading and preprocessing (section 4.1), all on the device:
//   1. validate ranges;
//   2. bucket transitions by action (LDS-privatised counting for K <= 4096);
//   3. leaders of pi_0: the smallest state of each initial class;
//   4. Algorithm 4, one round per action a that occurs: mark the sources of
//      a-transitions, split states whose mark differs from their leader's,
//      the smallest such state leading the split-off part.  The same round
//      hands every a-transition its slot rank order_i = the number of
//      distinct actions of its source below a (the rank that the
//      (source, action) sort plus Algorithm 5's segmented scan computes);
//   5. nr_marks, mark_length, and the packing of mark slots into 64-bit words;
//   6. transitions regrouped by target (CSR), carrying (source, order), so
//      that the mark step can visit the in-transitions of the splitter's
//      members instead of testing all m targets.
#include <cstdlib>
#include <vector>

#include "internal.h"

namespace bisim {

namespace {
constexpr int kT = 256;
constexpr int kLdsLabels = 4096;
constexpr int kChunk = kT * 16;

inline unsigned grid_for(int64_t work, int num_cu) {
  int64_t g = (work + kT - 1) / kT;
  int64_t cap = (int64_t)num_cu * 16;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (unsigned)g;
}

#define GSTRIDE(i, count)                                                        \
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (count); \
       i += (int64_t)gridDim.x * blockDim.x)

__global__ void k_validate(const int32_t* __restrict__ src, const int32_t* __restrict__ lab,
                           const int32_t* __restrict__ dst, int64_t m, int32_t n, int32_t K,
                           const int32_t* __restrict__ init, uint32_t* err) {
  bool bad = false;
  GSTRIDE(i, m) {
    bad |= (uint32_t)src[i] >= (uint32_t)n || (uint32_t)dst[i] >= (uint32_t)n ||
           (uint32_t)lab[i] >= (uint32_t)K;
  }
  if (init) {
    GSTRIDE(s, (int64_t)n) { bad |= (uint32_t)init[s] >= (uint32_t)n; }
  }
  if (bad) atomicOr(err, 1u);
}

__global__ void __launch_bounds__(kT) k_lab_hist(const int32_t* __restrict__ lab, int64_t m,
                                                 int32_t K, uint32_t* __restrict__ cnt) {
  __shared__ uint32_t h[kLdsLabels];
  const int64_t c0 = (int64_t)blockIdx.x * kChunk;
  const int64_t c1 = min(c0 + kChunk, m);
  if (K <= kLdsLabels) {
    for (int a = threadIdx.x; a < K; a += kT) h[a] = 0;
    __syncthreads();
    for (int64_t i = c0 + threadIdx.x; i < c1; i += kT) atomicAdd(&h[lab[i]], 1u);
    __syncthreads();
    for (int a = threadIdx.x; a < K; a += kT)
      if (h[a]) atomicAdd(&cnt[a], h[a]);
  } else {
    for (int64_t i = c0 + threadIdx.x; i < c1; i += kT) atomicAdd(&cnt[lab[i]], 1u);
  }
}

__global__ void __launch_bounds__(kT) k_lab_scatter(const int32_t* __restrict__ lab, int64_t m,
                                                    int32_t K, uint32_t* __restrict__ cursor,
                                                    uint32_t* __restrict__ idx) {
  __shared__ uint32_t h[kLdsLabels];
  const int64_t c0 = (int64_t)blockIdx.x * kChunk;
  const int64_t c1 = min(c0 + kChunk, m);
  if (K <= kLdsLabels) {
    for (int a = threadIdx.x; a < K; a += kT) h[a] = 0;
    __syncthreads();
    for (int64_t i = c0 + threadIdx.x; i < c1; i += kT) atomicAdd(&h[lab[i]], 1u);
    __syncthreads();
    for (int a = threadIdx.x; a < K; a += kT)
      if (h[a]) h[a] = atomicAdd(&cursor[a], h[a]);
    __syncthreads();
    for (int64_t i = c0 + threadIdx.x; i < c1; i += kT) {
      uint32_t p = atomicAdd(&h[lab[i]], 1u);
      idx[p] = (uint32_t)i;
    }
  } else {
    for (int64_t i = c0 + threadIdx.x; i < c1; i += kT) {
      uint32_t p = atomicAdd(&cursor[lab[i]], 1u);
      idx[p] = (uint32_t)i;
    }
  }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t count) {
  GSTRIDE(i, count) { p[i] = v; }
}

// new_leader[I_s] := s, the smallest s winning
__global__ void k_init_leaders_min(int32_t n, const int32_t* __restrict__ init,
                                   uint32_t* __restrict__ newl) {
  GSTRIDE(s, (int64_t)n) { atomicMin(&newl[init[s]], (uint32_t)s); }
}
__global__ void k_init_leaders_set(int32_t n, const int32_t* __restrict__ init,
                                   const uint32_t* __restrict__ newl,
                                   int32_t* __restrict__ block) {
  GSTRIDE(s, (int64_t)n) { block[s] = init ? (int32_t)newl[init[s]] : 0; }
}

// Algorithm 4, round a: mark sources of a-transitions and rank the action.
__global__ void k_round_mark(const uint32_t* __restrict__ idx, uint32_t beg, uint32_t end,
                             const int32_t* __restrict__ src, const int32_t* __restrict__ cnt,
                             int32_t* __restrict__ ord, uint8_t* __restrict__ has) {
  GSTRIDE(j, (int64_t)(end - beg)) {
    uint32_t i = idx[beg + j];
    int32_t s = src[i];
    ord[i] = cnt[s];
    has[s] = 1;
  }
}
// ... tag states whose mark differs from their leader's and elect (max of
// (epoch, ~s) == smallest s of this round).  A wave's 64 consecutive states
// mostly share their block (a large block splits its whole remainder in a
// round), so the splitting lanes of the first splitting lane's block bid once,
// with their smallest state; the others bid one by one.
__global__ void k_round_split(int32_t n, const int32_t* __restrict__ block,
                              const uint8_t* __restrict__ has, uint64_t* __restrict__ nlw,
                              uint8_t* __restrict__ flag, uint64_t epoch) {
  const int64_t waves = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; w * kWave < n;
       w += waves) {  // wave-uniform
    const int64_t s = w * kWave + lane();
    int32_t b = -1;
    bool sp = false;
    if (s < n) {
      b = block[s];
      sp = has[s] != has[b];
    }
    const uint64_t bal = __ballot(sp);
    if (!bal) continue;
    const int l0 = __ffsll((unsigned long long)bal) - 1;
    const int32_t b0 = __shfl(b, l0, kWave);
    const bool same = sp && b == b0;
    const uint32_t sm = wave_min_u32(same ? (uint32_t)s : kNone);
    // the bids of one round only grow, so a bid not above the current value
    // cannot win and skips the atomic
    auto bid = [&](int32_t blk, uint32_t st) {
      const uint64_t val = epoch | (uint64_t)(kNone - st);
      if (__hip_atomic_load(&nlw[blk], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < val)
        atomicMax((unsigned long long*)&nlw[blk], (unsigned long long)val);
    };
    if ((int)lane() == l0) bid(b0, sm);
    if (sp && !same) bid(b, (uint32_t)s);
    if (sp) flag[s] = 1;
  }
}
// ... relabel, and advance every marked state's action count
__global__ void k_round_relabel(int32_t n, int32_t* __restrict__ block,
                                const uint64_t* __restrict__ nlw, uint8_t* __restrict__ flag,
                                uint8_t* __restrict__ has, int32_t* __restrict__ cnt) {
  GSTRIDE(s, (int64_t)n) {
    if (flag[s]) {
      block[s] = (int32_t)(kNone - (uint32_t)nlw[block[s]]);
      flag[s] = 0;
    }
    if (has[s]) {
      cnt[s] += 1;
      has[s] = 0;
    }
  }
}

// red[0] = max nr_marks, red[1] = #leaders; red64 = sum nr_marks
__global__ void k_reduce(int32_t n, const int32_t* __restrict__ cnt,
                         const int32_t* __restrict__ block, uint32_t* red,
                         unsigned long long* red64) {
  uint32_t mx = 0, leaders = 0;
  unsigned long long sum = 0;
  GSTRIDE(s, (int64_t)n) {
    uint32_t c = (uint32_t)cnt[s];
    mx = max(mx, c);
    sum += c;
    leaders += (block[s] == (int32_t)s);
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    mx = max(mx, (uint32_t)__shfl_xor((int)mx, d, kWave));
    leaders += (uint32_t)__shfl_xor((int)leaders, d, kWave);
    sum += (unsigned long long)__shfl_xor((long long)sum, d, kWave);
  }
  if (lane() == 0) {
    atomicMax(&red[0], mx);
    atomicAdd(&red[1], leaders);
    atomicAdd(red64, sum);
  }
}

__global__ void k_words(int32_t n, const int32_t* __restrict__ cnt, uint32_t* __restrict__ w) {
  GSTRIDE(s, (int64_t)n) { w[s] = ((uint32_t)cnt[s] + 63u) >> 6; }
}

__global__ void k_indeg(const int32_t* __restrict__ dst, int64_t m, uint32_t* __restrict__ deg) {
  GSTRIDE(i, m) { atomicAdd(&deg[dst[i]], 1u); }
}

__global__ void k_max_u32(int32_t n, const uint32_t* __restrict__ v, uint32_t* mx_out) {
  uint32_t mx = 0;
  GSTRIDE(s, (int64_t)n) { mx = max(mx, v[s]); }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, d, kWave));
  if (lane() == 0) atomicMax(mx_out, mx);
}

// ---------------------------------------------------------------------------
// One-pass preprocessing (many actions, every state with at most 64 outgoing
// transitions).  The action-by-action rounds above reach the partition of
// states by (pi_0 block, set of outgoing actions) and rank each state's
// actions in increasing order; these kernels compute the same three results
// directly: one wave per state ranks the state's actions among its distinct
// actions and hashes the set; states are grouped by (pi_0 label, hash) in an
// open-addressing table whose entries keep their smallest state; a second
// pass checks every state's set and pi_0 label against its group leader's,
// so a hash collision is detected (the caller then runs the rounds).
// ---------------------------------------------------------------------------
constexpr uint32_t kOnePassMaxOut = kWave;
// with at most this many actions the rounds cost no more than the one pass's
// extra passes over the transitions (at 10M states and 64 actions: 57 ms
// against 86 ms)
constexpr int32_t kOnePassMinK = 64;

// SplitMix64's output function (Steele, Lea and Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void k_out_scatter(const int32_t* __restrict__ src, int64_t m,
                              uint32_t* __restrict__ cursor, uint32_t* __restrict__ out_idx) {
  GSTRIDE(i, m) { out_idx[atomicAdd(&cursor[src[i]], 1u)] = (uint32_t)i; }
}

// the actions of state s in the lanes (lane j < d holds transition j's
// action; other lanes hold none); wave-uniform
struct LaneActions {
  int32_t a;
  bool valid;
  uint32_t t;
};
__device__ __forceinline__ LaneActions lane_actions(const uint32_t* __restrict__ out_ptr,
                                                    const uint32_t* __restrict__ out_idx,
                                                    const int32_t* __restrict__ lab, int64_t s) {
  const uint32_t p0 = out_ptr[s], d = out_ptr[s + 1] - p0;
  LaneActions r{0, lane() < d, 0u};
  if (r.valid) {
    r.t = out_idx[p0 + lane()];
    r.a = lab[r.t];
  }
  return r;
}

__global__ void k_sets(int32_t n, const uint32_t* __restrict__ out_ptr,
                       const uint32_t* __restrict__ out_idx, const int32_t* __restrict__ lab,
                       const int32_t* __restrict__ pi0, int32_t* __restrict__ ord,
                       int32_t* __restrict__ nr_marks, unsigned long long* __restrict__ keys,
                       uint32_t* __restrict__ minst, uint32_t cap_mask,
                       uint32_t* __restrict__ slot, uint64_t key_mask, uint32_t* err) {
  const int64_t waves = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; s < n;
       s += waves) {  // wave-uniform
    if (out_ptr[s + 1] - out_ptr[s] > kOnePassMaxOut) {  // the caller checked; never expected
      if (lane() == 0) {
        slot[s] = 0;
        atomicOr(err, 1u);
      }
      continue;
    }
    const LaneActions x = lane_actions(out_ptr, out_idx, lab, s);
    // the first lane holding an action represents it; the rank of an action
    // is the number of distinct actions of s below it
    bool dup = false;
    uint32_t below = 0;
    for (int k = 0; k < (int)kWave; ++k) {
      const int32_t ak = __shfl(x.a, k, kWave);
      const bool vk = __shfl((int)x.valid, k, kWave) != 0;
      if (vk && ak == x.a && k < (int)lane()) dup = true;
    }
    const bool first = x.valid && !dup;
    for (int k = 0; k < (int)kWave; ++k) {
      const int32_t ak = __shfl(x.a, k, kWave);
      const bool fk = __shfl((int)first, k, kWave) != 0;
      if (fk && ak < x.a) ++below;
    }
    if (x.valid) ord[x.t] = (int32_t)below;
    const uint32_t distinct = (uint32_t)__popcll(__ballot(first));
    uint64_t h = first ? mix64((uint64_t)(uint32_t)x.a + 0x9E3779B97F4A7C15ull) : 0ull;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) h += (uint64_t)__shfl_xor((unsigned long long)h, d, kWave);
    if (lane() == 0) {
      nr_marks[s] = (int32_t)distinct;
      const uint64_t key =
          (mix64(h ^ mix64((uint64_t)(uint32_t)pi0[s] * 0x9E3779B97F4A7C15ull + distinct)) &
           key_mask) | 1ull;
      uint32_t q = (uint32_t)key & cap_mask;
      bool placed = false;
      for (uint32_t probe = 0; probe <= cap_mask && !placed; ++probe) {
        const unsigned long long old = atomicCAS(&keys[q], 0ull, (unsigned long long)key);
        placed = old == 0ull || old == key;
        if (!placed) q = (q + 1u) & cap_mask;
      }
      if (!placed) atomicOr(err, 4u);  // a table of 2n entries cannot fill; never expected
      atomicMin(&minst[q], (uint32_t)s);
      slot[s] = q;
    }
  }
}

__global__ void k_sets_label(int32_t n, const uint32_t* __restrict__ minst,
                             const uint32_t* __restrict__ slot, int32_t* __restrict__ block) {
  GSTRIDE(s, (int64_t)n) { block[s] = (int32_t)minst[slot[s]]; }
}

// every state's pi_0 label and action set equal its group leader's
__global__ void k_sets_verify(int32_t n, const uint32_t* __restrict__ out_ptr,
                              const uint32_t* __restrict__ out_idx,
                              const int32_t* __restrict__ lab, const int32_t* __restrict__ pi0,
                              const int32_t* __restrict__ nr_marks,
                              const int32_t* __restrict__ block, uint32_t* err) {
  const int64_t waves = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t s = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; s < n;
       s += waves) {  // wave-uniform
    const int32_t l = block[s];
    if (l == (int32_t)s) continue;
    if (l < 0 || l >= n || pi0[l] != pi0[s] || nr_marks[l] != nr_marks[s]) {
      if (lane() == 0) atomicOr(err, 2u);
      continue;
    }
    const LaneActions xs = lane_actions(out_ptr, out_idx, lab, s);
    const LaneActions xl = lane_actions(out_ptr, out_idx, lab, l);
    // with equal numbers of distinct actions, the sets are equal when each
    // action of s is one of l's
    bool found = !xs.valid;
    for (int k = 0; k < (int)kWave; ++k) {
      const int32_t ak = __shfl(xl.a, k, kWave);
      const bool vk = __shfl((int)xl.valid, k, kWave) != 0;
      if (vk && ak == xs.a) found = true;
    }
    if (__ballot(!found) && lane() == 0) atomicOr(err, 2u);
  }
}

__global__ void k_in_scatter(const int32_t* __restrict__ src, const int32_t* __restrict__ dst,
                             const int32_t* __restrict__ ord, int64_t m,
                             uint32_t* __restrict__ cursor, int32_t* __restrict__ in_src,
                             int32_t* __restrict__ in_ord) {
  GSTRIDE(i, m) {
    uint32_t p = atomicAdd(&cursor[dst[i]], 1u);
    in_src[p] = src[i];
    in_ord[p] = ord[i];
  }
}

// outgoing / incoming transitions of every state by label mod 8 (block
// features of the learned splitter policy are sums of these)
__global__ void k_static_features(const int32_t* __restrict__ src, const int32_t* __restrict__ lab,
                                  const int32_t* __restrict__ dst, int64_t m,
                                  uint32_t* __restrict__ sfeat) {
  GSTRIDE(i, m) {
    const uint32_t q = (uint32_t)lab[i] & 7u;
    atomicAdd(&sfeat[(size_t)src[i] * 16 + q], 1u);
    atomicAdd(&sfeat[(size_t)dst[i] * 16 + 8 + q], 1u);
  }
}

template <class T>
bisim_status dalloc(T** p, size_t count, hipStream_t s) {
  if (count == 0) count = 1;
  hipError_t e = dev_alloc((void**)p, sizeof(T) * count, s);
  if (e != hipSuccess) {
    set_error("device allocation of %zu bytes failed: %s", sizeof(T) * count, hipGetErrorString(e));
    return BISIM_E_NOMEM;
  }
  return BISIM_OK;
}

struct Temps {
  hipStream_t s = nullptr;
  std::vector<void*> ptrs;
  template <class T>
  bisim_status get(T** p, size_t count) {
    BISIM_TRY(dalloc(p, count, s));
    if (!arena_active()) ptrs.push_back((void*)*p);  // arena memory is never freed singly
    return BISIM_OK;
  }
  ~Temps() {
    for (void* p : ptrs) (void)dev_free(p, s);
  }
};
}  // namespace

bisim_status setup_load(bisim_lts* h, const int32_t* src, const int32_t* lab,
                        const int32_t* dst, const int32_t* init) {
  const int32_t n = h->n;
  const int64_t m = h->m;
  const int32_t K = h->K;
  hipStream_t st = h->stream;
  const int cu = h->num_cu;
  Temps tmp;
  tmp.s = st;

  // 1. validation
  uint32_t* err;
  BISIM_TRY(tmp.get(&err, 1));
  BISIM_TRY_HIP(hipMemsetAsync(err, 0, sizeof(uint32_t), st));
  hipLaunchKernelGGL(k_validate, dim3(grid_for(m > n ? m : n, cu)), dim3(kT), 0, st, src, lab,
                     dst, m, n, K, init, err);
  BISIM_TRY_HIP(hipGetLastError());
  uint32_t err_h = 0;
  BISIM_TRY_HIP(hipMemcpyAsync(&err_h, err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  BISIM_TRY_HIP(hipStreamSynchronize(st));
  if (err_h) {
    set_error("lts_load: a source/target is outside [0,n), a label outside [0,K), or an "
              "init_partition value outside [0,n)");
    return BISIM_E_RANGE;
  }

  // persistent preprocessed arrays
  BISIM_TRY(dalloc(&h->pre_block, (size_t)n, st));
  BISIM_TRY(dalloc(&h->nr_marks, (size_t)n, st));
  BISIM_TRY(dalloc(&h->in_ptr, (size_t)n + 1, st));
  BISIM_TRY(dalloc(&h->in_src, (size_t)m, st));
  BISIM_TRY(dalloc(&h->in_ord, (size_t)m, st));

  int32_t* ord;
  uint32_t *lab_cnt, *lab_ptr, *cursor, *idx, *newl, *red;
  uint8_t *has, *flag;
  uint64_t* nlw;
  unsigned long long* red64;
  BISIM_TRY(tmp.get(&ord, (size_t)m));
  BISIM_TRY(tmp.get(&lab_cnt, (size_t)K));
  BISIM_TRY(tmp.get(&lab_ptr, (size_t)K + 1));
  BISIM_TRY(tmp.get(&cursor, (size_t)(K > n ? K : n) + 1));
  BISIM_TRY(tmp.get(&idx, (size_t)m));
  BISIM_TRY(tmp.get(&newl, (size_t)n));
  BISIM_TRY(tmp.get(&red, 4));
  BISIM_TRY(tmp.get(&red64, 1));
  BISIM_TRY(tmp.get(&has, (size_t)n));
  BISIM_TRY(tmp.get(&flag, (size_t)n));
  BISIM_TRY(tmp.get(&nlw, (size_t)n));

  // 2. bucket transitions by action
  BISIM_TRY_HIP(hipMemsetAsync(lab_cnt, 0, sizeof(uint32_t) * K, st));
  const unsigned chunks = (unsigned)((m + kChunk - 1) / kChunk);
  if (m > 0) {
    hipLaunchKernelGGL(k_lab_hist, dim3(chunks), dim3(kT), 0, st, lab, m, K, lab_cnt);
    BISIM_TRY_HIP(hipGetLastError());
  }
  BISIM_TRY(exclusive_scan_u32(lab_cnt, lab_ptr, K, st));
  BISIM_TRY_HIP(hipMemcpyAsync(cursor, lab_ptr, sizeof(uint32_t) * K, hipMemcpyDeviceToDevice, st));
  if (m > 0) {
    hipLaunchKernelGGL(k_lab_scatter, dim3(chunks), dim3(kT), 0, st, lab, m, K, cursor, idx);
    BISIM_TRY_HIP(hipGetLastError());
  }

  // 3. leaders of pi_0
  const unsigned gn = grid_for(n, cu);
  if (init) {
    hipLaunchKernelGGL(k_fill_u32, dim3(gn), dim3(kT), 0, st, newl, kNone, (int64_t)n);
    hipLaunchKernelGGL(k_init_leaders_min, dim3(gn), dim3(kT), 0, st, n, init, newl);
  }
  hipLaunchKernelGGL(k_init_leaders_set, dim3(gn), dim3(kT), 0, st, n, init, newl, h->pre_block);
  BISIM_TRY_HIP(hipGetLastError());
  if (K == 1) {  // kept for Algorithm 2, which starts from pi_0 itself
    BISIM_TRY(dalloc(&h->init_block, (size_t)n, st));
    BISIM_TRY_HIP(hipMemcpyAsync(h->init_block, h->pre_block, sizeof(int32_t) * (size_t)n,
                                 hipMemcpyDeviceToDevice, st));
  }

  // 4. pi_pre and the action ranks: in one pass when there are many actions
  // and every state has at most 64 outgoing transitions (the rounds below
  // cost three launches per action), else by Algorithm 4's action rounds;
  // the one-pass result is checked and the rounds run if the check fails
  bool rounds = true;
  if (!arena_active() && K > kOnePassMinK && m > 0 && n > 0) {
    uint32_t* odeg;
    BISIM_TRY(tmp.get(&odeg, (size_t)n));
    BISIM_TRY_HIP(hipMemsetAsync(odeg, 0, sizeof(uint32_t) * (size_t)n, st));
    BISIM_TRY_HIP(hipMemsetAsync(red, 0, sizeof(uint32_t), st));
    hipLaunchKernelGGL(k_indeg, dim3(grid_for(m, cu)), dim3(kT), 0, st, src, m, odeg);
    hipLaunchKernelGGL(k_max_u32, dim3(gn), dim3(kT), 0, st, n, odeg, red);
    uint32_t max_out = 0;
    BISIM_TRY_HIP(hipMemcpyAsync(&max_out, red, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    BISIM_TRY_HIP(hipStreamSynchronize(st));
    if (max_out <= kOnePassMaxOut) {
      uint32_t *out_ptr, *out_idx, *minst, *slot, *err2;
      int32_t* pi0;
      unsigned long long* keys;
      uint32_t cap = 64;
      while (cap < 2u * (uint32_t)n) cap <<= 1;
      BISIM_TRY(tmp.get(&out_ptr, (size_t)n + 1));
      BISIM_TRY(tmp.get(&out_idx, (size_t)m));
      BISIM_TRY(tmp.get(&pi0, (size_t)n));
      BISIM_TRY(tmp.get(&keys, (size_t)cap));
      BISIM_TRY(tmp.get(&minst, (size_t)cap));
      BISIM_TRY(tmp.get(&slot, (size_t)n));
      BISIM_TRY(tmp.get(&err2, 1));
      BISIM_TRY(exclusive_scan_u32(odeg, out_ptr, n, st));
      BISIM_TRY_HIP(hipMemcpyAsync(cursor, out_ptr, sizeof(uint32_t) * (size_t)n,
                                   hipMemcpyDeviceToDevice, st));
      hipLaunchKernelGGL(k_out_scatter, dim3(grid_for(m, cu)), dim3(kT), 0, st, src, m, cursor,
                         out_idx);
      BISIM_TRY_HIP(hipMemcpyAsync(pi0, h->pre_block, sizeof(int32_t) * (size_t)n,
                                   hipMemcpyDeviceToDevice, st));
      BISIM_TRY_HIP(hipMemsetAsync(keys, 0, sizeof(unsigned long long) * cap, st));
      hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(cap, cu)), dim3(kT), 0, st, minst, kNone,
                         (int64_t)cap);
      BISIM_TRY_HIP(hipMemsetAsync(err2, 0, sizeof(uint32_t), st));
      const unsigned gw = grid_for((int64_t)n * kWave, cu);  // a wave per state
      // test hook: BISIM_ONEPASS_COLLIDE=1 gives every state the same key, so
      // the check fails wherever two states differ and the rounds run
      const char* collide = getenv("BISIM_ONEPASS_COLLIDE");
      const uint64_t key_mask = (collide && collide[0] == '1') ? 0ull : ~0ull;
      hipLaunchKernelGGL(k_sets, dim3(gw), dim3(kT), 0, st, n, out_ptr, out_idx, lab, pi0, ord,
                         h->nr_marks, keys, minst, cap - 1, slot, key_mask, err2);
      hipLaunchKernelGGL(k_sets_label, dim3(gn), dim3(kT), 0, st, n, minst, slot, h->pre_block);
      hipLaunchKernelGGL(k_sets_verify, dim3(gw), dim3(kT), 0, st, n, out_ptr, out_idx, lab, pi0,
                         h->nr_marks, h->pre_block, err2);
      BISIM_TRY_HIP(hipGetLastError());
      uint32_t err2_h = 0;
      BISIM_TRY_HIP(hipMemcpyAsync(&err2_h, err2, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
      BISIM_TRY_HIP(hipStreamSynchronize(st));
      if (err2_h == 0) {
        rounds = false;
      } else {  // a hash collision merged two action sets: back to pi_0 and the rounds
        BISIM_TRY_HIP(hipMemcpyAsync(h->pre_block, pi0, sizeof(int32_t) * (size_t)n,
                                     hipMemcpyDeviceToDevice, st));
      }
    }
  }
  if (rounds) {
  // Algorithm 4 rounds, fused with the action ranking
  BISIM_TRY_HIP(hipMemsetAsync(has, 0, (size_t)n, st));
  BISIM_TRY_HIP(hipMemsetAsync(flag, 0, (size_t)n, st));
  BISIM_TRY_HIP(hipMemsetAsync(h->nr_marks, 0, sizeof(int32_t) * (size_t)n, st));
  BISIM_TRY_HIP(hipMemsetAsync(nlw, 0, sizeof(uint64_t) * (size_t)n, st));
  // the host reads the action buckets' bounds a piece at a time
  constexpr int32_t kLp = 2048;
  uint32_t lp[kLp + 1];
  uint64_t epoch = 0;
  for (int32_t a0 = 0; a0 < K; a0 += kLp) {
    const int32_t cnt = K - a0 < kLp ? K - a0 : kLp;
    BISIM_TRY_HIP(hipMemcpyAsync(lp, lab_ptr + a0, sizeof(uint32_t) * (size_t)(cnt + 1),
                                 hipMemcpyDeviceToHost, st));
    BISIM_TRY_HIP(hipStreamSynchronize(st));
    for (int32_t j = 0; j < cnt; ++j) {
      const uint32_t b0 = lp[j], b1 = lp[j + 1];
      if (b1 == b0) continue;
      ++epoch;
      hipLaunchKernelGGL(k_round_mark, dim3(grid_for(b1 - b0, cu)), dim3(kT), 0, st, idx, b0, b1,
                         src, h->nr_marks, ord, has);
      hipLaunchKernelGGL(k_round_split, dim3(gn), dim3(kT), 0, st, n, h->pre_block, has, nlw,
                         flag, epoch << 32);
      hipLaunchKernelGGL(k_round_relabel, dim3(gn), dim3(kT), 0, st, n, h->pre_block, nlw, flag,
                         has, h->nr_marks);
      BISIM_TRY_HIP(hipGetLastError());
    }
  }
  }
  h->one_pass = !rounds;

  // 5. slot statistics and mark-word layout
  BISIM_TRY_HIP(hipMemsetAsync(red, 0, sizeof(uint32_t) * 4, st));
  BISIM_TRY_HIP(hipMemsetAsync(red64, 0, sizeof(unsigned long long), st));
  hipLaunchKernelGGL(k_reduce, dim3(gn), dim3(kT), 0, st, n, h->nr_marks, h->pre_block, red,
                     red64);
  BISIM_TRY_HIP(hipGetLastError());
  uint32_t red_h[4];
  unsigned long long red64_h = 0;
  BISIM_TRY_HIP(hipMemcpyAsync(red_h, red, sizeof(red_h), hipMemcpyDeviceToHost, st));
  BISIM_TRY_HIP(hipMemcpyAsync(&red64_h, red64, sizeof(red64_h), hipMemcpyDeviceToHost, st));
  BISIM_TRY_HIP(hipStreamSynchronize(st));
  h->pre_blocks = red_h[1];
  h->mark_length = (int64_t)red64_h;
  h->uniform = red_h[0] <= 64;
  h->max_ranks = red_h[0];
  if (h->uniform) {
    h->nwords = (uint64_t)n;
  } else {
    uint32_t* words;
    BISIM_TRY(tmp.get(&words, (size_t)n));
    BISIM_TRY(dalloc(&h->woff, (size_t)n + 1, st));
    hipLaunchKernelGGL(k_words, dim3(gn), dim3(kT), 0, st, n, h->nr_marks, words);
    BISIM_TRY(exclusive_scan_u32(words, h->woff, n, st));
    uint32_t nw = 0;
    BISIM_TRY_HIP(hipMemcpyAsync(&nw, h->woff + n, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    BISIM_TRY_HIP(hipStreamSynchronize(st));
    h->nwords = nw;
  }

  // 6. largest out-degree, then transitions grouped by target
  uint32_t* deg;
  BISIM_TRY(tmp.get(&deg, (size_t)n));
  BISIM_TRY_HIP(hipMemsetAsync(deg, 0, sizeof(uint32_t) * (size_t)n, st));
  BISIM_TRY_HIP(hipMemsetAsync(red, 0, sizeof(uint32_t), st));
  if (m > 0) {
    hipLaunchKernelGGL(k_indeg, dim3(grid_for(m, cu)), dim3(kT), 0, st, src, m, deg);
    hipLaunchKernelGGL(k_max_u32, dim3(gn), dim3(kT), 0, st, n, deg, red);
  }
  BISIM_TRY_HIP(hipMemcpyAsync(&h->max_out, red, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  BISIM_TRY_HIP(hipStreamSynchronize(st));
  BISIM_TRY_HIP(hipMemsetAsync(deg, 0, sizeof(uint32_t) * (size_t)n, st));
  if (m > 0) hipLaunchKernelGGL(k_indeg, dim3(grid_for(m, cu)), dim3(kT), 0, st, dst, m, deg);
  BISIM_TRY(exclusive_scan_u32(deg, h->in_ptr, n, st));
  BISIM_TRY_HIP(hipMemcpyAsync(cursor, h->in_ptr, sizeof(uint32_t) * (size_t)n,
                               hipMemcpyDeviceToDevice, st));
  if (m > 0)
    hipLaunchKernelGGL(k_in_scatter, dim3(grid_for(m, cu)), dim3(kT), 0, st, src, dst, ord, m,
                       cursor, h->in_src, h->in_ord);
  BISIM_TRY_HIP(hipGetLastError());

  // 7. per-state transition counts by label bucket (block features; not
  // kept by the allocation-free entry point, which runs the plain policy)
  if (arena_active()) return BISIM_OK;
  BISIM_TRY(dalloc(&h->sfeat, 16 * (size_t)n, st));
  BISIM_TRY_HIP(hipMemsetAsync(h->sfeat, 0, sizeof(uint32_t) * 16 * (size_t)n, st));
  if (m > 0)
    hipLaunchKernelGGL(k_static_features, dim3(grid_for(m, cu)), dim3(kT), 0, st, src, lab, dst,
                       m, h->sfeat);
  BISIM_TRY_HIP(hipGetLastError());
  return BISIM_OK;
}

}  // namespace bisim
