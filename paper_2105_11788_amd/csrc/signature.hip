// Multi-way signature refinement: the signature-based splitting used by the
// GPU systems the paper compares against in section 5 (there: Wijs' Wms),
// built here as an in-house baseline beside the paper's method.  It is not
// part of the paper's algorithms.
//
// From pi_pre (section 4.1), every round gives each state s the signature
// sig(s) = {(a, block(t)) : s -a-> t} and regroups the states by
// (block(s), sig(s)); a new block is named by its smallest state.  The round
// that changes nothing ends the run.  A round on the GPU:
//   1. every transition s -a-> t gets the value x = rank * n + block(t)
//      (rank: the action's rank among the source's actions; within a block of
//      pi_pre, and so of every later partition, ranks name the same actions,
//      so (rank, block) pairs stand for (action, block) pairs);
//   2. sig(s) = sum over the distinct values of s of a 64-bit hash of x (a
//      set hash: duplicates count once).  The first kSortedRounds rounds give
//      every transition the key (s << xbits) | x (xbits: the bits that
//      x < (actions per state) * n needs) and radix-sort the keys, so equal
//      pairs are adjacent, and reduce per wave over the sorted segments.  The
//      last of them sorts the transitions' indices along, and its order is
//      kept as the transitions' layout by source: in later rounds a source
//      with at most 64 transitions is handled by the lanes of one or two
//      waves, each lane comparing its x with the earlier ones of its source
//      by shuffles; the (s, x) pairs of larger sources go into a hash table
//      (up to kHashMax of them; only a fresh insertion counts) or are sorted.
//      (Shallow LTSs reach the fixpoint within the sorted rounds: there the
//      layout, about as costly as two sorted rounds, would not pay.);
//   3. the states are grouped by a hash of (block(s), sig(s)): up to
//      kHashMax states in a hash table whose slot keeps its group's smallest
//      state, beyond that by a radix sort stable in the state index (each run
//      of equal hashes starts at its smallest state) and a max-scan of the
//      run heads; either names every state's new block.
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
#include <cstdlib>

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

// key[e] = (source << xbits) | x for every transition, and idx[e] = e when
// idx is given (the sort that lays the transitions out carries them)
__global__ void k_keys(int64_t m, uint32_t n, int xbits, const int32_t* __restrict__ in_src,
                       const int32_t* __restrict__ in_ord, const int32_t* __restrict__ tgt,
                       const int32_t* __restrict__ blk, uint64_t* __restrict__ key,
                       uint32_t* __restrict__ idx) {
  SSTRIDE(e, m) {
    key[e] = ((uint64_t)(uint32_t)in_src[e] << xbits) |
             (uint32_t)((uint32_t)in_ord[e] * n + (uint32_t)blk[tgt[e]]);
    if (idx) idx[e] = (uint32_t)e;
  }
}

// the by-source layout from the first round's sorted keys and indices
__global__ void k_layout(int64_t m, uint32_t n, int xbits, const uint64_t* __restrict__ keys,
                         const uint32_t* __restrict__ perm, const int32_t* __restrict__ in_ord,
                         const int32_t* __restrict__ tgt, int32_t* __restrict__ o_src,
                         uint32_t* __restrict__ o_rn, int32_t* __restrict__ o_tgt) {
  SSTRIDE(p, m) {
    const uint32_t e = perm[p];
    o_src[p] = (int32_t)(keys[p] >> xbits);
    o_rn[p] = (uint32_t)in_ord[e] * n;
    o_tgt[p] = tgt[e];
  }
}

// out_ptr[s] = the first position whose source is s or larger (out_ptr[n] = m):
// every position writes the entries of the sources from just after its
// predecessor's up to its own
__global__ void k_seg_starts(int64_t m, int32_t n, const int32_t* __restrict__ o_src,
                             uint32_t* __restrict__ out_ptr) {
  SSTRIDE(p, m + 1) {
    const int32_t lo = p == 0 ? -1 : o_src[p - 1];
    const int32_t hi = p == m ? n : o_src[p];
    for (int32_t s = lo + 1; s <= hi; ++s) out_ptr[s] = (uint32_t)p;
  }
}

// positions (in the by-source layout) of the transitions of sources with more
// than kWave transitions
__global__ void __launch_bounds__(kT) k_big_list(int64_t m, const int32_t* __restrict__ o_src,
                                                 const uint32_t* __restrict__ out_ptr,
                                                 int32_t* __restrict__ big,
                                                 uint32_t* __restrict__ count) {
  for (int64_t b0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave * kWave; b0 < m;
       b0 += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = b0 + lane();
    bool is_big = false;
    if (e < m) {
      const int32_t s = o_src[e];
      is_big = out_ptr[s + 1] - out_ptr[s] > (uint32_t)kWave;
    }
    wave_push(big, count, (int32_t)e, is_big);
  }
}

__global__ void k_keys_big(int64_t mb, int xbits, const int32_t* __restrict__ big,
                           const int32_t* __restrict__ o_src, const uint32_t* __restrict__ o_rn,
                           const int32_t* __restrict__ o_tgt, const int32_t* __restrict__ blk,
                           uint64_t* __restrict__ key) {
  SSTRIDE(i, mb) {
    const int32_t e = big[i];
    key[i] = ((uint64_t)(uint32_t)o_src[e] << xbits) |
             (uint32_t)(o_rn[e] + (uint32_t)blk[o_tgt[e]]);
  }
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, d, kWave));
  return v;
}

// sig[s] += hash(x) over the distinct values x of the sources with at most
// kWave transitions, one lane per transition of the by-source layout.  A
// lane's value is a duplicate if an earlier transition of its source has it:
// those in the same wave are reached by shuffles, those before the wave (a
// source that starts in the previous wave) by loads.  One atomic per source
// piece within a wave.  All lanes of a wave reach the shuffles.
__global__ void __launch_bounds__(kT) k_sig_small(int64_t m, const int32_t* __restrict__ o_src,
                                                  const uint32_t* __restrict__ o_rn,
                                                  const int32_t* __restrict__ o_tgt,
                                                  const uint32_t* __restrict__ out_ptr,
                                                  const int32_t* __restrict__ blk, uint64_t seed,
                                                  uint64_t* __restrict__ sig) {
  const int64_t waves = (int64_t)gridDim.x * (kT / kWave);
  const int64_t gw = (int64_t)blockIdx.x * (kT / kWave) + threadIdx.x / kWave;
  const int l = (int)lane();
  for (int64_t base = gw * kWave; base < m; base += waves * kWave) {
    const int64_t e = base + l;
    int32_t s = -1;
    uint32_t lo = 0, hi = 0, x = 0;
    if (e < m) {
      s = o_src[e];
      lo = out_ptr[s];
      hi = out_ptr[s + 1];
    }
    const bool small = e < m && hi - lo <= (uint32_t)kWave;
    if (small) x = o_rn[e] + (uint32_t)blk[o_tgt[e]];
    // earlier transitions of the source inside this wave: lanes l - back .. l - 1
    const int64_t first = (int64_t)lo > base ? (int64_t)lo : base;
    const uint32_t back = small ? (uint32_t)(e - first) : 0u;
    const uint32_t reach = wave_max_u32(back);
    bool dup = false;
    for (uint32_t d = 1; d <= reach; ++d) {
      const uint32_t xd = (uint32_t)__shfl_up((int)x, d, kWave);
      dup |= d <= back && xd == x;
    }
    if (small && (int64_t)lo < base) {
      for (int64_t j = lo; j < base; ++j) dup |= o_rn[j] + (uint32_t)blk[o_tgt[j]] == x;
    }
    uint64_t v = (small && !dup) ? mix64((uint64_t)x + seed) : 0ull;
    const int32_t s_next = __shfl_down(s, 1, kWave);
    const bool tail = small && (l == kWave - 1 || e + 1 >= m || s_next != s);
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

// sig[s] += hash(rank, block) over the distinct sorted keys of source s; one
// atomic per segment piece within a wave (all lanes of a wave reach the
// shuffles).
__global__ void __launch_bounds__(kT) k_sig_sum(int64_t m, int xbits,
                                                const uint64_t* __restrict__ key,
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
    const uint32_t s = (uint32_t)(k >> xbits);
    uint64_t v = distinct ? mix64((k & ((1ull << xbits) - 1ull)) + seed) : 0ull;
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

// open-addressing tables of 64-bit keys (kEmpty: a free slot) with linear
// probing, sized to at least twice their entries
constexpr uint64_t kEmpty = ~0ull;

__global__ void k_fill_u64(uint64_t* __restrict__ t, int64_t count, uint64_t v) {
  SSTRIDE(i, count) { t[i] = v; }
}
__global__ void k_fill_i32(int32_t* __restrict__ t, int64_t count, int32_t v) {
  SSTRIDE(i, count) { t[i] = v; }
}

// the slot holding key (inserting it if absent; *fresh tells which), or
// kNone if the table is full.  A slot is read before it is claimed, so a key
// that many threads insert (a large group) costs one atomic, not one each.
__device__ __forceinline__ uint32_t table_insert(uint64_t* tab, uint32_t mask, uint64_t key,
                                                 bool* fresh) {
  uint32_t h = (uint32_t)mix64(key) & mask;
  *fresh = false;
  for (uint32_t probe = 0; probe <= mask; ++probe) {
    const uint64_t cur = __hip_atomic_load(tab + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (cur == key) return h;
    if (cur == kEmpty) {
      const uint64_t prev = atomicCAS((unsigned long long*)(tab + h), (unsigned long long)kEmpty,
                                      (unsigned long long)key);
      if (prev == kEmpty) {
        *fresh = true;
        return h;
      }
      if (prev == key) return h;
    }
    h = (h + 1) & mask;
  }
  return kNone;
}

// The lowest lane of each group of lanes of a wave that hold the same key
// (a wave-uniform loop of ballots over the distinct keys, no memory access):
// only these lanes touch the table, all at once, so a key that many lanes
// hold (the transitions of a hub into one block, the states of a large
// group) does not serialise the table's atomics.  Returns the lane's leader.
__device__ __forceinline__ int wave_key_leader(bool valid, uint64_t key) {
  int mine = -1;
  uint64_t pending = __ballot(valid);
  while (pending) {  // wave-uniform
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const uint64_t lk = (uint64_t)__shfl((unsigned long long)key, leader, kWave);
    const uint64_t peers = __ballot(((pending >> lane()) & 1ull) && key == lk);
    if ((peers >> lane()) & 1ull) mine = leader;
    pending &= ~peers;
  }
  return mine;
}

// sig[s] += hash(x) over the distinct (s, x) of the large sources'
// transitions, found by inserting every pair into a table: only a fresh
// insertion counts.  Sums are combined per source piece within a wave (one
// atomic each).  All lanes of a wave reach the shuffles.
__global__ void __launch_bounds__(kT) k_sig_big_hash(int64_t mb, int xbits,
                                                     const int32_t* __restrict__ big,
                                                     const int32_t* __restrict__ o_src,
                                                     const uint32_t* __restrict__ o_rn,
                                                     const int32_t* __restrict__ o_tgt,
                                                     const int32_t* __restrict__ blk,
                                                     uint64_t seed, uint64_t* tab, uint32_t mask,
                                                     uint64_t* __restrict__ sig,
                                                     unsigned long long* fail) {
  const int64_t waves = (int64_t)gridDim.x * (kT / kWave);
  const int64_t gw = (int64_t)blockIdx.x * (kT / kWave) + threadIdx.x / kWave;
  const int l = (int)lane();
  for (int64_t base = gw * kWave; base < mb; base += waves * kWave) {
    const int64_t i = base + l;
    const bool valid = i < mb;
    int32_t s = -1;
    uint32_t x = 0;
    uint64_t key = 0;
    if (valid) {
      const int32_t e = big[i];
      s = o_src[e];
      x = o_rn[e] + (uint32_t)blk[o_tgt[e]];
      key = ((uint64_t)(uint32_t)s << xbits) | x;
    }
    uint64_t v = 0;
    if (wave_key_leader(valid, key) == l) {
      bool fresh;
      if (table_insert(tab, mask, key, &fresh) == kNone) atomicAdd(fail, 1ull);
      if (fresh) v = mix64((uint64_t)x + seed);
    }
    const int32_t s_next = __shfl_down(s, 1, kWave);
    const bool tail = valid && (l == kWave - 1 || i + 1 >= mb || s_next != s);
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

// groups of equal hk by table: every state finds its group's slot (slot_of),
// the slot's value becomes the group's smallest state, and the groups are
// counted.  One insertion and at most one atomicMin per distinct key and
// wave.  All lanes of a wave reach the shuffles.
__global__ void __launch_bounds__(kT) k_group_insert(int32_t n, const uint64_t* __restrict__ hk,
                                                     uint64_t* tab, int32_t* val, uint32_t mask,
                                                     int32_t* __restrict__ slot_of,
                                                     unsigned long long* groups,
                                                     unsigned long long* fail) {
  const int64_t waves = (int64_t)gridDim.x * (kT / kWave);
  const int64_t gw = (int64_t)blockIdx.x * (kT / kWave) + threadIdx.x / kWave;
  const int l = (int)lane();
  uint32_t c = 0;
  for (int64_t base = gw * kWave; base < n; base += waves * kWave) {
    const int64_t s = base + l;
    const bool valid = s < n;
    uint64_t key = 0;
    if (valid) key = hk[s] == kEmpty ? kEmpty - 1 : hk[s];
    // a leader is the lowest lane of its group, so its state is the group's
    // smallest in this wave
    const int leader = wave_key_leader(valid, key);
    uint32_t h = kNone;
    if (leader == l) {
      bool fresh;
      h = table_insert(tab, mask, key, &fresh);
      if (h == kNone) {
        atomicAdd(fail, 1ull);
      } else {
        c += fresh ? 1u : 0u;
        if ((int32_t)s < __hip_atomic_load(val + h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
          atomicMin(val + h, (int32_t)s);
      }
    }
    h = (uint32_t)__shfl((int)h, leader < 0 ? 0 : leader, kWave);
    if (valid) slot_of[s] = h == kNone ? -1 : (int32_t)h;
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) c += (uint32_t)__shfl_xor((int)c, d, kWave);
  if (l == 0 && c != 0) atomicAdd(groups, (unsigned long long)c);
}

__global__ void k_group_assign(int32_t n, const int32_t* __restrict__ slot_of,
                               const int32_t* __restrict__ val, int32_t* __restrict__ nb) {
  SSTRIDE(s, (int64_t)n) {
    const int32_t h = slot_of[s];
    nb[s] = h >= 0 ? val[h] : (int32_t)s;
  }
}

// hk[s]: the low hbits of a hash of (block(s), sig(s))
__global__ void k_state_keys(int32_t n, uint64_t hmask, const int32_t* __restrict__ blk,
                             const uint64_t* __restrict__ sig, uint64_t* __restrict__ hk,
                             int32_t* __restrict__ idx) {
  SSTRIDE(s, (int64_t)n) {
    hk[s] = hmask & mix64(sig[s] ^ mix64((uint64_t)(uint32_t)blk[s] + 0x9E3779B97F4A7C15ull));
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
  // one atomic per wave (a million threads adding to one word serialise)
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) c += (uint32_t)__shfl_xor((int)c, d, kWave);
  if (lane() == 0 && c != 0) atomicAdd(count, (unsigned long long)c);
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

// device buffers of a run: the handle's slots, taken in a fixed order (so a
// later run on the same handle finds its buffers allocated), kept until
// lts_free
struct Bufs {
  bisim_lts* h;
  int k = 0;
  template <class T>
  bisim_status get(T** out, size_t count) {
    const size_t bytes = sizeof(T) * (count == 0 ? 1 : count);
    if (k == bisim_lts::kSigSlots) {
      set_error("signature refinement: too many buffers");
      return BISIM_E_INVALID;
    }
    const int i = k++;
    if (h->sig_bytes[i] < bytes) {
      if (h->sig_buf[i]) (void)hipFreeAsync(h->sig_buf[i], h->stream);
      h->sig_buf[i] = nullptr;
      h->sig_bytes[i] = 0;
      if (hipMallocAsync(&h->sig_buf[i], bytes, h->stream) != hipSuccess) {
        h->sig_buf[i] = nullptr;
        set_error("signature refinement: out of device memory (%zu bytes)", bytes);
        return BISIM_E_NOMEM;
      }
      h->sig_bytes[i] = bytes;
    }
    *out = (T*)h->sig_buf[i];
    return BISIM_OK;
  }
};

}  // namespace

constexpr int64_t kHybridStall = 64;
// up to this many entries, grouping and duplicate removal use hash tables
// instead of radix sorts (fewer launches per round)
constexpr int64_t kHashMax = 1 << 22;
// a power of two of at least twice the entries (and at least 256)
static uint32_t table_size(int64_t entries) {
  uint32_t t = 256;
  while ((int64_t)t < 2 * entries) t <<= 1;
  return t;
}
// rounds that sort all transitions; the last of them lays the transitions out
constexpr int64_t kSortedRounds = 4;

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
  Bufs b{h};
  int32_t *tgt, *blk, *nb, *idx, *idxs, *hp, *hp2, *o_src, *o_tgt, *big;
  uint32_t *out_ptr, *o_rn, *nbig, *pidx = nullptr, *perm = nullptr;
  uint64_t *key, *keys, *sig, *hk, *hks;
  unsigned long long* cnt;
  BISIM_TRY(b.get(&tgt, (size_t)m));
  BISIM_TRY(b.get(&blk, (size_t)n));
  BISIM_TRY(b.get(&nb, (size_t)n));
  BISIM_TRY(b.get(&idx, (size_t)n));
  BISIM_TRY(b.get(&idxs, (size_t)n));
  BISIM_TRY(b.get(&hp, (size_t)n));
  BISIM_TRY(b.get(&hp2, (size_t)n));
  BISIM_TRY(b.get(&sig, (size_t)n));
  BISIM_TRY(b.get(&hk, 2 * (size_t)n));
  BISIM_TRY(b.get(&cnt, 4));
  hks = hk + n;
  nbig = (uint32_t*)(cnt + 3);  // count of the large sources' transitions
  unsigned long long* fail = cnt + 2;  // a full hash table (never expected)
  BISIM_TRY_HIP(hipMemsetAsync(fail, 0, sizeof(unsigned long long), st));
  // states grouped by a table of their hashes, up to kHashMax states (a
  // stable sort of the hashes beyond)
  // test hook: BISIM_SIGNATURE_SORT_ONLY=1 takes the radix sorts at every size
  const char* sort_only = getenv("BISIM_SIGNATURE_SORT_ONLY");
  const int64_t hash_max = (sort_only && sort_only[0] == '1') ? -1 : kHashMax;
  const bool group_hash = n <= hash_max;
  const uint32_t tsz = group_hash ? table_size(n) : 0u;
  uint64_t* gtab = nullptr;
  int32_t* gval = nullptr;
  if (group_hash) {
    BISIM_TRY(b.get(&gtab, tsz));
    BISIM_TRY(b.get(&gval, tsz));
  }
  o_src = o_tgt = big = nullptr;
  out_ptr = o_rn = nullptr;

  if (m > 0)
    hipLaunchKernelGGL(k_targets, dim3(grid_of(n, cu)), dim3(kT), 0, st, n, h->in_ptr, tgt);
  BISIM_TRY_HIP(hipGetLastError());
  BISIM_TRY(b.get(&key, (size_t)m));
  BISIM_TRY(b.get(&keys, (size_t)m));
  // key widths: source bits above xbits bits of x < max_ranks * n; the state
  // hash, when sorted, keeps 2 log2(n) + 24 bits (whole bytes), so that two
  // of at most n groups share a hash with probability below 2^-25 per round
  // (a merge is caught by the check, which then repeats the run with other
  // seeds)
  int kbits = 1;
  while (kbits < 31 && (1ll << kbits) < n) ++kbits;
  int xbits = 1;
  while (xbits < 32 && (1ull << xbits) < (uint64_t)(h->max_ranks ? h->max_ranks : 1) * (uint64_t)n)
    ++xbits;
  const int hbits = 2 * kbits + 24 >= 64 ? 64 : (2 * kbits + 24 + 7) / 8 * 8;
  const uint64_t hmask = hbits >= 64 ? ~0ull : (1ull << hbits) - 1ull;
  const size_t t1 = radix_sort_temp_bytes(m, false), t2 = radix_sort_temp_bytes(n, true);
  const size_t tb = t1 > t2 ? t1 : t2;
  uint8_t* temp;
  BISIM_TRY(b.get(&temp, tb));

  // the by-source layout, and the list of the transitions whose source has
  // more than a wave's worth (their duplicates go by a table or the sort)
  bool by_source = false, big_hash = false;
  uint32_t mb = 0, btsz = 0;
  uint64_t* btab = nullptr;
  // sig[s] += hash(x) over the distinct pairs of the large sources, by table
  auto big_by_table = [&](uint64_t sd) -> bisim_status {
    if (mb == 0) return BISIM_OK;
    hipLaunchKernelGGL(k_fill_u64, dim3(grid_of(btsz, cu)), dim3(kT), 0, st, btab, (int64_t)btsz,
                       kEmpty);
    hipLaunchKernelGGL(k_sig_big_hash, dim3(grid_of(mb, cu)), dim3(kT), 0, st, (int64_t)mb, xbits,
                       big, o_src, o_rn, o_tgt, blk, sd, btab, btsz - 1u, sig, fail);
    BISIM_TRY_HIP(hipGetLastError());
    return BISIM_OK;
  };
  int64_t sorted_keys = 0;  // keys[0, sorted_keys): the last round's sorted keys
  auto lay_out = [&]() -> bisim_status {
    BISIM_TRY(b.get(&o_src, (size_t)m));
    BISIM_TRY(b.get(&o_rn, (size_t)m));
    BISIM_TRY(b.get(&o_tgt, (size_t)m));
    BISIM_TRY(b.get(&big, (size_t)m));
    BISIM_TRY(b.get(&out_ptr, (size_t)n + 1));
    hipLaunchKernelGGL(k_layout, dim3(grid_of(m, cu)), dim3(kT), 0, st, m, (uint32_t)n, xbits, keys,
                       perm, h->in_ord, tgt, o_src, o_rn, o_tgt);
    hipLaunchKernelGGL(k_seg_starts, dim3(grid_of(m + 1, cu)), dim3(kT), 0, st, m, n, o_src,
                       out_ptr);
    BISIM_TRY_HIP(hipMemsetAsync(nbig, 0, sizeof(uint32_t), st));
    hipLaunchKernelGGL(k_big_list, dim3(grid_of(m, cu)), dim3(kT), 0, st, m, o_src, out_ptr, big,
                       nbig);
    BISIM_TRY_HIP(hipGetLastError());
    BISIM_TRY_HIP(hipMemcpyAsync(&mb, nbig, sizeof(mb), hipMemcpyDeviceToHost, st));
    BISIM_TRY_HIP(hipStreamSynchronize(st));
    big_hash = (int64_t)mb <= hash_max;
    btsz = big_hash ? table_size(mb) : 0u;
    BISIM_TRY(b.get(&btab, big_hash ? btsz : 1u));
    by_source = true;
    return BISIM_OK;
  };
  // sig[s] = the set hash of s's (rank, block) pairs under `sd`
  // (lay: sort the transitions' indices along and keep the order as the layout)
  auto signatures = [&](uint64_t sd, bool lay) -> bisim_status {
    BISIM_TRY_HIP(hipMemsetAsync(sig, 0, sizeof(uint64_t) * n, st));
    if (m == 0) return BISIM_OK;
    if (!by_source) {
      if (lay) {
        const size_t tbv = radix_sort_temp_bytes(m, true);
        uint8_t* tv;
        BISIM_TRY(b.get(&pidx, (size_t)m));
        BISIM_TRY(b.get(&perm, (size_t)m));
        BISIM_TRY(b.get(&tv, tbv));
        hipLaunchKernelGGL(k_keys, dim3(grid_of(m, cu)), dim3(kT), 0, st, m, (uint32_t)n, xbits,
                           h->in_src, h->in_ord, tgt, blk, key, pidx);
        BISIM_TRY(radix_sort_u64(tv, tbv, key, keys, pidx, perm, m, 0, xbits + kbits, st));
      } else {
        hipLaunchKernelGGL(k_keys, dim3(grid_of(m, cu)), dim3(kT), 0, st, m, (uint32_t)n, xbits,
                           h->in_src, h->in_ord, tgt, blk, key, (uint32_t*)nullptr);
        BISIM_TRY(radix_sort_u64(temp, tb, key, keys, nullptr, nullptr, m, 0, xbits + kbits, st));
      }
      hipLaunchKernelGGL(k_sig_sum, dim3(grid_of(m, cu)), dim3(kT), 0, st, m, xbits, keys, sd,
                         sig);
      BISIM_TRY_HIP(hipGetLastError());
      sorted_keys = m;
      return lay ? lay_out() : BISIM_OK;
    }
    hipLaunchKernelGGL(k_sig_small, dim3(grid_of(m, cu)), dim3(kT), 0, st, m, o_src, o_rn, o_tgt,
                       out_ptr, blk, sd, sig);
    if (big_hash) {
      BISIM_TRY(big_by_table(sd));
      sorted_keys = 0;
      return BISIM_OK;
    }
    if (mb > 0) {
      hipLaunchKernelGGL(k_keys_big, dim3(grid_of(mb, cu)), dim3(kT), 0, st, (int64_t)mb, xbits,
                         big, o_src, o_rn, o_tgt, blk, key);
      BISIM_TRY(radix_sort_u64(temp, tb, key, keys, nullptr, nullptr, mb, 0, xbits + kbits, st));
      hipLaunchKernelGGL(k_sig_sum, dim3(grid_of(mb, cu)), dim3(kT), 0, st, (int64_t)mb, xbits,
                         keys, sd, sig);
    }
    BISIM_TRY_HIP(hipGetLastError());
    sorted_keys = mb;
    return BISIM_OK;
  };

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
      BISIM_TRY(signatures(seed, rounds == kSortedRounds));
      BISIM_TRY_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), st));
      if (group_hash) {
        hipLaunchKernelGGL(k_state_keys, dim3(grid_of(n, cu)), dim3(kT), 0, st, n, ~0ull, blk, sig,
                           hk, idx);
        hipLaunchKernelGGL(k_fill_u64, dim3(grid_of(tsz, cu)), dim3(kT), 0, st, gtab,
                           (int64_t)tsz, kEmpty);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_of(tsz, cu)), dim3(kT), 0, st, gval,
                           (int64_t)tsz, (int32_t)0x7FFFFFFF);
        hipLaunchKernelGGL(k_group_insert, dim3(grid_of(n, cu)), dim3(kT), 0, st, n, hk, gtab,
                           gval, tsz - 1u, idxs, cnt, fail);
        hipLaunchKernelGGL(k_group_assign, dim3(grid_of(n, cu)), dim3(kT), 0, st, n, idxs, gval,
                           nb);
      } else {
        hipLaunchKernelGGL(k_state_keys, dim3(grid_of(n, cu)), dim3(kT), 0, st, n, hmask, blk,
                           sig, hk, idx);
        BISIM_TRY(radix_sort_u64(temp, tb, hk, hks, (const uint32_t*)idx, (uint32_t*)idxs, n, 0,
                                 hbits, st));
        hipLaunchKernelGGL(k_heads, dim3(grid_of(n, cu)), dim3(kT), 0, st, n, hks, hp, cnt);
        BISIM_TRY(inclusive_max_scan_u32((const uint32_t*)hp, (uint32_t*)hp2, n, st));
        hipLaunchKernelGGL(k_assign, dim3(grid_of(n, cu)), dim3(kT), 0, st, n, idxs, hp2, nb);
      }
      BISIM_TRY_HIP(hipGetLastError());
      unsigned long long hc[3] = {0, 0, 0};
      BISIM_TRY_HIP(hipMemcpyAsync(hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, st));
      BISIM_TRY_HIP(hipStreamSynchronize(st));
      const unsigned long long c = hc[0];
      if (hc[2] != 0) {
        set_error("signature refinement: a hash table overflowed");
        return BISIM_E_DEVICE;
      }
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
    // check with an independent hash of the final partition's signatures
    // (the last round's sorted keys hold them: at the fixpoint its partition,
    // named by smallest states, is the final one), or, after a stall, only
    // that pi_pre is refined
    if (fixpoint) {
      const uint64_t sd = seed ^ 0xD1B54A32D192ED03ull;
      BISIM_TRY_HIP(hipMemsetAsync(sig, 0, sizeof(uint64_t) * n, st));
      if (sorted_keys < m) {  // the last round ran on the layout
        hipLaunchKernelGGL(k_sig_small, dim3(grid_of(m, cu)), dim3(kT), 0, st, m, o_src, o_rn,
                           o_tgt, out_ptr, blk, sd, sig);
        if (big_hash) BISIM_TRY(big_by_table(sd));
      }
      if (sorted_keys > 0)
        hipLaunchKernelGGL(k_sig_sum, dim3(grid_of(sorted_keys, cu)), dim3(kT), 0, st,
                           sorted_keys, xbits, keys, sd, sig);
      BISIM_TRY_HIP(hipGetLastError());
    }
    BISIM_TRY_HIP(hipMemsetAsync(cnt + 1, 0, sizeof(unsigned long long), st));
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
