// Batched refinement of many independent LTSs in one launch.
//
// Loading: the instances are shifted into one id space (instance k's states
// start at n_off[k]; its initial blocks stay separate) and preprocessed
// together by the single-instance loader: the preprocessing is per state and
// per transition, and no block ever spans two instances, so the result is
// every instance's own preprocessing side by side.
//
// Refinement: one launch of a kernel whose workgroups claim instances from a
// device queue (largest first).  A workgroup runs the whole Algorithm 3 loop
// of its instance with workgroup barriers between the phases (select+mark,
// compare+elect, relabel), exactly as the single-instance engines do with grid
// barriers, so every instance gets the same splitter sequence and #It as a
// single-instance run.  Instance state (block ids, mark words, new-leader
// bids, unstable/touched/leader-touched bitmaps) lives in LDS when it fits the
// workgroup's LDS budget and in a global-memory slice otherwise.  The
// workgroup size, LDS budget and grid are chosen by an autotuner that times
// candidate configurations and caches the winner per device and batch shape.
// The queue reset and the launch are captured once into a hipGraph and
// replayed.
#include <sys/stat.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

struct bisim_batch {
  int32_t count = 0;
  int64_t N = 0, M = 0;
  int32_t Kmax = 1;
  hipStream_t stream = nullptr;
  hipStream_t own_stream = nullptr;
  int device = 0, num_cu = 0;
  int lds_max = 0;
  bisim_lts* u = nullptr;  // the preprocessed union
  std::vector<int64_t> n_off;
  uint32_t* n_off_d = nullptr;  // [count+1]
  uint32_t* bw_off_d = nullptr; // [count+1] bitmap word offsets
  int32_t* order_d = nullptr;   // instance ids, largest first
  int mask64 = 1;               // 64-bit mark words (else 32-bit)
  // global-tier scratch
  int32_t* blk = nullptr;
  uint64_t* mw = nullptr;
  uint64_t* nlb = nullptr;
  uint64_t* ub = nullptr;
  uint64_t* tb = nullptr;
  uint64_t* lt = nullptr;
  int32_t* tl = nullptr;
  int32_t* sl = nullptr;
  // member-list tier scratch
  int32_t *perm = nullptr, *pos = nullptr, *bs = nullptr, *be = nullptr, *cnt = nullptr,
          *fc = nullptr, *gc = nullptr, *tmp = nullptr, *rk = nullptr, *fi = nullptr,
          *ob = nullptr, *nev = nullptr, *ltl = nullptr, *tlb = nullptr, *se = nullptr,
          *sgs = nullptr, *llo = nullptr, *lsz = nullptr;
  uint64_t *sf = nullptr, *us = nullptr, *tmp64 = nullptr, *pin = nullptr;
  uint32_t* iters_d = nullptr;  // [count]
  uint32_t* ctl_d = nullptr;    // [0] queue head, [1] error
  unsigned long long* work_d = nullptr;  // [16] work totals per tier
  // options / tuning
  int opt_wg = 0, opt_grid = 0, opt_lds = 0, opt_retune = 0;
  int wg = 0, grid = 0, lds_bytes = 0;
  bool tuned = false;
  hipGraphExec_t gexec = nullptr;
  int g_wg = -1, g_grid = -1, g_lds = -1;
  int32_t* g_out = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double t_pre_ms = 0, t_alg_ms = 0;
  int64_t lds_inst = 0, glob_inst = 0;
};

namespace bisim {
bisim_status lts_create_union(int32_t n, int64_t m, int32_t K, const int32_t* src,
                              const int32_t* lab, const int32_t* dst, const int32_t* init,
                              hipStream_t stream, bisim_lts** out);
void lts_destroy(bisim_lts* h);

namespace {
constexpr int kT = 256;

struct BArgs {
  int32_t count;
  const uint32_t* __restrict__ n_off;
  const uint32_t* __restrict__ bw_off;
  const int32_t* __restrict__ order;
  const int32_t* __restrict__ pre_block;
  const uint32_t* __restrict__ in_ptr;
  const int32_t* __restrict__ in_src;
  const int32_t* __restrict__ in_ord;
  int32_t* blk;
  void* mw;
  uint64_t* nlb;
  uint64_t* ub;
  uint64_t* tb;
  uint64_t* lt;
  int32_t* tl;
  int32_t* sl;
  int32_t *perm, *pos, *bs, *be, *cnt, *fc, *gc, *tmp, *rk, *fi, *ob, *nev, *ltl, *tlb, *se, *sgs,
      *llo, *lsz;
  uint64_t *sf, *us, *tmp64, *pin;
  int32_t* out;
  uint32_t* iters;
  uint32_t* ctl;
  unsigned long long* work;  // [2][8] totals per tier (see bisim_batch_stats)
  uint32_t lds_bytes;
};

__device__ __forceinline__ uint32_t atomic_or(uint32_t* p, uint32_t v) { return atomicOr(p, v); }
__device__ __forceinline__ uint64_t atomic_or(uint64_t* p, uint64_t v) {
  return atomicOr((unsigned long long*)p, (unsigned long long)v);
}

template <class MaskT>
struct WArr {
  int32_t* blk;
  MaskT* mw;
  uint64_t* nlb;
  uint64_t* ub;
  uint64_t* tb;
  uint64_t* lt;
};

template <class MaskT>
__host__ __device__ inline uint64_t lds_need(uint32_t n) {
  const uint64_t nw = (n + 63u) / 64u;
  return 8ull * 3 * nw + 8ull * n + ((sizeof(MaskT) * (uint64_t)n + 7) & ~7ull) + 4ull * n;
}

constexpr uint32_t kCU = 4;  // member-list tier: split-list entries per thread and step
constexpr int kBatchWG = 256;  // the one workgroup size the batched kernel is built for

struct Shared {
  uint32_t cand[2];
  uint32_t nT[2];
  uint32_t nS[2];
  uint32_t ltany[2];
  uint32_t nL[2];  // member-list tier: touched leaders
  uint32_t wsum[16];  // member-list tier: per-wave sums of the block-size scan
  uint32_t bad;       // member-list tier: inconsistent block sizes (never expected)
  uint32_t job;
  // work totals of the current instance: in-transitions of the splitters,
  // splitter members (LDS tier), member visits and split blocks (member lists)
  unsigned long long wE, wM, wV, wB;
};

__device__ __forceinline__ void wg_min(uint32_t* dst, uint32_t v) {
  v = wave_min_u32(v);
  if (lane() == 0 && v != kNone) atomicMin(dst, v);
}

// Append for lanes with pred; one LDS atomic per wave.  Wave-uniform call.
__device__ __forceinline__ void push(int32_t* list, uint32_t* cnt, int32_t v, bool pred) {
  uint64_t bal = __ballot(pred);
  if (!bal) return;
  int leader = __ffsll((unsigned long long)bal) - 1;
  uint32_t base = 0;
  if ((int)lane() == leader) base = atomicAdd(cnt, (uint32_t)__popcll(bal));
  base = (uint32_t)__shfl((int)base, leader, kWave);
  if (pred) list[base + __popcll(bal & ((1ull << lane()) - 1ull))] = v;
}

// The whole refinement loop of one instance by one workgroup; U chunks of 64
// states per wave and step in the scans over all states of the instance.
template <class MaskT, uint32_t U>
__device__ __forceinline__ uint32_t wg_refine(const BArgs& a, Shared& sh, WArr<MaskT> w,
                                              int32_t* T, int32_t* S, uint32_t s0, uint32_t n) {
  const uint32_t tid = threadIdx.x, nthr = blockDim.x;
  const uint32_t wid = tid / kWave, nwav = nthr / kWave;
  const uint32_t nw = (n + 63u) >> 6;
  for (uint32_t s = tid; s < n; s += nthr) {
    w.blk[s] = a.pre_block[s0 + s] - (int32_t)s0;
    w.mw[s] = 0;
    w.nlb[s] = 0;
  }
  for (uint32_t q = tid; q < nw; q += nthr) {
    uint64_t bits = 0;
    for (uint32_t j = 0; j < 64 && (q << 6) + j < n; ++j)
      if ((uint32_t)(a.pre_block[s0 + (q << 6) + j] - (int32_t)s0) == (q << 6) + j)
        bits |= 1ull << j;
    w.ub[q] = bits;
    w.tb[q] = 0;
    w.lt[q] = 0;
  }
  if (tid == 0) {
    sh.cand[0] = n ? 0u : kNone;
    sh.cand[1] = kNone;
    sh.nT[0] = sh.nT[1] = sh.nS[0] = sh.nS[1] = 0;
    sh.ltany[0] = sh.ltany[1] = 0;
    sh.wE = sh.wM = 0;
  }
  __syncthreads();
  const uint32_t cap = 3u * n + 1u;
  uint32_t it = 0;
  uint64_t sT = 0, sS = 0;  // work totals (thread 0)
  for (;; ++it) {
    const uint32_t par = it & 1;
    const uint32_t C = sh.cand[par];
    if (C == kNone) break;
    if (it + 1 > cap) {
      if (tid == 0) atomicOr(&a.ctl[1], 1u);
      break;
    }
    const uint64_t epoch = (uint64_t)(it + 1) << 32;
    // ---- A: select next candidate, mark
    {
      uint32_t best = kNone;
      for (uint32_t q = tid; q < nw; q += nthr) {
        uint64_t bits = w.ub[q];
        if (q == (C >> 6)) {
          bits &= ~(1ull << (C & 63));
          w.ub[q] = bits;
        }
        if (bits) best = min(best, (q << 6) + (uint32_t)(__ffsll((unsigned long long)bits) - 1));
      }
      wg_min(&sh.cand[par ^ 1], best);
      if (tid == 0) {
        sh.nT[par ^ 1] = 0;
        sh.nS[par ^ 1] = 0;
        sh.ltany[par ^ 1] = 0;
      }
      // U chunks of 64 states per wave and step: their block ids are loaded
      // together, so a step waits for one memory latency, not U
      for (uint32_t base0 = wid * kWave * U; base0 < n; base0 += nwav * kWave * U) {
        const uint32_t hm = hit_mask<U>(w.blk, base0, n, C);
        if (__ballot(hm != 0) == 0) continue;
       for (uint32_t u = 0; u < U; ++u) {
        const uint32_t base = base0 + u * kWave;
        const uint32_t t = base + lane();
        const bool hit = (hm >> u) & 1u;
        const uint64_t hb = __ballot(hit);
        if (hb == 0) continue;
        uint32_t beg = 0, deg = 0;
        if (hit) {
          beg = a.in_ptr[s0 + t];
          deg = a.in_ptr[s0 + t + 1] - beg;
        }
        const uint32_t incl = wave_incl_scan_u32(deg);
        const uint32_t total = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
        if (lane() == 0) {
          atomicAdd(&sh.wE, (unsigned long long)total);
          atomicAdd(&sh.wM, (unsigned long long)__popcll(hb));
        }
        for (uint32_t e0 = 0; e0 < total; e0 += kWave) {
          const uint32_t e = e0 + lane();
          const bool valid = e < total;
          const uint32_t ee = valid ? e : total - 1;
          uint32_t j = 0;
#pragma unroll
          for (uint32_t step = 32; step >= 1; step >>= 1) {
            const uint32_t probe = (uint32_t)__shfl((int)incl, (int)(j + step - 1), kWave);
            if (probe <= ee) j += step;
          }
          const uint32_t jb = (uint32_t)__shfl((int)beg, (int)j, kWave);
          const uint32_t ji = (uint32_t)__shfl((int)incl, (int)j, kWave);
          const uint32_t jd = (uint32_t)__shfl((int)deg, (int)j, kWave);
          bool first = false;
          int32_t s = 0;
          if (valid) {
            const uint32_t edge = jb + (ee - (ji - jd));
            s = a.in_src[edge] - (int32_t)s0;
            const int32_t o = a.in_ord[edge];
            const MaskT bit = (MaskT)1 << (o & (int)(sizeof(MaskT) * 8 - 1));
            const MaskT old = atomic_or(&w.mw[s], bit);
            first = (old == 0);
            if (first) {
              const uint64_t tbit = 1ull << (s & 63);
              atomicOr((unsigned long long*)&w.tb[s >> 6], (unsigned long long)tbit);
              if (w.blk[s] == s) {
                atomicOr((unsigned long long*)&w.lt[s >> 6], (unsigned long long)tbit);
                sh.ltany[par] = 1;
              }
            }
          }
          push(T, &sh.nT[par], s, first);
        }
       }
      }
    }
    __syncthreads();
    // ---- B: compare with the leader, elect
    {
      const uint32_t nT = sh.nT[par];
      for (uint32_t i0 = wid * kWave; i0 < nT; i0 += nwav * kWave) {
        const uint32_t i = i0 + lane();
        bool sp = false;
        int32_t s = 0, b = 0;
        if (i < nT) {
          s = T[i];
          b = w.blk[s];
          sp = (s != b) && (w.mw[s] != w.mw[b]);
        }
        if (sp)
          atomicMax((unsigned long long*)&w.nlb[b],
                    (unsigned long long)(epoch | (uint64_t)(kNone - (uint32_t)s)));
        push(S, &sh.nS[par], s, sp);
      }
      if (sh.ltany[par]) {
        for (uint32_t base0 = wid * kWave * U; base0 < n; base0 += nwav * kWave * U) {
          // block ids, then leader-touched bits, then touched bits of U
          // chunks: three memory latencies per step
          int32_t bv[U];
          uint64_t lw[U], tw[U];
#pragma unroll
          for (uint32_t u = 0; u < U; ++u) {
            const uint32_t s = base0 + u * kWave + lane();
            bv[u] = s < n ? w.blk[s] : 0;
          }
#pragma unroll
          for (uint32_t u = 0; u < U; ++u) lw[u] = w.lt[(uint32_t)bv[u] >> 6];
#pragma unroll
          for (uint32_t u = 0; u < U; ++u)
            tw[u] = base0 + u * kWave < n ? w.tb[(base0 + u * kWave) >> 6] : 0ull;
#pragma unroll
          for (uint32_t u = 0; u < U; ++u) {
            const uint32_t s = base0 + u * kWave + lane();
            const int32_t b = bv[u];
            const bool sp = s < n && ((lw[u] >> (b & 63)) & 1ull) && !((tw[u] >> (s & 63)) & 1ull);
            if (sp)
              atomicMax((unsigned long long*)&w.nlb[b],
                        (unsigned long long)(epoch | (uint64_t)(kNone - s)));
            push(S, &sh.nS[par], (int32_t)s, sp);
          }
        }
      }
    }
    __syncthreads();
    // ---- C: relabel, unstable updates, clear marks
    {
      const uint32_t nS = sh.nS[par], nT = sh.nT[par];
      if (tid == 0) {
        sT += nT;
        sS += nS;
      }
      uint32_t best = kNone;
      for (uint32_t i = tid; i < nS; i += nthr) {
        const int32_t s = S[i];
        const int32_t old = w.blk[s];
        const int32_t nl = (int32_t)(kNone - (uint32_t)w.nlb[old]);
        w.blk[s] = nl;
        if (s == nl) {
          atomicOr((unsigned long long*)&w.ub[old >> 6], 1ull << (old & 63));
          atomicOr((unsigned long long*)&w.ub[nl >> 6], 1ull << (nl & 63));
          best = min(best, (uint32_t)old);
        }
      }
      for (uint32_t i = tid; i < nT; i += nthr) {
        const int32_t s = T[i];
        w.mw[s] = 0;
        w.tb[s >> 6] = 0;
        w.lt[s >> 6] = 0;
      }
      wg_min(&sh.cand[par ^ 1], best);
      if (tid == 0) {
        if (nS > 0) {
          atomicOr((unsigned long long*)&w.ub[C >> 6], 1ull << (C & 63));
          atomicMin(&sh.cand[par ^ 1], C);
        }
        sh.cand[par] = kNone;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    atomicAdd(&a.work[0], (unsigned long long)(it + 1));
    atomicAdd(&a.work[1], sh.wM);
    atomicAdd(&a.work[2], sh.wE);
    atomicAdd(&a.work[3], (unsigned long long)sT);
    atomicAdd(&a.work[5], (unsigned long long)sS);
    atomicAdd(&a.work[7], 1ull);
  }
  for (uint32_t s = tid; s < n; s += nthr) a.out[s0 + s] = w.blk[s];
  return it + 1;
}

// Member-list tier (instances too large for LDS): the partition is also kept
// as a refinable partition, so an iteration visits C's members, the touched
// states and the members of blocks whose leader was touched instead of all
// n states.  perm lists the states block by block; block b (a label) owns
// perm[bs[b] .. be[b]).  A split moves the split-off states to the end of the
// block's range by swaps and gives that tail to the new label.
//
// One workgroup refines the instance; every phase is a chain of dependent
// global-memory round trips, so the layout keeps that chain short: the
// unstable, touched and split bitmaps (and the unstable summary) sit in LDS
// when they fit beside a minimum of list space, and so do the per-iteration
// lists (touched states with their block, touched leaders with their block's
// range, split states with everything the later phases need); list entries
// beyond the LDS capacity spill to per-instance global arrays.  A state's
// block and, should it lead that block, the block's range are loaded together
// at its first touch.  The wave that finds the next splitter also loads its
// range and its first members' in-transition ranges into LDS; when nothing
// splits in the iteration (most iterations) the next one starts marking from
// there.  Ranks within a block's split part are taken when the split is found,
// so the relabel and the search for staying states in the tail run in one
// phase, and the staying state found for a tail position is stored with it,
// so the swap is one more round trip.
struct GList {
  int32_t* perm;    // [n] states ordered by block
  int32_t* pos;     // [n] position of each state in perm
  int32_t* bs;      // [n] per label: first position of its block
  int32_t* be;      // [n] per label: one past the last position
  int32_t* cnt;     // [n] per label: states split off this iteration (0 between iterations)
  int32_t* fc;      // [n] per label: split states found in the front part
  int32_t* gc;      // [n] per label: staying states found in the tail
  uint64_t* tmp64;  // [n] per tail position: (staying state << 32) | its position, by index
  uint64_t* pin;    // [n] per position p: in-transition range of perm[p] (first edge << 32 | count)
  // global spill of the lists (entry i >= the LDS capacity)
  int32_t *ts, *tb_, *lb, *llo, *lsz, *ss, *sb_, *sr, *sf_, *sn, *sp, *se, *sgs;
  uint64_t* sf;     // [ceil(n/64)] split flags (global fallback)
  uint64_t* ml;     // [ceil(n/64)] labels of blocks with more than one state (global fallback)
  uint64_t* us;     // [ceil(n/4096)] summary of the unstable bitmap (global fallback)
};

// A list field: entry i in LDS when i < cap, else in global memory.
struct LField {
  int32_t* l;
  int32_t* g;
};
__device__ __forceinline__ int32_t* ent(const LField& f, uint32_t cap, uint32_t i) {
  return i < cap ? f.l + i : f.g + i;
}

// Append one entry for lanes with pred (one LDS atomic per wave); returns the
// entry's index, or kNone for lanes without pred.  Wave-uniform call.
__device__ __forceinline__ uint32_t push_idx(uint32_t* cnt, bool pred) {
  const uint64_t bal = __ballot(pred);
  if (!bal) return kNone;
  const int leader = __ffsll((unsigned long long)bal) - 1;
  uint32_t base = 0;
  if ((int)lane() == leader) base = atomicAdd(cnt, (uint32_t)__popcll(bal));
  base = (uint32_t)__shfl((int)base, leader, kWave);
  return pred ? base + (uint32_t)__popcll(bal & ((1ull << lane()) - 1ull)) : kNone;
}

// Set unstable bit b and keep the summary exact (sets only; the one clear per
// iteration happens in the selection, never concurrently with sets).
__device__ __forceinline__ void wg_unstable_set(uint64_t* ub, uint64_t* us, uint32_t b) {
  const uint32_t w = b >> 6;
  const uint64_t old = atomicOr((unsigned long long*)&ub[w], 1ull << (b & 63));
  if (old == 0) atomicOr((unsigned long long*)&us[w >> 6], 1ull << (w & 63));
}

// bytes of LDS per unit of list capacity: touched (state, block), touched
// leader (state, first position, size), split (state, block, rank, front
// index, tail start, position, end, start of the block's range)
constexpr uint32_t kListBytes = 4u * (2 + 3 + 8);
constexpr uint32_t kMinListCap = 256;
// the next splitter, prefetched: two slots by iteration parity, each a header
// (label, first position, size, valid) and the in-transition ranges (first
// edge, count) of its first kWave members
constexpr uint32_t kPfWords = 4u + 2u * kWave;
constexpr uint32_t kPfBytes = 4u * 2u * kPfWords;

// The refinement loop of one instance by one workgroup, member-list tier.
// Same phases and the same splitter sequence as wg_refine.
template <class MaskT>
__device__ uint32_t wg_refine_lists(const BArgs& a, Shared& sh, int32_t* blk, MaskT* mw,
                                    uint64_t* nlb, GList g, uint64_t* lds, uint32_t lds_bytes,
                                    uint64_t* gub, uint64_t* gtb, uint32_t s0, uint32_t n) {
  const uint32_t tid = threadIdx.x, nthr = blockDim.x;
  const uint32_t wid = tid / kWave, nwav = nthr / kWave;
  const uint32_t nw = (n + 63u) >> 6, nsw = (nw + 63u) >> 6;
  // LDS: bitmaps first (when they fit beside the prefetch slots and
  // kMinListCap list entries), the prefetch slots, then lists
  const uint32_t bm_bytes = 8u * (4u * nw + nsw);
  const bool bm_lds = bm_bytes + kPfBytes + kMinListCap * kListBytes <= lds_bytes;
  uint64_t *ub, *tb, *sf, *ml, *us;
  char* lp = reinterpret_cast<char*>(lds);
  uint32_t lbytes = lds_bytes;
  if (bm_lds) {
    ub = lds;
    tb = lds + nw;
    sf = lds + 2 * nw;
    ml = lds + 3 * nw;
    us = lds + 4 * nw;
    lp += bm_bytes;
    lbytes -= bm_bytes;
  } else {
    ub = gub;
    tb = gtb;
    sf = g.sf;
    ml = g.ml;
    us = g.us;
  }
  // the prefetch slots, when the LDS left holds them ([2][kPfWords])
  const bool pf_on = lbytes >= kPfBytes;
  uint32_t* pf = reinterpret_cast<uint32_t*>(lp);
  if (pf_on) {
    lp += kPfBytes;
    lbytes -= kPfBytes;
  }
  const uint32_t cap = lbytes / kListBytes;
  int32_t* li = reinterpret_cast<int32_t*>(lp);
  const LField Ts{li, g.ts}, Tb{li + cap, g.tb_}, Lb{li + 2 * cap, g.lb},
      Llo{li + 3 * cap, g.llo}, Lsz{li + 4 * cap, g.lsz};
  const LField Ss{li + 5 * cap, g.ss}, Sb{li + 6 * cap, g.sb_}, Sr{li + 7 * cap, g.sr},
      Sf{li + 8 * cap, g.sf_}, Sn{li + 9 * cap, g.sn}, Sp{li + 10 * cap, g.sp},
      Se{li + 11 * cap, g.se}, Sg{li + 12 * cap, g.sgs};

  // ---- initial state: blocks of the preprocessed partition, all unstable
  for (uint32_t s = tid; s < n; s += nthr) {
    blk[s] = a.pre_block[s0 + s] - (int32_t)s0;
    mw[s] = 0;
    nlb[s] = 0;
    g.cnt[s] = 0;
    g.fc[s] = 0;
    g.gc[s] = 0;
  }
  for (uint32_t q = tid; q < nw; q += nthr) {
    uint64_t bits = 0;
    for (uint32_t j = 0; j < 64 && (q << 6) + j < n; ++j)
      if ((uint32_t)(a.pre_block[s0 + (q << 6) + j] - (int32_t)s0) == (q << 6) + j)
        bits |= 1ull << j;
    ub[q] = bits;
    tb[q] = 0;
    sf[q] = 0;
    ml[q] = 0;
  }
  for (uint32_t q = tid; q < nsw; q += nthr) us[q] = 0;
  if (pf_on && tid < 2) pf[tid * kPfWords + 3] = 0;
  if (tid == 0) {
    sh.cand[0] = n ? 0u : kNone;
    sh.cand[1] = kNone;
    sh.nT[0] = sh.nT[1] = sh.nS[0] = sh.nS[1] = 0;
    sh.nL[0] = sh.nL[1] = 0;
    sh.bad = 0;
    sh.wE = sh.wV = sh.wB = 0;
  }
  __syncthreads();
  for (uint32_t q = tid; q < nw; q += nthr)
    if (ub[q]) atomicOr((unsigned long long*)&us[q >> 6], 1ull << (q & 63));
  for (uint32_t s = tid; s < n; s += nthr) atomicAdd(&g.cnt[blk[s]], 1);
  __syncthreads();
  // block ranges: exclusive prefix sums of the block sizes in label order
  // (thread-contiguous label ranges; wave scan, then the <= 16 wave totals)
  {
    const uint32_t per = (n + nthr - 1) / nthr;
    const uint32_t lo = min(n, tid * per), hi = min(n, lo + per);
    uint32_t sum = 0;
    for (uint32_t b = lo; b < hi; ++b) sum += (uint32_t)g.cnt[b];
    const uint32_t incl = wave_incl_scan_u32(sum);
    if (lane() == kWave - 1) sh.wsum[wid] = incl;
    __syncthreads();
    uint32_t run = incl - sum;
    for (uint32_t q = 0; q < wid; ++q) run += sh.wsum[q];
    for (uint32_t b = lo; b < hi; ++b) {
      const uint32_t c = (uint32_t)g.cnt[b];
      g.bs[b] = (int32_t)run;
      g.be[b] = (int32_t)run;  // fill cursor, ends at the block's end
      if (c > 1) atomicOr((unsigned long long*)&ml[b >> 6], 1ull << (b & 63));
      run += c;
    }
  }
  __syncthreads();
  for (uint32_t s = tid; s < n; s += nthr) {
    const uint32_t p = (uint32_t)atomicAdd(&g.be[blk[s]], 1);
    if (p >= n) {  // cannot happen with consistent counts; report, never write
      sh.bad = 1;
      continue;
    }
    g.perm[p] = (int32_t)s;
    g.pos[s] = (int32_t)p;
    const uint32_t e0 = a.in_ptr[s0 + s];
    g.pin[p] = ((uint64_t)e0 << 32) | (a.in_ptr[s0 + s + 1] - e0);
  }
  __syncthreads();
  if (sh.bad) {  // workgroup-uniform
    if (tid == 0) atomicOr(&a.ctl[1], 2u);
    return 0;
  }
  for (uint32_t s = tid; s < n; s += nthr) g.cnt[s] = 0;
  __syncthreads();

  const uint32_t itcap = 3u * n + 1u;
  uint32_t it = 0;
  uint64_t sM = 0, sT = 0, sL = 0, sS = 0;  // work totals (thread 0)
  for (;; ++it) {
    const uint32_t par = it & 1;
    const uint32_t C = sh.cand[par];
    if (C == kNone) break;
    if (it + 1 > itcap) {
      if (tid == 0) atomicOr(&a.ctl[1], 1u);
      break;
    }
    const uint64_t epoch = (uint64_t)(it + 1) << 32;
    // ---- A: clear C, next candidate (one wave, through the summary), mark.
    // The search runs on the last wave: marking a small splitter's
    // in-transitions falls to the first waves.  A state's first touch (its
    // touched bit set by this lane) lists it with its block, and a touched
    // leader of a block with more than one state is listed with the block's
    // range.  The range of C and its first members' in-transition ranges come
    // from the prefetch slot when the previous iteration filled it for C and
    // split nothing.
    uint32_t next = kNone;
    if (wid == nwav - 1) {
      const uint32_t w0 = C >> 6;
      const uint64_t bits = ub[w0] & ~(1ull << (C & 63));
      if (lane() == 0) {
        ub[w0] = bits;
        if (bits == 0) atomicAnd((unsigned long long*)&us[w0 >> 6], ~(1ull << (w0 & 63)));
      }
      // C is the smallest unstable label: the next one is the next set bit
      for (uint32_t q = w0 >> 6; q < nsw; q += kWave) {
        const uint32_t qq = q + lane();
        uint64_t sv = qq < nsw ? us[qq] : 0ull;
        if (qq == (w0 >> 6)) {
          sv &= ~0ull << (w0 & 63);
          const uint64_t b0 = 1ull << (w0 & 63);
          sv = bits ? (sv | b0) : (sv & ~b0);
        }
        const uint64_t bal = __ballot(sv != 0);
        if (bal) {
          const int l = __ffsll((unsigned long long)bal) - 1;
          const uint64_t v = (uint64_t)__shfl((unsigned long long)sv, l, kWave);
          const uint32_t word = ((q + (uint32_t)l) << 6) + (uint32_t)(__ffsll((unsigned long long)v) - 1);
          const uint64_t wb = (word == w0) ? bits : ub[word];
          if (wb) next = (word << 6) + (uint32_t)(__ffsll((unsigned long long)wb) - 1);
          break;
        }
      }
      if (lane() == 0 && next != kNone) atomicMin(&sh.cand[par ^ 1], next);
    }
    if (tid == 0) {
      sh.nT[par ^ 1] = 0;
      sh.nS[par ^ 1] = 0;
      sh.nL[par ^ 1] = 0;
    }
    {
      const uint32_t* pc = pf + par * kPfWords;  // filled in the previous iteration
      const bool pre = pf_on && pc[3] != 0 && pc[0] == C;
      uint32_t cb, csz;
      if (pre) {
        cb = pc[1];
        csz = pc[2];
      } else {
        cb = (uint32_t)g.bs[C];
        csz = (uint32_t)g.be[C] - cb;
        if (cb > n || csz > n - cb) {  // never expected: report, visit nothing
          sh.bad = 1;
          csz = 0;
        }
      }
      if (tid == 0) sM += csz;
      for (uint32_t i0 = wid * kWave; i0 < csz; i0 += nwav * kWave) {
        const uint32_t i = i0 + lane();
        const bool hit = i < csz;
        uint32_t beg = 0, deg = 0;
        if (hit) {
          if (pre && i0 == 0) {
            beg = pc[4 + lane()];
            deg = pc[4 + kWave + lane()];
          } else {
            const uint64_t x = g.pin[cb + i];
            beg = (uint32_t)(x >> 32);
            deg = (uint32_t)x;
          }
        }
        const uint32_t incl = wave_incl_scan_u32(deg);
        const uint32_t total = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
        if (lane() == 0 && total) atomicAdd(&sh.wE, (unsigned long long)total);
        for (uint32_t e0 = 0; e0 < total; e0 += kWave) {
          const uint32_t e = e0 + lane();
          const bool valid = e < total;
          const uint32_t ee = valid ? e : total - 1;
          uint32_t j = 0;
#pragma unroll
          for (uint32_t step = 32; step >= 1; step >>= 1) {
            const uint32_t probe = (uint32_t)__shfl((int)incl, (int)(j + step - 1), kWave);
            if (probe <= ee) j += step;
          }
          const uint32_t jb = (uint32_t)__shfl((int)beg, (int)j, kWave);
          const uint32_t ji = (uint32_t)__shfl((int)incl, (int)j, kWave);
          const uint32_t jd = (uint32_t)__shfl((int)deg, (int)j, kWave);
          bool first = false, lead = false;
          int32_t s = 0, b = 0, lo = 0, hi = 0;
          if (valid) {
            const uint32_t edge = jb + (ee - (ji - jd));
            s = a.in_src[edge] - (int32_t)s0;
            const int32_t o = a.in_ord[edge];
            const MaskT bit = (MaskT)1 << (o & (int)(sizeof(MaskT) * 8 - 1));
            atomic_or(&mw[s], bit);
            const uint64_t tbit = 1ull << (s & 63);
            const uint64_t old =
                atomicOr((unsigned long long*)&tb[s >> 6], (unsigned long long)tbit);
            first = !(old & tbit);
            // a touched leader of a one-state block has no untouched member;
            // a leader of a larger one is listed with its block's range,
            // loaded beside its block id
            lead = first && test_bit(ml, (uint32_t)s);
            if (first) b = blk[s];
            if (lead) {
              lo = g.bs[s];
              hi = g.be[s];
            }
          }
          const uint32_t ti = push_idx(&sh.nT[par], first);
          if (first) {
            *ent(Ts, cap, ti) = s;
            *ent(Tb, cap, ti) = b;
          }
          const uint32_t li_ = push_idx(&sh.nL[par], lead);
          if (lead) {
            *ent(Lb, cap, li_) = s;
            *ent(Llo, cap, li_) = lo;
            *ent(Lsz, cap, li_) = hi - lo;
          }
        }
      }
    }
    // prefetch for the next iteration (slot par ^ 1): the candidate found
    // above, its range and its first kWave members' in-transition ranges.
    // Valid only if the candidate stands and nothing splits in this iteration
    // (then no range, member list or candidate changes); the split phase
    // clears it otherwise.
    if (pf_on && wid == nwav - 1) {
      uint32_t* pn = pf + (par ^ 1) * kPfWords;
      uint32_t ncb = 0, nsz = 0;
      bool ok = false;
      if (next != kNone) {
        ncb = (uint32_t)g.bs[next];
        nsz = (uint32_t)g.be[next] - ncb;
        ok = ncb <= n && nsz <= n - ncb;
      }
      uint32_t beg = 0, deg = 0;
      if (ok && lane() < nsz) {
        const uint64_t x = g.pin[ncb + lane()];
        beg = (uint32_t)(x >> 32);
        deg = (uint32_t)x;
      }
      pn[4 + lane()] = beg;
      pn[4 + kWave + lane()] = deg;
      if (lane() == 0) {
        pn[0] = next;
        pn[1] = ncb;
        pn[2] = nsz;
        pn[3] = ok ? 1u : 0u;
      }
    }
    __syncthreads();
    // ---- B: compare touched states with their leader; untouched members of
    // blocks whose leader was touched differ from it.  A split state bids for
    // its block's new leader, takes its rank within the block's split part
    // and sets its split flag.
    {
      const uint32_t nT = sh.nT[par];
      for (uint32_t i0 = tid; i0 < nT; i0 += nthr * kCU) {
        int32_t sv[kCU], bv[kCU];
        MaskT ms[kCU], mb[kCU];
#pragma unroll
        for (uint32_t u = 0; u < kCU; ++u) {
          const uint32_t i = i0 + u * nthr;
          sv[u] = i < nT ? *ent(Ts, cap, i) : -1;
          bv[u] = i < nT ? *ent(Tb, cap, i) : 0;
        }
#pragma unroll
        for (uint32_t u = 0; u < kCU; ++u) {
          ms[u] = sv[u] >= 0 ? mw[sv[u]] : (MaskT)0;
          mb[u] = sv[u] >= 0 ? mw[bv[u]] : (MaskT)0;
        }
#pragma unroll
        for (uint32_t u = 0; u < kCU; ++u) {
          const bool sp = sv[u] >= 0 && sv[u] != bv[u] && ms[u] != mb[u];
          int32_t r = 0;
          if (sp) {
            atomicMax((unsigned long long*)&nlb[bv[u]],
                      (unsigned long long)(epoch | (uint64_t)(kNone - (uint32_t)sv[u])));
            r = atomicAdd(&g.cnt[bv[u]], 1);
            atomicOr((unsigned long long*)&sf[sv[u] >> 6], 1ull << (sv[u] & 63));
          }
          const uint32_t si = push_idx(&sh.nS[par], sp);
          if (sp) {
            *ent(Ss, cap, si) = sv[u];
            *ent(Sb, cap, si) = bv[u];
            *ent(Sr, cap, si) = r;
          }
        }
      }
      // members of the blocks whose leader was touched, 64 blocks at a time:
      // their member slots are spread over all waves by a prefix sum of the
      // block sizes (a block can hold most of the instance); each listed
      // leader carries its block's range
      const uint32_t nL = sh.nL[par];
      for (uint32_t j0 = 0; j0 < nL; j0 += kWave) {
        const uint32_t j = j0 + lane();
        int32_t b = 0;
        uint32_t lo = 0, sz = 0;
        if (j < nL) {
          b = *ent(Lb, cap, j);
          lo = (uint32_t)*ent(Llo, cap, j);
          sz = (uint32_t)*ent(Lsz, cap, j);
        }
        const uint32_t incl = wave_incl_scan_u32(sz);
        const uint32_t total = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
        if (wid == 0 && lane() == 0) atomicAdd(&sh.wV, (unsigned long long)total);
        for (uint32_t e0 = wid * kWave; e0 < total; e0 += nwav * kWave) {
          const uint32_t e = e0 + lane();
          const bool valid = e < total;
          const uint32_t ee = valid ? e : total - 1;
          uint32_t o = 0;  // owner lane: the first with incl > ee
#pragma unroll
          for (uint32_t step = 32; step >= 1; step >>= 1) {
            const uint32_t probe = (uint32_t)__shfl((int)incl, (int)(o + step - 1), kWave);
            if (probe <= ee) o += step;
          }
          const int32_t ob_ = __shfl(b, (int)o, kWave);
          const uint32_t olo = (uint32_t)__shfl((int)lo, (int)o, kWave);
          const uint32_t oin = (uint32_t)__shfl((int)incl, (int)o, kWave);
          const uint32_t osz = (uint32_t)__shfl((int)sz, (int)o, kWave);
          int32_t s = 0;
          bool sp = false;
          if (valid) {
            s = g.perm[olo + (ee - (oin - osz))];
            sp = !test_bit(tb, (uint32_t)s);
          }
          int32_t r = 0;
          if (sp) {
            atomicMax((unsigned long long*)&nlb[ob_],
                      (unsigned long long)(epoch | (uint64_t)(kNone - (uint32_t)s)));
            r = atomicAdd(&g.cnt[ob_], 1);
            atomicOr((unsigned long long*)&sf[s >> 6], 1ull << (s & 63));
          }
          const uint32_t si = push_idx(&sh.nS[par], sp);
          if (sp) {
            *ent(Ss, cap, si) = s;
            *ent(Sb, cap, si) = ob_;
            *ent(Sr, cap, si) = r;
          }
        }
      }
    }
    __syncthreads();
    const uint32_t nS = sh.nS[par], nT = sh.nT[par];
    if (tid == 0) {
      sT += nT;
      sS += nS;
      sL += sh.nL[par];
    }
    if (nS == 0) {  // workgroup-uniform
      // nothing split (most iterations): clear the touched states' marks and
      // flags and the candidate slot of iteration it + 2, behind one barrier
      // instead of the two of the split phases
      for (uint32_t i = tid; i < nT; i += nthr) {
        const int32_t s = *ent(Ts, cap, i);
        mw[s] = 0;
        tb[s >> 6] = 0;
      }
      if (tid == 0) sh.cand[par] = kNone;
      __syncthreads();
      if (sh.bad) {  // workgroup-uniform
        if (tid == 0) atomicOr(&a.ctl[1], 2u);
        break;
      }
      continue;
    }
    // The split phases take kCU entries per thread and step; each stage issues
    // the loads (or atomics) of all of them before using any, so a step waits
    // for one memory latency per stage, not kCU.
    // ---- C1: relabel each split state (its block's winning bid); the split
    // part goes to the tail [ne, be) of the block's range: index the split
    // states in front of ne, and record each staying state found in the tail
    // (the state at ne + the split state's rank) under its index; clear the
    // touched states' marks
    for (uint32_t i0 = tid; i0 < nS; i0 += nthr * kCU) {
      int32_t sv[kCU], bv[kCU], rv[kCU], ev[kCU], cv[kCU], pv[kCU], uv[kCU], fv[kCU], gv[kCU];
      uint64_t nv[kCU];
#pragma unroll
      for (uint32_t u = 0; u < kCU; ++u) {
        const uint32_t i = i0 + u * nthr;
        const bool ok = i < nS;
        sv[u] = ok ? *ent(Ss, cap, i) : -1;
        bv[u] = ok ? *ent(Sb, cap, i) : 0;
        rv[u] = ok ? *ent(Sr, cap, i) : 0;
      }
#pragma unroll
      for (uint32_t u = 0; u < kCU; ++u) {
        nv[u] = sv[u] >= 0 ? nlb[bv[u]] : 0ull;
        ev[u] = sv[u] >= 0 ? g.be[bv[u]] : 0;
        gv[u] = sv[u] >= 0 ? g.bs[bv[u]] : 0;
        cv[u] = sv[u] >= 0 ? g.cnt[bv[u]] : 0;
        pv[u] = sv[u] >= 0 ? g.pos[sv[u]] : 0;
      }
#pragma unroll
      for (uint32_t u = 0; u < kCU; ++u) {
        uv[u] = -1;
        fv[u] = -1;
        if (sv[u] < 0) continue;
        const int32_t e = ev[u], ne = e - cv[u], q = ne + rv[u];
        blk[sv[u]] = (int32_t)(kNone - (uint32_t)nv[u]);
        if (ne < 0 || q < ne || q >= e || e > (int32_t)n || pv[u] < 0 || pv[u] >= (int32_t)n) {
          sh.bad = 1;  // never expected: the entry is recorded as doing nothing
          uv[u] = -2;
          continue;
        }
        if (pv[u] < ne) fv[u] = atomicAdd(&g.fc[bv[u]], 1);
        uv[u] = g.perm[q];  // every tail position is examined once
      }
#pragma unroll
      for (uint32_t u = 0; u < kCU; ++u) {
        if (sv[u] < 0) continue;
        const uint32_t i = i0 + u * nthr;
        const int32_t e = ev[u], ne = e - cv[u];
        const int32_t nl = (int32_t)(kNone - (uint32_t)nv[u]);
        const bool ok = uv[u] != -2;
        *ent(Sf, cap, i) = ok ? fv[u] : -1;
        *ent(Sn, cap, i) = ok ? ne : 0;
        *ent(Sp, cap, i) = ok ? pv[u] : 0;
        *ent(Se, cap, i) = (ok && nl == sv[u]) ? e : -1;
        *ent(Sg, cap, i) = gv[u];
        if (uv[u] < 0 || uv[u] >= (int32_t)n) {
          sh.bad = 1;
          continue;
        }
        if (test_bit(sf, (uint32_t)uv[u])) continue;
        const int32_t j = atomicAdd(&g.gc[bv[u]], 1);
        if (ne + j < e)
          g.tmp64[ne + j] = ((uint64_t)(uint32_t)uv[u] << 32) | (uint32_t)(ne + rv[u]);
        else
          sh.bad = 1;
      }
    }
    for (uint32_t i = tid; i < nT; i += nthr) {
      const int32_t s = *ent(Ts, cap, i);
      mw[s] = 0;
      tb[s >> 6] = 0;
    }
    __syncthreads();
    if (sh.bad) {  // workgroup-uniform
      if (tid == 0) atomicOr(&a.ctl[1], 2u);
      break;
    }
    // ---- C2: swap the i-th front split state with the i-th tail staying
    // state; the new leader of each split block sets both ranges; unstable
    // updates (be, bs, cnt, fc, gc of a block are read by no other thread here)
    {
      uint32_t best = kNone;
      for (uint32_t i0 = tid; i0 < nS; i0 += nthr * kCU) {
        int32_t sv[kCU], bv[kCU], fv[kCU], nev[kCU], psv[kCU], ev[kCU], gv[kCU];
        uint64_t xv[kCU];
#pragma unroll
        for (uint32_t u = 0; u < kCU; ++u) {
          const uint32_t i = i0 + u * nthr;
          const bool ok = i < nS;
          sv[u] = ok ? *ent(Ss, cap, i) : -1;
          bv[u] = ok ? *ent(Sb, cap, i) : 0;
          fv[u] = ok ? *ent(Sf, cap, i) : -1;
          nev[u] = ok ? *ent(Sn, cap, i) : 0;
          psv[u] = ok ? *ent(Sp, cap, i) : 0;
          ev[u] = ok ? *ent(Se, cap, i) : -1;
          gv[u] = ok ? *ent(Sg, cap, i) : 0;
        }
#pragma unroll
        for (uint32_t u = 0; u < kCU; ++u) {
          if (fv[u] >= 0 && (nev[u] < 0 || nev[u] + fv[u] >= (int32_t)n)) {  // never expected
            sh.bad = 1;
            fv[u] = -1;
          }
          xv[u] = (sv[u] >= 0 && fv[u] >= 0) ? g.tmp64[nev[u] + fv[u]] : 0ull;
        }
        // the in-transition ranges by position travel with the swapped states
        uint64_t pq[kCU], pp[kCU];
#pragma unroll
        for (uint32_t u = 0; u < kCU; ++u) {
          const int32_t q = (int32_t)(uint32_t)xv[u];
          const bool sw = sv[u] >= 0 && fv[u] >= 0 && q >= nev[u] && q < (int32_t)n &&
                          psv[u] >= 0 && psv[u] < nev[u];
          pq[u] = sw ? g.pin[q] : 0ull;
          pp[u] = sw ? g.pin[psv[u]] : 0ull;
        }
#pragma unroll
        for (uint32_t u = 0; u < kCU; ++u) {
          if (sv[u] < 0) continue;
          const int32_t s = sv[u], b = bv[u], ne = nev[u];
          if (fv[u] >= 0) {
            const int32_t q = (int32_t)(uint32_t)xv[u], su = (int32_t)(xv[u] >> 32);
            const int32_t ps = psv[u];
            if (q < ne || q >= (int32_t)n || ps < 0 || ps >= ne || su < 0 || su >= (int32_t)n) {
              sh.bad = 1;  // never expected
            } else {
              g.perm[ps] = su;
              g.pos[su] = ps;
              g.pin[ps] = pq[u];
              g.perm[q] = s;
              g.pos[s] = q;
              g.pin[q] = pp[u];
            }
          }
          if (ev[u] >= 0) {  // the new leader: one thread per split block
            g.bs[s] = ne;
            g.be[s] = ev[u];
            g.be[b] = ne;
            g.cnt[b] = 0;
            g.fc[b] = 0;
            g.gc[b] = 0;
            if (ev[u] - ne > 1) atomicOr((unsigned long long*)&ml[s >> 6], 1ull << (s & 63));
            if (ne - gv[u] == 1) atomicAnd((unsigned long long*)&ml[b >> 6], ~(1ull << (b & 63)));
            wg_unstable_set(ub, us, (uint32_t)b);
            wg_unstable_set(ub, us, (uint32_t)s);
            best = min(best, (uint32_t)b);
            atomicAdd(&sh.wB, 1ull);
          }
          atomicAnd((unsigned long long*)&sf[s >> 6], ~(1ull << (s & 63)));
        }
      }
      wg_min(&sh.cand[par ^ 1], best);
      if (tid == 0) {
        if (nS > 0) {
          wg_unstable_set(ub, us, C);
          atomicMin(&sh.cand[par ^ 1], C);
          if (pf_on) pf[(par ^ 1) * kPfWords + 3] = 0;  // ranges changed: the prefetch is stale
        }
        sh.cand[par] = kNone;
      }
    }
    __syncthreads();
    if (sh.bad) {  // workgroup-uniform
      if (tid == 0) atomicOr(&a.ctl[1], 2u);
      break;
    }
  }
  if (tid == 0) {
    unsigned long long* w = a.work + 8;
    atomicAdd(&w[0], (unsigned long long)(it + 1));
    atomicAdd(&w[1], (unsigned long long)sM);
    atomicAdd(&w[2], sh.wE);
    atomicAdd(&w[3], (unsigned long long)sT);
    atomicAdd(&w[4], (unsigned long long)sL);
    atomicAdd(&w[5], sh.wV);
    atomicAdd(&w[6], (unsigned long long)sS);
    atomicAdd(&w[7], sh.wB);
  }
  for (uint32_t s = tid; s < n; s += nthr) a.out[s0 + s] = blk[s];
  return it + 1;
}

// Built for 256-thread workgroups only, with that launch bound, so that the
// register budget (up to 512 per lane) holds the whole kernel and nothing
// spills to scratch.  Larger workgroups are not built: builds of this tier
// for 512 and 1024 threads, which kept 128 registers and spilled 212-332
// bytes per lane, made illegal memory accesses on the GPU for reasons not
// found (builds spilling at most 160 bytes passed every test).
template <class MaskT, int WG>
__global__ void __launch_bounds__(WG) k_batch(BArgs a) {
  extern __shared__ uint64_t lds[];
  __shared__ Shared sh;
  for (;;) {
    if (threadIdx.x == 0) sh.job = atomicAdd(&a.ctl[0], 1u);
    __syncthreads();
    const uint32_t job = sh.job;
    if (job >= (uint32_t)a.count) break;
    const int32_t k = a.order[job];
    const uint32_t s0 = a.n_off[k], n = a.n_off[k + 1] - s0;
    int32_t* T = a.tl + s0;
    int32_t* S = a.sl + s0;
    uint32_t its;
    if (lds_need<MaskT>(n) <= a.lds_bytes) {
      const uint32_t nw = (n + 63u) >> 6;
      WArr<MaskT> w;
      w.ub = lds;
      w.tb = lds + nw;
      w.lt = lds + 2 * nw;
      w.nlb = lds + 3 * nw;
      w.mw = reinterpret_cast<MaskT*>(lds + 3 * nw + n);
      w.blk = reinterpret_cast<int32_t*>(lds + 3 * nw + n + (sizeof(MaskT) * n + 7) / 8);
      its = wg_refine<MaskT, 1>(a, sh, w, T, S, s0, n);
    } else {
      const uint32_t b0 = a.bw_off[k];
      GList g;
      g.perm = a.perm + s0;
      g.pos = a.pos + s0;
      g.bs = a.bs + s0;
      g.be = a.be + s0;
      g.cnt = a.cnt + s0;
      g.fc = a.fc + s0;
      g.gc = a.gc + s0;
      g.tmp64 = a.tmp64 + s0;
      g.pin = a.pin + s0;
      g.ts = T;
      g.tb_ = a.tlb + s0;
      g.lb = a.ltl + s0;
      g.llo = a.llo + s0;
      g.lsz = a.lsz + s0;
      g.sgs = a.sgs + s0;
      g.ss = S;
      g.sb_ = a.ob + s0;
      g.sr = a.rk + s0;
      g.sf_ = a.fi + s0;
      g.sn = a.nev + s0;
      g.sp = a.tmp + s0;
      g.se = a.se + s0;
      g.sf = a.sf + b0;
      g.ml = a.lt + b0;
      g.us = a.us + b0;
      its = wg_refine_lists<MaskT>(a, sh, a.blk + s0, reinterpret_cast<MaskT*>(a.mw) + s0,
                                   a.nlb + s0, g, lds, a.lds_bytes, a.ub + b0, a.tb + b0, s0, n);
    }
    if (threadIdx.x == 0) a.iters[k] = its;
    __syncthreads();
  }
}

__global__ void k_reset_queue(uint32_t* ctl, unsigned long long* work) {
  if (blockIdx.x == 0 && threadIdx.x < 16) work[threadIdx.x] = 0;
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl[0] = 0;
    ctl[1] = 0;
  }
}

// shift instance-local ids into the union's id space, validating ranges
__device__ __forceinline__ int32_t find_instance(const uint32_t* off, int32_t count, uint64_t x) {
  int32_t lo = 0, hi = count;  // off[lo] <= x < off[hi]
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if ((uint64_t)off[mid] <= x) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ void k_globalize(int32_t count, const uint32_t* __restrict__ n_off,
                            const uint32_t* __restrict__ m_off, const int32_t* __restrict__ K,
                            const int32_t* __restrict__ src, const int32_t* __restrict__ lab,
                            const int32_t* __restrict__ dst, const int32_t* __restrict__ init,
                            uint64_t M, uint64_t N, int32_t* __restrict__ gsrc,
                            int32_t* __restrict__ gdst, int32_t* __restrict__ ginit,
                            uint32_t* err) {
  bool bad = false;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M; i += stride) {
    const int32_t k = find_instance(m_off, count, i);
    const uint32_t nk = n_off[k + 1] - n_off[k];
    const int32_t s = src[i], d = dst[i], l = lab[i];
    bad |= (uint32_t)s >= nk || (uint32_t)d >= nk || (uint32_t)l >= (uint32_t)K[k];
    gsrc[i] = (int32_t)n_off[k] + ((uint32_t)s < nk ? s : 0);
    gdst[i] = (int32_t)n_off[k] + ((uint32_t)d < nk ? d : 0);
  }
  for (uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; s < N; s += stride) {
    const int32_t k = find_instance(n_off, count, s);
    const uint32_t nk = n_off[k + 1] - n_off[k];
    int32_t v = 0;
    if (init) {
      v = init[s];
      bad |= (uint32_t)v >= nk;
      if ((uint32_t)v >= nk) v = 0;
    }
    ginit[s] = (int32_t)n_off[k] + v;
  }
  if (bad) atomicOr(err, 1u);
}

template <class T>
bisim_status dmalloc(T** p, size_t count) {
  *p = nullptr;
  hipError_t e = hipMalloc((void**)p, sizeof(T) * (count ? count : 1));
  if (e != hipSuccess) {
    set_error("device allocation of %zu bytes failed: %s", sizeof(T) * count, hipGetErrorString(e));
    return BISIM_E_NOMEM;
  }
  return BISIM_OK;
}

void free_batch(bisim_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  void* ptrs[] = {b->n_off_d, b->bw_off_d, b->order_d, b->blk, b->mw,      b->nlb,  b->ub,
                  b->tb,      b->lt,       b->tl,      b->sl,  b->iters_d, b->ctl_d, b->perm,
                  b->pos,     b->bs,       b->be,      b->cnt, b->fc,      b->gc,    b->tmp,
                  b->rk,      b->fi,       b->ltl,     b->sf,  b->us,      b->ob,    b->nev,
                  b->tlb,     b->se,       b->tmp64,   b->sgs,    b->work_d, b->llo, b->lsz,
                  b->pin};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (b->u) lts_destroy(b->u);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  if (b->own_stream) (void)hipStreamDestroy(b->own_stream);
  delete b;
}

BArgs make_args(bisim_batch* b, int32_t* out) {
  BArgs a{};
  a.count = b->count;
  a.n_off = b->n_off_d;
  a.bw_off = b->bw_off_d;
  a.order = b->order_d;
  a.pre_block = b->u->pre_block;
  a.in_ptr = b->u->in_ptr;
  a.in_src = b->u->in_src;
  a.in_ord = b->u->in_ord;
  a.blk = b->blk;
  a.mw = b->mw;
  a.nlb = b->nlb;
  a.ub = b->ub;
  a.tb = b->tb;
  a.lt = b->lt;
  a.tl = b->tl;
  a.sl = b->sl;
  a.perm = b->perm;
  a.pos = b->pos;
  a.bs = b->bs;
  a.be = b->be;
  a.cnt = b->cnt;
  a.fc = b->fc;
  a.gc = b->gc;
  a.tmp = b->tmp;
  a.rk = b->rk;
  a.fi = b->fi;
  a.ob = b->ob;
  a.nev = b->nev;
  a.ltl = b->ltl;
  a.tlb = b->tlb;
  a.se = b->se;
  a.sgs = b->sgs;
  a.llo = b->llo;
  a.lsz = b->lsz;
  a.tmp64 = b->tmp64;
  a.pin = b->pin;
  a.sf = b->sf;
  a.us = b->us;
  a.out = out;
  a.iters = b->iters_d;
  a.ctl = b->ctl_d;
  a.work = b->work_d;
  a.lds_bytes = (uint32_t)b->lds_bytes;
  return a;
}

// allow dynamic LDS up to the device's per-workgroup maximum
void allow_lds(bisim_batch* b) {
  const void* fns[] = {(const void*)k_batch<uint64_t, kBatchWG>,
                       (const void*)k_batch<uint32_t, kBatchWG>};
  for (const void* f : fns)
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, b->lds_max);
  (void)hipGetLastError();
}

bisim_status launch_once(bisim_batch* b, int32_t* out, int wg, int grid, int lds) {
  BArgs a = make_args(b, out);
  a.lds_bytes = (uint32_t)lds;
  hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, b->stream, b->ctl_d, b->work_d);
  if (wg != kBatchWG) {
    set_error("batched kernel: workgroup size %d is not built (%d)", wg, kBatchWG);
    return BISIM_E_INVALID;
  }
  if (b->mask64)
    hipLaunchKernelGGL((k_batch<uint64_t, kBatchWG>), dim3(grid), dim3(wg), lds, b->stream, a);
  else
    hipLaunchKernelGGL((k_batch<uint32_t, kBatchWG>), dim3(grid), dim3(wg), lds, b->stream, a);
  BISIM_TRY_HIP(hipGetLastError());
  return BISIM_OK;
}

int max_resident(bisim_batch* b, int wg, int lds) {
  int per_cu = 0;
  if (wg != kBatchWG) return 0;
  const void* f = b->mask64 ? (const void*)k_batch<uint64_t, kBatchWG>
                            : (const void*)k_batch<uint32_t, kBatchWG>;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, wg, lds);
  if (e != hipSuccess || per_cu < 1) return 0;
  return per_cu * b->num_cu;
}

std::string tune_key(bisim_batch* b) {
  hipDeviceProp_t p;
  std::string arch = "gpu";
  if (hipGetDeviceProperties(&p, b->device) == hipSuccess) arch = p.gcnArchName;
  for (char& c : arch)
    if (c == ' ' || c == ':') c = '_';
  int lc = 0, ln = 0, lm = 0;
  for (int64_t v = b->count; v > 1; v >>= 1) ++lc;
  for (int64_t v = b->N; v > 1; v >>= 1) ++ln;
  for (int64_t v = b->M; v > 1; v >>= 1) ++lm;
  char buf[256];
  snprintf(buf, sizeof buf, "%s_cu%d_c%d_n%d_m%d_k%d", arch.c_str(), b->num_cu, lc, ln, lm,
           b->mask64);
  return buf;
}

std::string tune_path() {
  const char* e = getenv("BISIM_TUNE_CACHE");
  if (e && *e) return e;
  const char* h = getenv("HOME");
  return std::string(h && *h ? h : "/tmp") + "/.cache/bisim_tune.txt";
}

bool tune_lookup(const std::string& key, int* wg, int* grid, int* lds) {
  FILE* f = fopen(tune_path().c_str(), "r");
  if (!f) return false;
  char k[256];
  int a, g, l;
  float ms;
  bool found = false;
  while (fscanf(f, "%255s %d %d %d %f", k, &a, &g, &l, &ms) == 5)
    if (key == k) {
      *wg = a;
      *grid = g;
      *lds = l;
      found = true;
    }
  fclose(f);
  return found;
}

void tune_store(const std::string& key, int wg, int grid, int lds, float ms) {
  std::string path = tune_path();
  std::string dir = path.substr(0, path.find_last_of('/'));
  if (!dir.empty()) {
    for (size_t i = 1; i <= dir.size(); ++i)
      if (i == dir.size() || dir[i] == '/') (void)mkdir(dir.substr(0, i).c_str(), 0755);
  }
  FILE* f = fopen(path.c_str(), "a");
  if (!f) return;
  fprintf(f, "%s %d %d %d %.4f\n", key.c_str(), wg, grid, lds, ms);
  fclose(f);
}

// Autotuner: time each candidate (workgroup size, LDS budget, grid = as many
// workgroups as stay resident) on the batch itself and keep the fastest.
bisim_status autotune(bisim_batch* b, int32_t* out) {
  const int wgs[] = {kBatchWG};
  std::vector<int> budgets;
  for (int l = b->lds_max; l >= 16384 && budgets.size() < 4; l /= 2) budgets.push_back(l);
  float best = 1e30f;
  int bw = 0, bg = 0, bl = 0;
  for (int wg : wgs) {
    for (int lds : budgets) {
      const int grid = max_resident(b, wg, lds);
      if (grid < 1) continue;
      BISIM_TRY_HIP(hipEventRecord(b->ev0, b->stream));
      BISIM_TRY(launch_once(b, out, wg, grid, lds));
      BISIM_TRY_HIP(hipEventRecord(b->ev1, b->stream));
      BISIM_TRY_HIP(hipEventSynchronize(b->ev1));
      float ms = 0;
      BISIM_TRY_HIP(hipEventElapsedTime(&ms, b->ev0, b->ev1));
      if (ms < best) {
        best = ms;
        bw = wg;
        bg = grid;
        bl = lds;
      }
    }
  }
  if (!bw) {
    set_error("batched kernel: no launch configuration is resident");
    return BISIM_E_DEVICE;
  }
  b->wg = bw;
  b->grid = bg;
  b->lds_bytes = bl;
  tune_store(tune_key(b), bw, bg, bl, best);
  return BISIM_OK;
}
}  // namespace
}  // namespace bisim

using namespace bisim;

extern "C" {

bisim_status lts_batch_load(int32_t count, const int64_t* n_off, const int64_t* m_off,
                            const int32_t* src, const int32_t* label, const int32_t* dst,
                            const int32_t* num_actions, const int32_t* init_partition,
                            void* hip_stream, bisim_batch** out) {
  if (!out) {
    set_error("lts_batch_load: out is NULL");
    return BISIM_E_INVALID;
  }
  *out = nullptr;
  if (count < 1 || !n_off || !m_off || !num_actions) {
    set_error("lts_batch_load: need count >= 1 and host offset/action arrays");
    return BISIM_E_INVALID;
  }
  if (n_off[0] != 0 || m_off[0] != 0) {
    set_error("lts_batch_load: offsets must start at 0");
    return BISIM_E_INVALID;
  }
  int32_t Kmax = 1;
  for (int32_t k = 0; k < count; ++k) {
    if (n_off[k + 1] < n_off[k] || m_off[k + 1] < m_off[k] || num_actions[k] < 1) {
      set_error("lts_batch_load: offsets must be non-decreasing and num_actions >= 1");
      return BISIM_E_INVALID;
    }
    Kmax = std::max(Kmax, num_actions[k]);
  }
  const int64_t N = n_off[count], M = m_off[count];
  if (N >= 0x7FFFFFFF || M >= 0xFFFFFFFFll) {
    set_error("lts_batch_load: totals beyond 2^31-1 states / 2^32-1 transitions");
    return BISIM_E_UNSUPPORTED;
  }
  if (M > 0 && (!src || !label || !dst)) {
    set_error("lts_batch_load: NULL transition array");
    return BISIM_E_INVALID;
  }
  bisim_batch* b = new (std::nothrow) bisim_batch;
  if (!b) return BISIM_E_NOMEM;
  b->count = count;
  b->N = N;
  b->M = M;
  b->Kmax = Kmax;
  b->n_off.assign(n_off, n_off + count + 1);
  bisim_status st = BISIM_OK;
  int32_t *gsrc = nullptr, *gdst = nullptr, *ginit = nullptr, *Kd = nullptr;
  uint32_t *m_off_d = nullptr, *err = nullptr;
  do {
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess)
      e = hipDeviceGetAttribute(&b->num_cu, hipDeviceAttributeMultiprocessorCount, b->device);
    if (e == hipSuccess)
      e = hipDeviceGetAttribute(&b->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device);
    if (e == hipSuccess) e = hipEventCreate(&b->ev0);
    if (e == hipSuccess) e = hipEventCreate(&b->ev1);
    if (e == hipSuccess && !hip_stream) e = hipStreamCreateWithFlags(&b->own_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      set_error("lts_batch_load: %s", hipGetErrorString(e));
      st = BISIM_E_DEVICE;
      break;
    }
    b->lds_max -= (int)sizeof(Shared) + 64;
    allow_lds(b);
    b->stream = hip_stream ? (hipStream_t)hip_stream : b->own_stream;
    hipStream_t s = b->stream;
    if (hipEventRecord(b->ev0, s) != hipSuccess) { st = BISIM_E_DEVICE; break; }
    std::vector<uint32_t> no(count + 1), mo(count + 1), bo(count + 1);
    bo[0] = 0;
    for (int32_t k = 0; k <= count; ++k) {
      no[k] = (uint32_t)n_off[k];
      mo[k] = (uint32_t)m_off[k];
      if (k < count) bo[k + 1] = bo[k] + (uint32_t)((n_off[k + 1] - n_off[k] + 63) / 64);
    }
    std::vector<int32_t> order(count);
    for (int32_t k = 0; k < count; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
      return n_off[x + 1] - n_off[x] > n_off[y + 1] - n_off[y];
    });
    if ((st = dmalloc(&b->n_off_d, count + 1)) || (st = dmalloc(&b->bw_off_d, count + 1)) ||
        (st = dmalloc(&b->order_d, count)) || (st = dmalloc(&m_off_d, count + 1)) ||
        (st = dmalloc(&Kd, count)) || (st = dmalloc(&err, 1)) ||
        (st = dmalloc(&gsrc, (size_t)M)) || (st = dmalloc(&gdst, (size_t)M)) ||
        (st = dmalloc(&ginit, (size_t)N)))
      break;
    e = hipMemcpyAsync(b->n_off_d, no.data(), 4 * (count + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(m_off_d, mo.data(), 4 * (count + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->bw_off_d, bo.data(), 4 * (count + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(b->order_d, order.data(), 4 * count, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(Kd, num_actions, 4 * count, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(err, 0, 4, s);
    if (e != hipSuccess) {
      set_error("lts_batch_load: %s", hipGetErrorString(e));
      st = BISIM_E_DEVICE;
      break;
    }
    int64_t g = (std::max(N, M) + kT - 1) / kT;
    g = std::min<int64_t>(std::max<int64_t>(g, 1), (int64_t)b->num_cu * 16);
    hipLaunchKernelGGL(k_globalize, dim3((unsigned)g), dim3(kT), 0, s, count, b->n_off_d, m_off_d,
                       Kd, src, label, dst, init_partition, (uint64_t)M, (uint64_t)N, gsrc, gdst,
                       ginit, err);
    uint32_t err_h = 0;
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&err_h, err, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      set_error("lts_batch_load: %s", hipGetErrorString(e));
      st = BISIM_E_DEVICE;
      break;
    }
    if (err_h) {
      set_error("lts_batch_load: an instance-local id, label or init value is out of range");
      st = BISIM_E_RANGE;
      break;
    }
    st = lts_create_union((int32_t)N, M, Kmax, gsrc, label, gdst, ginit, s, &b->u);
    if (st != BISIM_OK) break;
    if (!b->u->uniform) {
      set_error("lts_batch_load: a state has more than 64 distinct outgoing actions");
      st = BISIM_E_UNSUPPORTED;
      break;
    }
    // 32-bit mark words suffice when no state has more than 32 actions
    b->mask64 = Kmax > 32;
    const size_t BW = bo[count];
    if ((st = dmalloc(&b->blk, (size_t)N)) || (st = dmalloc(&b->mw, (size_t)N)) ||
        (st = dmalloc(&b->nlb, (size_t)N)) || (st = dmalloc(&b->ub, BW)) ||
        (st = dmalloc(&b->tb, BW)) || (st = dmalloc(&b->lt, BW)) ||
        (st = dmalloc(&b->tl, (size_t)N)) || (st = dmalloc(&b->sl, (size_t)N)) ||
        (st = dmalloc(&b->perm, (size_t)N)) || (st = dmalloc(&b->pos, (size_t)N)) ||
        (st = dmalloc(&b->bs, (size_t)N)) || (st = dmalloc(&b->be, (size_t)N)) ||
        (st = dmalloc(&b->cnt, (size_t)N)) || (st = dmalloc(&b->fc, (size_t)N)) ||
        (st = dmalloc(&b->gc, (size_t)N)) || (st = dmalloc(&b->tmp, (size_t)N)) ||
        (st = dmalloc(&b->rk, (size_t)N)) || (st = dmalloc(&b->fi, (size_t)N)) ||
        (st = dmalloc(&b->ltl, (size_t)N)) || (st = dmalloc(&b->sf, BW)) ||
        (st = dmalloc(&b->ob, (size_t)N)) || (st = dmalloc(&b->nev, (size_t)N)) ||
        (st = dmalloc(&b->us, BW)) || (st = dmalloc(&b->tlb, (size_t)N)) ||
        (st = dmalloc(&b->se, (size_t)N)) || (st = dmalloc(&b->tmp64, (size_t)N)) ||
        (st = dmalloc(&b->pin, (size_t)N)) ||
        (st = dmalloc(&b->sgs, (size_t)N)) || (st = dmalloc(&b->llo, (size_t)N)) ||
        (st = dmalloc(&b->lsz, (size_t)N)) ||
        (st = dmalloc(&b->iters_d, count)) || (st = dmalloc(&b->ctl_d, 2)) ||
        (st = dmalloc(&b->work_d, 16)))
      break;
    float ms = 0;
    if (hipEventRecord(b->ev1, s) != hipSuccess || hipEventSynchronize(b->ev1) != hipSuccess ||
        hipEventElapsedTime(&ms, b->ev0, b->ev1) != hipSuccess) {
      st = BISIM_E_DEVICE;
      break;
    }
    b->t_pre_ms = ms;
  } while (0);
  if (gsrc) (void)hipFree(gsrc);
  if (gdst) (void)hipFree(gdst);
  if (ginit) (void)hipFree(ginit);
  if (Kd) (void)hipFree(Kd);
  if (m_off_d) (void)hipFree(m_off_d);
  if (err) (void)hipFree(err);
  if (st != BISIM_OK) {
    free_batch(b);
    return st;
  }
  *out = b;
  return BISIM_OK;
}

bisim_status coarsest_partition_batch(bisim_batch* b, int32_t* block_id, int64_t* iterations,
                                      bisim_batch_stats* st) {
  if (!b || (!block_id && b->N > 0)) {
    set_error("coarsest_partition_batch: NULL handle or output");
    return BISIM_E_INVALID;
  }
  // configuration: explicit options, else the cached or freshly tuned choice
  if (!b->tuned || b->opt_retune) {
    int wg = 0, grid = 0, lds = 0;
    const bool fixed = b->opt_wg || b->opt_grid || b->opt_lds;
    if (fixed) {
      wg = b->opt_wg ? b->opt_wg : kBatchWG;
      lds = b->opt_lds ? std::min(b->opt_lds, b->lds_max) : b->lds_max;
      grid = b->opt_grid ? b->opt_grid : max_resident(b, wg, lds);
      b->wg = wg;
      b->grid = grid;
      b->lds_bytes = lds;
    } else if (!b->opt_retune && tune_lookup(tune_key(b), &wg, &grid, &lds) && wg && grid &&
               lds <= b->lds_max && max_resident(b, wg, lds) >= grid) {
      b->wg = wg;
      b->grid = grid;
      b->lds_bytes = lds;
    } else {
      BISIM_TRY(autotune(b, block_id));
    }
    if (b->grid < 1) {
      set_error("coarsest_partition_batch: configuration not resident");
      return BISIM_E_DEVICE;
    }
    b->tuned = true;
    b->opt_retune = 0;
  }
  // graph of (queue reset, batched kernel); the configuration and the output
  // pointer are baked into it, so it is re-captured when either changes
  const bool need_graph = !b->gexec || b->g_wg != b->wg || b->g_grid != b->grid ||
                          b->g_lds != b->lds_bytes || b->g_out != block_id;
  if (need_graph) {
    if (b->gexec) {
      (void)hipGraphExecDestroy(b->gexec);
      b->gexec = nullptr;
    }
    hipGraph_t graph = nullptr;
    BISIM_TRY_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    bisim_status ls = launch_once(b, block_id, b->wg, b->grid, b->lds_bytes);
    hipError_t ec = hipStreamEndCapture(b->stream, &graph);
    if (ls != BISIM_OK) return ls;
    BISIM_TRY_HIP(ec);
    hipError_t ei = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    BISIM_TRY_HIP(ei);
    b->g_wg = b->wg;
    b->g_grid = b->grid;
    b->g_lds = b->lds_bytes;
    b->g_out = block_id;
  }
  BISIM_TRY_HIP(hipEventRecord(b->ev0, b->stream));
  BISIM_TRY_HIP(hipGraphLaunch(b->gexec, b->stream));
  BISIM_TRY_HIP(hipEventRecord(b->ev1, b->stream));
  std::vector<uint32_t> its(b->count);
  uint32_t ctl_h[2] = {0, 0};
  BISIM_TRY_HIP(hipMemcpyAsync(its.data(), b->iters_d, 4 * b->count, hipMemcpyDeviceToHost, b->stream));
  BISIM_TRY_HIP(hipMemcpyAsync(ctl_h, b->ctl_d, 8, hipMemcpyDeviceToHost, b->stream));
  unsigned long long work_h[16];
  BISIM_TRY_HIP(hipMemcpyAsync(work_h, b->work_d, sizeof(work_h), hipMemcpyDeviceToHost,
                               b->stream));
  BISIM_TRY_HIP(hipStreamSynchronize(b->stream));
  float ms = 0;
  BISIM_TRY_HIP(hipEventElapsedTime(&ms, b->ev0, b->ev1));
  b->t_alg_ms = ms;
  if (ctl_h[1] & 2u) {
    set_error("coarsest_partition_batch: inconsistent block ranges in the member-list tier");
    return BISIM_E_DEVICE;
  }
  if (ctl_h[1]) {
    set_error("coarsest_partition_batch: an instance exceeded its iteration cap");
    return BISIM_E_ITERCAP;
  }
  int64_t mx = 0, sum = 0, nl = 0, ng = 0;
  for (int32_t k = 0; k < b->count; ++k) {
    mx = std::max<int64_t>(mx, its[k]);
    sum += its[k];
    if (iterations) iterations[k] = its[k];
    const uint32_t n = (uint32_t)(b->n_off[k + 1] - b->n_off[k]);
    const uint64_t need = b->mask64 ? lds_need<uint64_t>(n) : lds_need<uint32_t>(n);
    (need <= (uint64_t)b->lds_bytes ? nl : ng) += 1;
  }
  if (st) {
    st->max_iterations = mx;
    st->sum_iterations = sum;
    st->lds_instances = nl;
    st->global_instances = ng;
    st->workgroup_size = b->wg;
    st->grid = b->grid;
    st->t_pre_ms = b->t_pre_ms;
    st->t_alg_ms = b->t_alg_ms;
    for (int i = 0; i < 16; ++i) st->work[i / 8][i % 8] = (int64_t)work_h[i];
  }
  return BISIM_OK;
}

void lts_batch_free(bisim_batch* b) { free_batch(b); }

bisim_status bisim_batch_set_option(bisim_batch* b, int32_t option, int64_t value) {
  if (!b) {
    set_error("bisim_batch_set_option: NULL handle");
    return BISIM_E_INVALID;
  }
  switch (option) {
    case BISIM_BOPT_WG_SIZE:
      if (value != 0 && value != kBatchWG) break;
      b->opt_wg = (int)value;
      b->tuned = false;
      return BISIM_OK;
    case BISIM_BOPT_GRID:
      if (value < 0 || value > (1 << 20)) break;
      b->opt_grid = (int)value;
      b->tuned = false;
      return BISIM_OK;
    case BISIM_BOPT_LDS_LIMIT:
      if (value < 0 || value > (1 << 22)) break;
      b->opt_lds = (int)value;
      b->tuned = false;
      return BISIM_OK;
    case BISIM_BOPT_TUNE:
      if (value != 0 && value != 1) break;
      b->opt_retune = (int)value;
      return BISIM_OK;
    default:
      break;
  }
  set_error("bisim_batch_set_option: bad option %d or value %lld", option, (long long)value);
  return BISIM_E_INVALID;
}

}  // extern "C"
