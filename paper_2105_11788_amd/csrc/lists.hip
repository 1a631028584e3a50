// Engine 3: the plain refinement loop (Algorithm 3, section 4) over the
// whole grid with work proportional to the splitter and the states it
// touches, not to n.
//
// Besides block[], the partition is kept as a refinable partition: perm
// lists the states block by block and the block labelled b owns
// perm[bs[b] .. be[b]).  One iteration is three kernels:
//
//   M  mark      C = the candidate (the smallest unstable label, the
//                priority reading of the concurrent write); clear its
//                unstable bit and search the next set bit (one wave); visit
//                the in-transitions of C's members (perm[bs[C] .. be[C]))
//                and set their mark bits; the first touch of a state sets
//                its touched bit, counts it for its block and lists it with
//                its block, and a touched leader of a block with more than
//                one state appends the block's member segments to a list.
//   K  compare   listed touched states whose marks differ from their
//                leader's split; so do the untouched members of the listed
//                blocks (none when the block's count equals its size).  A
//                split state bids for its block's new leader (64-bit max of
//                (epoch, ~state): the smallest state wins), takes its rank
//                within the block's split part, sets its split bit and is
//                listed.  One wave prefetches the next splitter's range and
//                first members for the next mark kernel.
//   S  split     every split state takes its block's winning bid as label;
//                the split part will be the tail [ne, be) of the block's
//                range: split states in front of ne take an index, and the
//                staying state found at ne + rank is recorded under an index
//                of its own.  The last workgroup to finish that then swaps
//                the i-th front split state with the i-th staying tail
//                state; the new leader of each split block sets both ranges
//                and the unstable bits, and the old label joins the next
//                candidate (with C if anything split, the lock-step reading
//                of Algorithm 3).  Marks, touched bits and counts are
//                cleared.
//
// Every per-iteration set (touched states, listed segments, split states) is
// a list built with wave-aggregated atomics, so no kernel scans anything of
// size n.  Iterations are captured in a hipGraph of kGraphIters iterations
// (3 kernels each, plus one that advances the iteration base the kernels add
// their position in the graph to) and replayed until the done flag is set.
// The splitter sequence, the split counts and the partitions are those of
// the other engines.  States with more than 64 actions use the mark-word
// offsets of the preprocessing.
#include <hip/hip_ext.h>

#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

namespace bisim {
namespace {

constexpr int kLT = 256;
constexpr uint32_t kSeg = 1024;       // members of a listed block per segment
constexpr uint32_t kGraphIters = 32;  // iterations per captured graph
static_assert(kGraphIters % 2 == 0, "the iteration parity is the launch position's");
// the next splitter, prefetched: two slots by iteration parity, each a header
// (label, first position, size, valid) and the in-transition ranges (first
// edge << 32 | count) of its first kWave members
constexpr uint32_t kPfWords = 4u + 2u * kWave;
constexpr int kPhases = 3;  // kernels per iteration

struct LArgs {
  uint32_t n;
  int uniform;
  uint64_t nwd;  // words of a per-state bitmap
  const uint32_t* __restrict__ in_ptr;
  const int32_t* __restrict__ in_src;
  const int32_t* __restrict__ in_ord;
  const uint32_t* __restrict__ woff;
  int32_t* block;
  uint64_t* mw;
  uint64_t* tb;   // touched states
  uint64_t* sf;   // split states
  uint64_t* ub;   // unstable labels
  uint64_t* us;   // summary of ub
  uint64_t* nlw;  // bids
  int32_t *perm, *pos, *bs, *be, *cnt, *fc, *gc;
  int32_t* tcn;  // per label: members first touched this iteration (0 between iterations)
  uint64_t* pin;  // per position p: in-transition range of perm[p] (first edge << 32 | count)
  uint32_t* pf;   // [2][kPfWords] the next splitter, prefetched
  uint64_t* tmp64;
  int32_t *lb, *lo, *lh;  // listed segments: block, first and end position
  uint32_t lcap;
  uint32_t mpw;  // splitter members per wave and step of the mark kernel
  int32_t *ts, *tbk;  // touched states and their blocks
  int32_t *ss, *sbk, *sr, *sfi, *sne, *sps, *sse;  // split states (by list index)
  uint64_t* work;  // [8] totals when counting
  int count;
  Ctl* ctl;
  uint32_t iter_cap;
  int32_t* trace_C;
  int64_t* trace_nsplit;
  uint32_t trace_cap;
};

struct GPart {
  uint32_t gtid, gthreads, gwave, gwaves;
};
__device__ __forceinline__ GPart gpart() {
  const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t gthreads = gridDim.x * blockDim.x;
  return {gtid, gthreads, gtid / kWave, gthreads / kWave};
}

// iteration of a launch: the base advanced after every graph replay (0 for
// eager launches) plus the launch's position.  The base stays even, so the
// iteration's parity is the position's, known without waiting for the load.
__device__ __forceinline__ uint32_t iter_of(const LArgs& a, uint32_t kofs) {
  return a.ctl->state.v[6] + kofs;
}

// wave-aggregated reservation of one list entry per lane with pred; returns
// the entry index (kNone without pred).  Wave-uniform call.
__device__ __forceinline__ uint32_t reserve(uint32_t* counter, bool pred) {
  const uint64_t bal = __ballot(pred);
  if (!bal) return kNone;
  const int leader = __ffsll((unsigned long long)bal) - 1;
  uint32_t base = 0;
  if ((int)lane() == leader) base = atomicAdd(counter, (uint32_t)__popcll(bal));
  base = (uint32_t)__shfl((int)base, leader, kWave);
  return pred ? base + (uint32_t)__popcll(bal & ((1ull << lane()) - 1ull)) : kNone;
}

__device__ __forceinline__ void set_unstable(const LArgs& a, uint32_t b) {
  const uint32_t w = b >> 6;
  const uint64_t old = atomicOr((unsigned long long*)&a.ub[w], 1ull << (b & 63));
  if (old == 0) atomicOr((unsigned long long*)&a.us[w >> 6], 1ull << (w & 63));
}

__device__ __forceinline__ void count_work(const LArgs& a, uint32_t i, uint64_t v) {
  if (a.count && v && lane() == 0) atomicAdd((unsigned long long*)&a.work[i], (unsigned long long)v);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += (uint64_t)__shfl_xor((unsigned long long)v, d, kWave);
  return v;
}

// mark word of slot o of state s
__device__ __forceinline__ uint64_t* mword(const LArgs& a, int32_t s, int32_t o) {
  return a.uniform ? &a.mw[s] : &a.mw[a.woff[s] + ((uint32_t)o >> 6)];
}

// marks of s differ from those of b (same action set: same number of words)
__device__ __forceinline__ bool marks_differ(const LArgs& a, int32_t s, int32_t b) {
  if (a.uniform) return a.mw[s] != a.mw[b];
  const uint32_t w0 = a.woff[s], w1 = a.woff[s + 1], v0 = a.woff[b];
  for (uint32_t w = w0; w < w1; ++w)
    if (a.mw[w] != a.mw[v0 + (w - w0)]) return true;
  return false;
}

// ---------------------------------------------------------------------------
// M: select, mark
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kLT) k_l_mark(LArgs a, uint32_t kofs) {
  const uint32_t done = a.ctl->state.v[1];
  const uint32_t k = iter_of(a, kofs);
  const uint32_t par = kofs & 1;
  const uint32_t C0 = a.ctl->cand[par].v[0];
  // the prefetch slot of this iteration, and the in-transition range this
  // lane would take from it for the wave's first member chunk
  const uint32_t* pc = a.pf + par * kPfWords;
  const uint32_t pf_ok = pc[3], pf_C = pc[0], pf_cb = pc[1], pf_n = pc[2];
  const GPart p = gpart();
  const uint32_t i_first = p.gwave * a.mpw + lane();
  const bool lane_first = lane() < a.mpw && i_first < kWave;
  const uint32_t pf_lo = lane_first ? pc[4 + 2 * i_first] : 0u;
  const uint32_t pf_hi = lane_first ? pc[5 + 2 * i_first] : 0u;
  if (done) return;
  const bool over = k + 1 > a.iter_cap;
  if (C0 == kNone || over) {  // the final pass, or the iteration cap
    if (p.gtid == 0) {
      a.ctl->state.v[0] = k + 1;
      a.ctl->state.v[1] = 1;
      if (over && C0 != kNone) a.ctl->state.v[2] = 1;
      if (k < a.trace_cap) {
        if (a.trace_C) a.trace_C[k] = -1;
        if (a.trace_nsplit) a.trace_nsplit[k] = 0;
      }
    }
    return;
  }
  const uint32_t C = C0;
  if (p.gtid == 0) {
    a.ctl->state.v[3] = C;
    a.ctl->cntT[par ^ 1].v[0] = 0;  // counters of the next iteration
    a.ctl->cntS[par ^ 1].v[0] = 0;
    a.ctl->cntC[par ^ 1].v[0] = 0;
    if (a.trace_C && k < a.trace_cap) a.trace_C[k] = (int32_t)C;
  }
  const uint32_t n = a.n;
  const uint32_t nw = (n + 63u) >> 6, nsw = (nw + 63u) >> 6;
  // clear C, find the next smallest unstable label: the last wave of the
  // first workgroup (dispatched first; members go to waves in order, so a
  // small splitter's marking falls to other waves)
  if (p.gwave == min(p.gwaves, (uint32_t)(kLT / kWave)) - 1) {
    const uint32_t w0 = C >> 6;
    const uint64_t bits = a.ub[w0] & ~(1ull << (C & 63));
    if (lane() == 0) {
      a.ub[w0] = bits;
      if (bits == 0) atomicAnd((unsigned long long*)&a.us[w0 >> 6], ~(1ull << (w0 & 63)));
    }
    uint32_t next = kNone;
    for (uint32_t q = w0 >> 6; q < nsw; q += kWave) {
      const uint32_t qq = q + lane();
      uint64_t sv = qq < nsw ? a.us[qq] : 0ull;
      if (qq == (w0 >> 6)) {
        sv &= ~0ull << (w0 & 63);
        const uint64_t b0 = 1ull << (w0 & 63);
        sv = bits ? (sv | b0) : (sv & ~b0);
      }
      const uint64_t bal = __ballot(sv != 0);
      if (bal) {
        const int l = __ffsll((unsigned long long)bal) - 1;
        const uint64_t v = (uint64_t)__shfl((unsigned long long)sv, l, kWave);
        const uint32_t word =
            ((q + (uint32_t)l) << 6) + (uint32_t)(__ffsll((unsigned long long)v) - 1);
        const uint64_t wb = (word == w0) ? bits : a.ub[word];
        if (wb) next = (word << 6) + (uint32_t)(__ffsll((unsigned long long)wb) - 1);
        break;
      }
    }
    if (lane() == 0 && next != kNone) atomicMin(&a.ctl->cand[par ^ 1].v[0], next);
  }
  const bool pre = pf_ok != 0 && pf_C == C;
  const uint32_t cb = pre ? pf_cb : (uint32_t)a.bs[C];
  uint32_t csz = pre ? pf_n : (uint32_t)a.be[C] - cb;
  if (cb > n || csz > n - cb) csz = 0;  // never expected
  if (p.gtid == 0 && a.count) {
    atomicAdd((unsigned long long*)&a.work[0], (unsigned long long)csz);
  }
  // a.mpw members per wave and step (about 64 / the mean in-degree), so that
  // a wave's in-transitions mostly fit one round of its 64 lanes
  for (uint32_t i0 = p.gwave * a.mpw; i0 < csz; i0 += p.gwaves * a.mpw) {
    const uint32_t i = i0 + lane();
    const bool hit = lane() < a.mpw && i < csz;
    uint32_t beg = 0, deg = 0;
    if (hit) {
      if (pre && lane_first && i0 == p.gwave * a.mpw) {  // the wave's first chunk
        beg = pf_hi;
        deg = pf_lo;
      } else {
        const uint64_t x = a.pin[cb + i];
        beg = (uint32_t)(x >> 32);
        deg = (uint32_t)x;
      }
    }
    const uint32_t incl = wave_incl_scan_u32(deg);
    const uint32_t total = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
    count_work(a, 1, total);
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
      int32_t s = 0, b = 0;
      uint32_t lo_ = 0, hi_ = 0;
      if (valid) {
        const uint32_t edge = jb + (ee - (ji - jd));
        s = a.in_src[edge];
        const int32_t o = a.in_ord[edge];
        // the source's block and, in case it leads that block, the block's
        // range are loaded beside the atomics (one round trip, not three)
        b = a.block[s];
        lo_ = (uint32_t)a.bs[s];
        hi_ = (uint32_t)a.be[s];
        atomicOr((unsigned long long*)mword(a, s, o), 1ull << (o & 63));
        const uint64_t tbit = 1ull << (s & 63);
        const uint64_t old = atomicOr((unsigned long long*)&a.tb[s >> 6], (unsigned long long)tbit);
        first = !(old & tbit);
        if (first) atomicAdd(&a.tcn[b], 1);
        // a touched leader of a one-state block has no untouched member
        lead = first && b == s && hi_ > lo_ + 1 && hi_ <= a.n;
      }
      // list entries for first touches and for the listed block's member
      // segments (each with its absolute position range): both wave-aggregated
      // reservations are issued before either result is used
      const uint64_t tbal = __ballot(first);
      count_work(a, 2, (uint64_t)__popcll(tbal));
      const uint32_t nseg = lead ? (hi_ - lo_ + kSeg - 1) / kSeg : 0u;
      const uint32_t sincl = wave_incl_scan_u32(nseg);
      const uint32_t stot = (uint32_t)__shfl((int)sincl, kWave - 1, kWave);
      count_work(a, 3, stot);
      const uint32_t tcnt = (uint32_t)__popcll(tbal);
      uint32_t tbase = 0, sbase = 0;
      if (lane() == 0 && (tcnt | stot) != 0) {
        // one lane, both atomics in flight before either result is waited
        // for; the lane-dependent (always 0) slot keeps the compiler from
        // rewriting each into a wave-wide reduction with its own wait
        const uint32_t z = lane();
        tbase = atomicAdd(&a.ctl->cntT[par].v[z], tcnt);
        sbase = atomicAdd(&a.ctl->cntC[par].v[z], stot);
      }
      tbase = (uint32_t)__shfl((int)tbase, 0, kWave);
      const uint32_t ti = tbase + (uint32_t)__popcll(tbal & ((1ull << lane()) - 1ull));
      if (first && ti < a.n) {
        a.ts[ti] = s;
        a.tbk[ti] = b;
      }
      if (stot) {
        const uint32_t base = (uint32_t)__shfl((int)sbase, 0, kWave) + sincl - nseg;
        for (uint32_t q = 0; q < nseg; ++q) {
          if (base + q >= a.lcap) break;  // never expected (capacity covers every block)
          a.lb[base + q] = s;
          a.lo[base + q] = (int32_t)(lo_ + q * kSeg);
          a.lh[base + q] = (int32_t)min(hi_, lo_ + (q + 1) * kSeg);
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// K: compare, elect, rank
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kLT) k_l_compare(LArgs a, uint32_t kofs) {
  const uint32_t done = a.ctl->state.v[1];
  const uint32_t k = iter_of(a, kofs);
  const uint32_t par = kofs & 1;
  const uint32_t nT = min(a.ctl->cntT[par].v[0], a.n);
  const uint32_t nL = a.ctl->cntC[par].v[0];
  if (done) return;
  const GPart p = gpart();
  const uint64_t epoch = (uint64_t)(k + 1) << 32;
  const uint32_t n = a.n;
  uint32_t* nS = &a.ctl->cntS[par].v[0];
  if (p.gwave == p.gwaves - 1) {
    // prefetch the next iteration's splitter: the candidate the mark kernel
    // found, its range and its first kWave members' in-transition ranges.
    // Should anything split in this iteration, the candidate may still
    // change and ranges move; the swap kernel then marks the slot stale.
    const uint32_t nx = a.ctl->cand[par ^ 1].v[0];
    uint32_t* pn = a.pf + (par ^ 1) * kPfWords;
    uint32_t ncb = 0, nsz = 0;
    bool ok = false;
    if (nx < n) {
      ncb = (uint32_t)a.bs[nx];
      nsz = (uint32_t)a.be[nx] - ncb;
      ok = ncb <= n && nsz <= n - ncb;
    }
    const uint64_t x = (ok && lane() < nsz) ? a.pin[ncb + lane()] : 0ull;
    reinterpret_cast<uint64_t*>(pn + 4)[lane()] = x;
    if (lane() == 0) {
      pn[0] = nx;
      pn[1] = ncb;
      pn[2] = nsz;
      pn[3] = ok ? 1u : 0u;
    }
  }
  const uint32_t half = p.gwaves > 1 ? p.gwaves / 2 : 1;
  if (p.gwave < half) {
    // listed touched states, one per thread of the first half of the grid
    for (uint32_t i0 = p.gwave * kWave; i0 < nT; i0 += half * kWave) {
      const uint32_t i = i0 + lane();
      int32_t s = 0, b = 0;
      bool sp = false;
      if (i < nT) {
        s = a.ts[i];
        b = a.tbk[i];
        sp = (b != s) && marks_differ(a, s, b);
      }
      int32_t r = 0;
      if (sp) {
        atomicMax((unsigned long long*)&a.nlw[b],
                  (unsigned long long)(epoch | (uint64_t)(kNone - (uint32_t)s)));
        r = atomicAdd(&a.cnt[b], 1);
        atomicOr((unsigned long long*)&a.sf[s >> 6], 1ull << (s & 63));
      }
      const uint32_t si = reserve(nS, sp);
      if (sp && si < n) {
        a.ss[si] = s;
        a.sbk[si] = b;
        a.sr[si] = r;
      }
    }
  } else {
    // untouched members of the listed blocks: one segment per wave and step;
    // a block all of whose members were touched has none (its count of first
    // touches equals its size) and is skipped
    for (uint32_t j = p.gwave - half; j < nL && j < a.lcap; j += p.gwaves - half) {
      const int32_t b = a.lb[j];
      const uint32_t lo = (uint32_t)a.lo[j], hi = (uint32_t)a.lh[j];
      if ((uint32_t)a.tcn[b] == (uint32_t)(a.be[b] - a.bs[b])) continue;
      const uint32_t cntm = hi > lo ? min(kSeg, hi - lo) : 0u;
      count_work(a, 4, cntm);
      for (uint32_t i0 = 0; i0 < cntm; i0 += kWave) {
        const uint32_t i = i0 + lane();
        int32_t s = 0;
        bool sp = false;
        if (i < cntm && lo + i < n) {
          s = a.perm[lo + i];
          sp = !test_bit(a.tb, (uint32_t)s);
        }
        const uint64_t bal = __ballot(sp);
        if (!bal) continue;
        // one bid (the smallest splitting state) and one rank reservation per step
        uint32_t sm = sp ? (uint32_t)s : kNone;
        sm = wave_min_u32(sm);
        uint32_t base = 0;
        if (lane() == 0) {
          atomicMax((unsigned long long*)&a.nlw[b],
                    (unsigned long long)(epoch | (uint64_t)(kNone - sm)));
          base = (uint32_t)atomicAdd(&a.cnt[b], (int)__popcll(bal));
        }
        base = (uint32_t)__shfl((int)base, 0, kWave);
        const int32_t r = (int32_t)(base + (uint32_t)__popcll(bal & ((1ull << lane()) - 1ull)));
        if (sp) atomicOr((unsigned long long*)&a.sf[s >> 6], 1ull << (s & 63));
        const uint32_t si = reserve(nS, sp);
        if (sp && si < n) {
          a.ss[si] = s;
          a.sbk[si] = b;
          a.sr[si] = r;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// S: relabel, tail bookkeeping, swaps, new ranges, unstable updates; clear
// marks, touched bits and touched counts.  The split states are relabelled by
// the first R workgroups (one state per thread); the last of them to finish
// (an arrival counter, behind agent-scope release fences, read with an
// acquire) swaps the states of the whole iteration and sets the new ranges,
// so the two steps that need every split state's bookkeeping in between take
// one kernel, not two.  Every workgroup then clears touched states.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void relabel_one(const LArgs& a, uint32_t i) {
  const uint32_t n = a.n;
  const int32_t s = a.ss[i], b = a.sbk[i], r = a.sr[i];
  const uint64_t nv = a.nlw[b];
  const int32_t e = a.be[b], c = a.cnt[b], pv = a.pos[s];
  const int32_t nl = (int32_t)(kNone - (uint32_t)nv);
  a.block[s] = nl;
  const int32_t ne = e - c, q = ne + r;
  int32_t fv = -1, uv = -1;
  const bool ok = ne >= 0 && q >= ne && q < e && e <= (int32_t)n && pv >= 0 && pv < (int32_t)n;
  if (ok) {
    if (pv < ne) fv = atomicAdd(&a.fc[b], 1);
    uv = a.perm[q];  // every tail position is examined once
  } else {
    a.ctl->state.v[4] = 1;  // never expected
  }
  a.sfi[i] = fv;
  a.sne[i] = ok ? ne : 0;
  a.sps[i] = ok ? pv : 0;
  a.sse[i] = (ok && nl == s) ? e : -1;
  if (uv >= 0 && uv < (int32_t)n && !test_bit(a.sf, (uint32_t)uv)) {
    const int32_t jj = atomicAdd(&a.gc[b], 1);
    if (ne + jj < e)
      a.tmp64[ne + jj] = ((uint64_t)(uint32_t)uv << 32) | (uint32_t)q;
    else
      a.ctl->state.v[4] = 1;
  }
}

// the swap of split state i with its staying tail state, and, for the new
// leader, the ranges and unstable bits; returns whether i is a new leader
__device__ __forceinline__ bool swap_one(const LArgs& a, uint32_t i, uint32_t& best) {
  const uint32_t n = a.n;
  const int32_t s = a.ss[i], b = a.sbk[i], fv = a.sfi[i], ne = a.sne[i], ps = a.sps[i];
  const int32_t e = a.sse[i];
  if (fv >= 0 && ne >= 0 && ne + fv < (int32_t)n) {
    const uint64_t x = a.tmp64[ne + fv];
    const int32_t q = (int32_t)(uint32_t)x, su = (int32_t)(x >> 32);
    if (q >= ne && q < (int32_t)n && ps >= 0 && ps < ne && su >= 0 && su < (int32_t)n) {
      const uint64_t xq = a.pin[q], xp = a.pin[ps];
      a.perm[ps] = su;
      a.pos[su] = ps;
      a.pin[ps] = xq;
      a.perm[q] = s;
      a.pos[s] = q;
      a.pin[q] = xp;
    } else {
      a.ctl->state.v[4] = 1;  // never expected
    }
  }
  bool lead = false;
  if (e >= 0) {  // the new leader: one thread per split block
    a.bs[s] = ne;
    a.be[s] = e;
    a.be[b] = ne;
    a.cnt[b] = 0;
    a.fc[b] = 0;
    a.gc[b] = 0;
    set_unstable(a, (uint32_t)b);
    set_unstable(a, (uint32_t)s);
    best = min(best, (uint32_t)b);
    lead = true;
  }
  atomicAnd((unsigned long long*)&a.sf[s >> 6], ~(1ull << (s & 63)));
  return lead;
}

__global__ void __launch_bounds__(kLT) k_l_split(LArgs a, uint32_t kofs) {
  __shared__ uint32_t last;
  const uint32_t done = a.ctl->state.v[1];
  const uint32_t k = iter_of(a, kofs);
  const uint32_t par = kofs & 1;
  const uint32_t nS = min(a.ctl->cntS[par].v[0], a.n);
  const uint32_t nT = min(a.ctl->cntT[par].v[0], a.n);
  const uint32_t C = a.ctl->state.v[3];
  if (done) return;
  const GPart p = gpart();
  if (p.gtid == 0) {
    a.ctl->cand[par].v[0] = kNone;  // the candidate slot of iteration k + 2
    if (a.trace_nsplit && k < a.trace_cap) a.trace_nsplit[k] = nS;
    if (nS > 0) {
      set_unstable(a, C);
      atomicMin(&a.ctl->cand[par ^ 1].v[0], C);
      a.pf[(par ^ 1) * kPfWords + 3] = 0;  // ranges changed: the prefetch is stale
    }
    count_work(a, 7, nS > 0 ? 1 : 0);
  }
  // workgroup-uniform: the first R workgroups relabel, one split state per thread
  const uint32_t R = min((nS + kLT - 1) / kLT, gridDim.x);
  if (blockIdx.x < R) {
    count_work(a, 5, p.gtid == 0 ? nS : 0);
    for (uint32_t i = p.gtid; i < nS; i += R * kLT) relabel_one(a, i);
    __threadfence();  // release this workgroup's bookkeeping
    __syncthreads();
    if (threadIdx.x == 0) {
      const uint32_t prev = atomicAdd(&a.ctl->ltany[0].v[0], 1u);
      last = (prev == R - 1) ? 1u : 0u;
      if (last) a.ctl->ltany[0].v[0] = 0;  // every arrival of this kernel is in
    }
    __syncthreads();
    if (last) {  // workgroup-uniform
      __threadfence();  // acquire the other workgroups' bookkeeping
      uint32_t best = kNone, leaders = 0;
      for (uint32_t i = threadIdx.x; i < nS; i += kLT)
        if (swap_one(a, i, best)) ++leaders;
      best = wave_min_u32(best);
      if (lane() == 0 && best != kNone) atomicMin(&a.ctl->cand[par ^ 1].v[0], best);
      count_work(a, 6, wave_sum_u64(leaders));
    }
  }
  // clear the marks, touched bits and touched counts of this iteration's
  // touched states
  for (uint32_t i = p.gtid; i < nT; i += p.gthreads) {
    const int32_t s = a.ts[i];
    a.tcn[a.tbk[i]] = 0;  // every touched state of the block clears it
    if (a.uniform) {
      a.mw[s] = 0;
    } else {
      for (uint32_t w = a.woff[s]; w < a.woff[s + 1]; ++w) a.mw[w] = 0;
    }
    a.tb[s >> 6] = 0;  // every touched state of the word clears it
  }
}

// after a graph replay of `by` iterations: advance the iteration base
__global__ void k_l_advance(LArgs a, uint32_t by) {
  if (threadIdx.x == 0 && blockIdx.x == 0) a.ctl->state.v[6] += by;
}

// ---------------------------------------------------------------------------
// per-run set-up of the refinable partition (after the common run
// initialisation has written block[], the bitmaps and the control block)
// ---------------------------------------------------------------------------
__global__ void k_l_zero(LArgs a) {
  const GPart p = gpart();
  for (uint32_t s = p.gtid; s < a.n; s += p.gthreads) {
    a.cnt[s] = 0;
    a.fc[s] = 0;
    a.gc[s] = 0;
    a.tcn[s] = 0;
  }
  if (p.gtid < 8) a.work[p.gtid] = 0;
  if (p.gtid < 2) a.pf[p.gtid * kPfWords + 3] = 0;
}
__global__ void k_l_count(LArgs a) {
  const GPart p = gpart();
  for (uint32_t s = p.gtid; s < a.n; s += p.gthreads) atomicAdd(&a.cnt[a.block[s]], 1);
}
__global__ void k_l_fill(LArgs a) {
  const GPart p = gpart();
  for (uint32_t s = p.gtid; s < a.n; s += p.gthreads) {
    const uint32_t q = (uint32_t)atomicAdd(&a.be[a.block[s]], 1);
    if (q < a.n) {
      a.perm[q] = (int32_t)s;
      a.pos[s] = (int32_t)q;
      const uint32_t e0 = a.in_ptr[s];
      a.pin[q] = ((uint64_t)e0 << 32) | (a.in_ptr[s + 1] - e0);
    } else {
      a.ctl->state.v[4] = 1;  // never expected
    }
  }
}
__global__ void k_l_zero_cnt(LArgs a) {
  const GPart p = gpart();
  for (uint32_t b = p.gtid; b < a.n; b += p.gthreads) a.cnt[b] = 0;
}

template <class T>
bisim_status lalloc(T** p, size_t count, hipStream_t s) {
  if (*p) return BISIM_OK;
  if (count == 0) count = 1;
  hipError_t e = dev_alloc((void**)p, sizeof(T) * count, s);
  if (e != hipSuccess) {
    set_error("device allocation of %zu bytes failed: %s", sizeof(T) * count, hipGetErrorString(e));
    return BISIM_E_NOMEM;
  }
  return BISIM_OK;
}

}  // namespace

// capacity of the segment list: every block contributes at most
// ceil(size / kSeg) <= size / kSeg + 1 segments
static uint64_t seg_capacity(uint64_t n) { return n + n / kSeg + 64; }

bisim_status lists_alloc(bisim_lts* h) {
  const size_t n = (size_t)h->n;
  hipStream_t s = h->stream;
  bisim_lists& L = h->lists;
  BISIM_TRY(lalloc(&L.perm, n, s));
  BISIM_TRY(lalloc(&L.pos, n, s));
  BISIM_TRY(lalloc(&L.bs, n + 1, s));
  BISIM_TRY(lalloc(&L.be, n, s));
  BISIM_TRY(lalloc(&L.cnt, n, s));
  BISIM_TRY(lalloc(&L.fc, n, s));
  BISIM_TRY(lalloc(&L.gc, n, s));
  BISIM_TRY(lalloc(&L.tcn, n, s));
  BISIM_TRY(lalloc(&L.pin, n, s));
  BISIM_TRY(lalloc(&L.pf, 2 * (size_t)kPfWords, s));
  BISIM_TRY(lalloc(&L.tmp64, n, s));
  BISIM_TRY(lalloc(&L.lb, seg_capacity(n), s));
  BISIM_TRY(lalloc(&L.lo, seg_capacity(n), s));
  BISIM_TRY(lalloc(&L.lh, seg_capacity(n), s));
  int32_t** lists[] = {&L.ts, &L.tbk, &L.ss, &L.sbk, &L.sr, &L.sfi, &L.sne, &L.sps, &L.sse};
  for (int32_t** q : lists) BISIM_TRY(lalloc(q, n, s));
  BISIM_TRY(lalloc(&L.work, 8, s));
  return BISIM_OK;
}

// The iteration loop of engine 3; the common run initialisation has been
// enqueued (block[] = the start partition, bitmaps, bids, control block).
bisim_status lists_loop(bisim_lts* h, uint32_t cap, bool count_work_totals) {
  BISIM_TRY(lists_alloc(h));
  hipStream_t st = h->stream;
  const uint32_t n = (uint32_t)h->n;
  bisim_lists& L = h->lists;
  LArgs a{};
  a.n = n;
  a.uniform = h->uniform;
  a.nwd = ((uint64_t)n + 63) / 64;
  a.in_ptr = h->in_ptr;
  a.in_src = h->in_src;
  a.in_ord = h->in_ord;
  a.woff = h->woff;
  a.block = h->block;
  a.mw = h->mw;
  a.tb = h->tb;
  a.sf = h->sb;
  a.ub = h->ub;
  a.us = h->us;
  a.nlw = h->nlw;
  a.perm = L.perm;
  a.pos = L.pos;
  a.bs = L.bs;
  a.be = L.be;
  a.cnt = L.cnt;
  a.fc = L.fc;
  a.gc = L.gc;
  a.tcn = L.tcn;
  a.pin = L.pin;
  a.pf = L.pf;
  a.tmp64 = L.tmp64;
  a.lb = L.lb;
  a.lo = L.lo;
  a.lh = L.lh;
  a.lcap = (uint32_t)seg_capacity(n);
  {
    const uint64_t deg = n > 0 ? ((uint64_t)h->m + n - 1) / n : 1;  // mean in-degree, rounded up
    uint32_t mpw = 64;
    while (mpw > 1 && (uint64_t)mpw * (deg ? deg : 1) > 64) mpw >>= 1;
    a.mpw = mpw;
  }
  a.ts = L.ts;
  a.tbk = L.tbk;
  a.ss = L.ss;
  a.sbk = L.sbk;
  a.sr = L.sr;
  a.sfi = L.sfi;
  a.sne = L.sne;
  a.sps = L.sps;
  a.sse = L.sse;
  a.work = L.work;
  a.count = count_work_totals ? 1 : 0;
  a.ctl = h->ctl;
  a.iter_cap = cap;
  a.trace_C = h->trace_C;
  a.trace_nsplit = h->trace_nsplit;
  a.trace_cap = (uint32_t)h->trace_cap;

  const int cu = h->num_cu > 0 ? h->num_cu : 1;
  int64_t gi = ((int64_t)n + kLT - 1) / kLT;
  gi = gi > cu * 8 ? cu * 8 : (gi < 1 ? 1 : gi);
  hipLaunchKernelGGL(k_l_zero, dim3((unsigned)gi), dim3(kLT), 0, st, a);
  hipLaunchKernelGGL(k_l_count, dim3((unsigned)gi), dim3(kLT), 0, st, a);
  BISIM_TRY_HIP(hipGetLastError());
  BISIM_TRY(exclusive_scan_u32(reinterpret_cast<const uint32_t*>(L.cnt),
                               reinterpret_cast<uint32_t*>(L.bs), n, st));
  if (n > 0)
    BISIM_TRY_HIP(hipMemcpyAsync(L.be, L.bs, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(k_l_fill, dim3((unsigned)gi), dim3(kLT), 0, st, a);
  hipLaunchKernelGGL(k_l_zero_cnt, dim3((unsigned)gi), dim3(kLT), 0, st, a);
  BISIM_TRY_HIP(hipGetLastError());

  const int grid = h->grid > 0 ? h->grid : cu * 8;
  h->run_grid = grid;
  const bool prof = h->profile_every > 0;
  std::vector<uint32_t> sampled;
  std::vector<hipEvent_t> starts;
  if (prof) {
    // eager launches (the iteration base stays 0), with events bound to the
    // ends of the kernels of every P-th iteration
    if (!h->pev) {
      h->pev = new (std::nothrow) hipEvent_t[8 * 256];
      if (!h->pev) return BISIM_E_NOMEM;
      for (int i = 0; i < 8 * 256; ++i) BISIM_TRY_HIP(hipEventCreate(&h->pev[i]));
      h->pev_slots = 256;
    }
    auto go = [&](auto kern, hipEvent_t stop, uint32_t k) {
      if (stop)
        hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kLT), 0, st, nullptr, stop, 0, a, k);
      else
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kLT), 0, st, a, k);
    };
    const uint64_t pe = (uint64_t)h->profile_every;
    hipEvent_t carry = nullptr;
    uint32_t k = 0, chunk = 8;
    for (;;) {
      for (uint32_t j = 0; j < chunk; ++j, ++k) {
        hipEvent_t ends[kPhases] = {nullptr, nullptr, nullptr};
        const size_t slot = sampled.size();
        if (carry && slot < (size_t)h->pev_slots) {
          for (int q = 0; q < kPhases; ++q) ends[q] = h->pev[8 * slot + 1 + q];
          sampled.push_back(k);
          starts.push_back(carry);
        }
        carry = nullptr;
        if ((k + 1) % pe == 0 && sampled.size() < (size_t)h->pev_slots) {
          if (!ends[kPhases - 1]) ends[kPhases - 1] = h->pev[8 * sampled.size()];
          carry = ends[kPhases - 1];
        }
        go(k_l_mark, ends[0], k);
        go(k_l_compare, ends[1], k);
        go(k_l_split, ends[2], k);
      }
      BISIM_TRY_HIP(hipGetLastError());
      BISIM_TRY_HIP(hipMemcpyAsync(&h->ctl_host->state, &h->ctl->state, sizeof(Line),
                                   hipMemcpyDeviceToHost, st));
      BISIM_TRY_HIP(hipStreamSynchronize(st));
      if (h->ctl_host->state.v[1]) break;
      if (k >= cap + 1) break;
      if (chunk < 256) chunk *= 2;
    }
  } else {
    // a graph of kGraphIters iterations, captured once per argument set and
    // replayed until the done flag is set.  The null stream cannot be
    // captured: the handle then uses a stream of its own, created blocking,
    // so that it is ordered with the null stream's work before and after.
    static_assert(sizeof(LArgs) <= sizeof(L.gargs), "graph argument record");
    if (!st && !L.own) BISIM_TRY_HIP(hipStreamCreate(&L.own));
    hipStream_t gs = st ? st : L.own;
    if (!L.gexec || L.ggrid != grid || memcmp(L.gargs, &a, sizeof(LArgs)) != 0) {
      if (L.gexec) {
        (void)hipGraphExecDestroy(L.gexec);
        L.gexec = nullptr;
      }
      hipGraph_t graph = nullptr;
      BISIM_TRY_HIP(hipStreamBeginCapture(gs, hipStreamCaptureModeThreadLocal));
      for (uint32_t j = 0; j < kGraphIters; ++j) {
        hipLaunchKernelGGL(k_l_mark, dim3(grid), dim3(kLT), 0, gs, a, j);
        hipLaunchKernelGGL(k_l_compare, dim3(grid), dim3(kLT), 0, gs, a, j);
        hipLaunchKernelGGL(k_l_split, dim3(grid), dim3(kLT), 0, gs, a, j);
      }
      hipLaunchKernelGGL(k_l_advance, dim3(1), dim3(64), 0, gs, a, kGraphIters);
      const hipError_t le = hipGetLastError();
      const hipError_t ce = hipStreamEndCapture(gs, &graph);
      BISIM_TRY_HIP(le);
      BISIM_TRY_HIP(ce);
      const hipError_t ie = hipGraphInstantiate(&L.gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      BISIM_TRY_HIP(ie);
      memcpy(L.gargs, &a, sizeof(LArgs));
      L.ggrid = grid;
    }
    uint64_t launched = 0;
    uint32_t reps = 1;
    for (;;) {
      for (uint32_t r = 0; r < reps; ++r) BISIM_TRY_HIP(hipGraphLaunch(L.gexec, gs));
      launched += (uint64_t)reps * kGraphIters;
      BISIM_TRY_HIP(hipMemcpyAsync(&h->ctl_host->state, &h->ctl->state, sizeof(Line),
                                   hipMemcpyDeviceToHost, gs));
      BISIM_TRY_HIP(hipStreamSynchronize(gs));
      if (h->ctl_host->state.v[1]) break;
      if (launched >= (uint64_t)cap + 1) break;
      if (reps < 8) reps *= 2;
    }
  }
  for (int q = 0; q < 4; ++q) {
    h->phase_ms[q] = 0;
    h->phase_cnt[q] = 0;
  }
  const uint64_t iters = h->ctl_host->state.v[0];
  for (size_t i = 0; i < sampled.size(); ++i) {
    if ((uint64_t)sampled[i] + 1 >= iters) continue;
    hipEvent_t prev = starts[i];
    for (int q = 0; q < kPhases; ++q) {
      hipEvent_t cur = h->pev[8 * i + 1 + q];
      float pm = 0.f;
      if (hipEventElapsedTime(&pm, prev, cur) == hipSuccess) {
        h->phase_ms[q] += pm;
        h->phase_cnt[q] += 1;
      }
      prev = cur;
    }
  }
  if (count_work_totals)
    BISIM_TRY_HIP(hipMemcpyAsync(h->lists_work, L.work, sizeof(h->lists_work),
                                 hipMemcpyDeviceToHost, st));
  else
    for (uint64_t& w : h->lists_work) w = 0;
  return BISIM_OK;
}

void lists_free(bisim_lts* h) {
  bisim_lists& L = h->lists;
  if (L.gexec) (void)hipGraphExecDestroy(L.gexec);
  if (L.own) {
    (void)hipStreamSynchronize(L.own);
    (void)hipStreamDestroy(L.own);
  }
  void* ptrs[] = {L.perm, L.pos, L.bs,  L.be,  L.cnt, L.fc,  L.gc,  L.tmp64, L.lb, L.lo, L.lh, L.ts,
                  L.tbk,  L.ss,  L.sbk, L.sr,  L.sfi, L.sne, L.sps, L.sse,   L.work, L.tcn,
                  L.pin,  L.pf};
  for (void* q : ptrs)
    if (q) (void)dev_free(q, h->stream);
  L = bisim_lists{};
}

}  // namespace bisim
