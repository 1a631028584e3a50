// Device-side phases of one refinement iteration (see refine.hip for the
// algorithm), shared by the refinement engines and the training-data
// collector.  Everything here has internal linkage: each translation unit
// that includes it gets its own copy of the kernels.
#pragma once

#include "internal.h"
#include "mlp_dev.h"

namespace bisim {
namespace {

struct Args {
  int32_t n;
  int uniform;
  int hot;      // some state has >= kHotDegree outgoing transitions: combine its marks
  const uint32_t* __restrict__ in_ptr;
  const int32_t* __restrict__ in_src;
  const int32_t* __restrict__ in_ord;
  const uint32_t* __restrict__ woff;
  int32_t* block;
  uint64_t* mw;
  uint64_t* tb;
  uint64_t* lt;
  uint64_t* ub;
  uint64_t* us;  // summary: bit w set iff ub[w] != 0
  uint64_t* nlw;
  int32_t* tlist;
  int32_t* slist;
  uint64_t* sb;     // [2][nwd] split flags (two-kernel engine)
  int32_t* nlist;   // [n] new leaders (two-kernel engine)
  uint64_t nwords;  // mark words per parity half
  uint32_t rcpp;    // Algorithm 2: the splitter is not made unstable again after a split
  Ctl* ctl;
  uint32_t iter_cap;
  int32_t* trace_C;
  int64_t* trace_nsplit;
  int64_t* trace_work;
  uint32_t trace_cap;
  // block features and the learned policy
  const uint32_t* sfeat;  // [n][16]
  uint32_t* acc;          // [n][17]
  uint32_t* born;         // [n] iterations completed when the block was created / last split
  uint32_t* used;         // [n] iterations completed when the block was last the splitter
  int32_t* chg;           // [2n] (old, new) label pairs of this iteration's splits
  const uint16_t* wbf;    // bf16 network parameters
  uint32_t rescore;       // full re-scoring period
  // learned policy: unstable labels by priority level, three bitmap levels
  // each (labels; words; summary words), kept exact
  uint8_t* lvl;   // [n] level of each label in the structure
  uint64_t* lvb;  // [kLevels][nwd]
  uint64_t* lvs;  // [kLevels][nsw]
  uint64_t* lvt;  // [kLevels][ntw]
  uint8_t* lvq;   // [2n+1] scratch: new level per re-scored entry
};

struct Part {
  uint32_t gtid, gthreads, gwave, gwaves;
};

// chunks per wave and step of the grid-wide block[] scans (the whole grid
// already keeps enough loads in flight)
constexpr uint32_t kGridScanU = 1;

__device__ __forceinline__ Part part() {
  const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t gthreads = gridDim.x * blockDim.x;
  return {gtid, gthreads, gtid / kWave, gthreads / kWave};
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t o = (uint64_t)__shfl_xor((unsigned long long)v, d, kWave);
    v = o > v ? o : v;
  }
  return v;
}

// Block features: size, outgoing and incoming transitions of the members by
// label mod 8, iterations since the block was created or last split (all
// log1p-scaled), and whether the block has been the splitter since it was
// created or last split (0/1).  kcur = number of iterations completed.
__device__ __forceinline__ float block_feature(const Args& a, uint32_t b, uint32_t f,
                                               uint32_t kcur) {
  if (f < 17) return log1pf((float)a.acc[(size_t)b * 17 + f]);
  if (f == 17) return log1pf((float)(kcur - a.born[b]));
  if (f == 18) return a.used[b] > a.born[b] ? 1.f : 0.f;
  return 0.f;
}

// one wave: priority level of block b (wave-uniform)
__device__ __forceinline__ uint32_t block_level(const Args& a, const MlpLds& M, uint32_t b,
                                                uint32_t kcur) {
  const float x = block_feature(a, b, lane(), kcur);
  float z1, z2;
  return score_level(mlp_forward_lanes(M, kPolicyF, x, &z1, &z2));
}

// ---- the level structure of the learned policy ----------------------------
struct LvDims {
  uint32_t nwd, nsw, ntw;
};
__device__ __forceinline__ LvDims lv_dims(const Args& a) {
  const uint32_t nwd = ((uint32_t)a.n + 63u) >> 6;
  const uint32_t nsw = (nwd + 63u) >> 6;
  return {nwd, nsw, (nsw + 63u) >> 6};
}
__device__ __forceinline__ uint64_t aload(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Insert label b at level L.  Safe against concurrent insertions.
__device__ __forceinline__ void lv_insert(const Args& a, uint32_t b, uint32_t L) {
  const LvDims d = lv_dims(a);
  const uint32_t w = b >> 6, sw = w >> 6;
  const uint64_t o1 = atomicOr((unsigned long long*)&a.lvb[(size_t)L * d.nwd + w], 1ull << (b & 63));
  if (o1 != 0) return;
  const uint64_t o2 = atomicOr((unsigned long long*)&a.lvs[(size_t)L * d.nsw + sw], 1ull << (w & 63));
  if (o2 != 0) return;
  atomicOr((unsigned long long*)&a.lvt[(size_t)L * d.ntw + (sw >> 6)], 1ull << (sw & 63));
}
// Remove label b from level L (no-op if absent).  Safe against concurrent
// removals; must not run concurrently with insertions.
__device__ __forceinline__ void lv_remove(const Args& a, uint32_t b, uint32_t L) {
  const LvDims d = lv_dims(a);
  const uint32_t w = b >> 6, sw = w >> 6;
  const uint64_t bit = 1ull << (b & 63), sbit = 1ull << (w & 63);
  const uint64_t o1 = atomicAnd((unsigned long long*)&a.lvb[(size_t)L * d.nwd + w], ~bit);
  if (!(o1 & bit) || (o1 & ~bit)) return;
  const uint64_t o2 = atomicAnd((unsigned long long*)&a.lvs[(size_t)L * d.nsw + sw], ~sbit);
  if (!(o2 & sbit) || (o2 & ~sbit)) return;
  atomicAnd((unsigned long long*)&a.lvt[(size_t)L * d.ntw + (sw >> 6)], ~(1ull << (sw & 63)));
}
// one wave, from the summary word chunk q whose ballot is bal: the smallest
// label of level L
__device__ __forceinline__ uint32_t lv_descend(const Args& a, const LvDims& d, uint32_t L,
                                               uint32_t q, uint64_t bal, uint64_t v) {
  const int l = __ffsll((unsigned long long)bal) - 1;
  const uint64_t tv = (uint64_t)__shfl((unsigned long long)v, l, kWave);
  const uint32_t sw = ((q + (uint32_t)l) << 6) + (uint32_t)(__ffsll((unsigned long long)tv) - 1);
  const uint64_t sv = aload(&a.lvs[(size_t)L * d.nsw + sw]);
  if (sv == 0) return kNone - 1;  // inconsistent structure
  const uint32_t w = (sw << 6) + (uint32_t)(__ffsll((unsigned long long)sv) - 1);
  const uint64_t wv = aload(&a.lvb[(size_t)L * d.nwd + w]);
  if (wv == 0) return kNone - 1;
  const uint32_t b = (w << 6) + (uint32_t)(__ffsll((unsigned long long)wv) - 1);
  return b < (uint32_t)a.n ? b : kNone - 1;
}
// one wave: the smallest label of the highest non-empty level, kNone if the
// structure is empty, kNone - 1 if it is inconsistent
__device__ uint32_t lv_search(const Args& a) {
  const LvDims d = lv_dims(a);
  if (d.ntw <= (uint32_t)kWave) {
    uint64_t v[kLevels];
#pragma unroll
    for (int L = 0; L < kLevels; ++L)
      v[L] = lane() < d.ntw ? aload(&a.lvt[(size_t)L * d.ntw + lane()]) : 0ull;
#pragma unroll
    for (int L = kLevels - 1; L >= 0; --L) {
      const uint64_t bal = __ballot(v[L] != 0);
      if (bal) return lv_descend(a, d, (uint32_t)L, 0, bal, v[L]);
    }
    return kNone;
  }
  for (int L = kLevels - 1; L >= 0; --L)
    for (uint32_t q = 0; q < d.ntw; q += kWave) {
      const uint64_t v = q + lane() < d.ntw ? aload(&a.lvt[(size_t)L * d.ntw + q + lane()]) : 0ull;
      const uint64_t bal = __ballot(v != 0);
      if (bal) return lv_descend(a, d, (uint32_t)L, q, bal, v);
    }
  return kNone;
}

// Start of iteration k: returns C, or kNone when the loop ends (no unstable
// block, which is the final counted pass, or the iteration cap).
__device__ uint32_t head(const Args& a, uint32_t k, const Part& p) {
  const uint32_t C = a.ctl->cand[k & 1].v[0];
  const bool over = (k + 1 > a.iter_cap);
  if (p.gtid == 0) {
    Ctl* c = a.ctl;
    if (C == kNone || over) {
      c->state.v[0] = k + 1;
      c->state.v[1] = 1;
      if (over && C != kNone) c->state.v[2] = 1;
      if (a.trace_C && k < a.trace_cap) a.trace_C[k] = -1;
      if (a.trace_nsplit && k < a.trace_cap) a.trace_nsplit[k] = 0;
      if (a.trace_work && k < a.trace_cap)
        for (int q = 0; q < 4; ++q) a.trace_work[4 * (uint64_t)k + q] = 0;
    } else {
      const uint32_t nx = (k & 1) ^ 1;
      c->state.v[3] = C;
      c->cntT[nx].v[0] = 0;
      c->cntS[nx].v[0] = 0;
      c->ltany[nx].v[0] = 0;
      c->work[nx].v[0] = 0;
      c->work[nx].v[1] = 0;
      c->cntC[nx].v[0] = 0;
      if (a.used) a.used[C] = k + 1;
      if (a.trace_C && k < a.trace_cap) a.trace_C[k] = (int32_t)C;
    }
  }
  return (C == kNone || over) ? kNone : C;
}

// set / clear an unstable label, keeping the summary level (one bit per
// non-zero word of ub) exact
__device__ __forceinline__ void unstable_set(const Args& a, uint32_t b) {
  const uint32_t w = b >> 6;
  const uint64_t old = atomicOr((unsigned long long*)&a.ub[w], 1ull << (b & 63));
  if (old == 0) atomicOr((unsigned long long*)&a.us[w >> 6], 1ull << (w & 63));
}

// A: clear C and, for the plain policy, find the next iteration's candidate.
// Plain policy: C is the smallest unstable label, so the smallest remaining
// one is the next set bit after C; one wave finds it through the summary
// level.  Labels made unstable later in this iteration are min-reduced into
// the candidate in C.  Learned policy: the candidate is chosen after the
// re-scoring at the end of the iteration.
template <bool L>
__device__ void phase_a_select(const Args& a, uint32_t par, uint32_t C, uint32_t k,
                               const Part& p) {
  if (p.gwave != 0) return;
  const uint32_t nwd = ((uint32_t)a.n + 63u) >> 6;
  const uint32_t w0 = C >> 6;
  const uint64_t bits = a.ub[w0] & ~(1ull << (C & 63));
  if (lane() == 0) {
    a.ub[w0] = bits;
    if (bits == 0) atomicAnd((unsigned long long*)&a.us[w0 >> 6], ~(1ull << (w0 & 63)));
  }
  if (L) return;
  // Labels below C are stable, except in the first iteration, where the
  // splitter may have been forced: search from word 0 there.  Word w0 is
  // taken from `bits` (this wave's own update may not be visible yet).
  const uint32_t from = (k == 0) ? 0u : w0;
  const uint32_t nsw = (nwd + 63u) >> 6;
  uint32_t next = kNone;
  for (uint32_t q = from >> 6; q < nsw; q += kWave) {
    const uint32_t qq = q + lane();
    uint64_t sv = qq < nsw ? a.us[qq] : 0ull;
    if (qq == (from >> 6)) sv &= ~0ull << (from & 63);
    if (qq == (w0 >> 6)) {
      const uint64_t b0 = 1ull << (w0 & 63);
      sv = bits ? (sv | b0) : (sv & ~b0);
    }
    const uint64_t bal = __ballot(sv != 0);
    if (bal) {
      const int l = __ffsll((unsigned long long)bal) - 1;
      const uint64_t v = (uint64_t)__shfl((unsigned long long)sv, l, kWave);
      const uint32_t word = ((q + (uint32_t)l) << 6) + (uint32_t)(__ffsll((unsigned long long)v) - 1);
      const uint64_t wb = (word == w0) ? bits : a.ub[word];
      if (wb) next = (word << 6) + (uint32_t)(__ffsll((unsigned long long)wb) - 1);
      break;
    }
  }
  if (lane() == 0 && next != kNone) a.ctl->cand[par ^ 1].v[0] = next;
}

__device__ __forceinline__ void mark_slot(const Args& a, uint32_t par, int32_t s, int32_t o,
                                          bool valid) {
  bool first = false;
  if (valid) {
    const uint64_t bit = 1ull << (o & 63);
    const uint64_t wi = a.uniform ? (uint64_t)s : (uint64_t)a.woff[s] + (uint32_t)(o >> 6);
    const uint64_t tbit = 1ull << (s & 63);
    if (a.uniform) {
      const uint64_t old = atomicOr((unsigned long long*)&a.mw[wi], (unsigned long long)bit);
      first = (old == 0);
      if (first) atomicOr((unsigned long long*)&a.tb[s >> 6], (unsigned long long)tbit);
    } else {
      atomicOr((unsigned long long*)&a.mw[wi], (unsigned long long)bit);
      first = !(atomicOr((unsigned long long*)&a.tb[s >> 6], (unsigned long long)tbit) & tbit);
    }
    if (first && a.block[s] == s) {
      atomicOr((unsigned long long*)&a.lt[s >> 6], (unsigned long long)tbit);
      a.ctl->ltany[par].v[0] = 1;
    }
  }
  wave_push(a.tlist, &a.ctl->cntT[par].v[0], s, first);
}

// A: mark.  Waves scan block[] (coalesced); the in-transitions of the hits
// are spread over the wave's 64 lanes by a prefix sum of in-degrees.
__device__ void phase_a_mark(const Args& a, uint32_t par, uint32_t C, const Part& p) {
  const uint32_t n = (uint32_t)a.n;
  for (uint32_t base0 = p.gwave * kWave * kGridScanU; base0 < n; base0 += p.gwaves * kWave * kGridScanU) {
   const uint32_t hm = hit_mask<kGridScanU>(a.block, base0, n, C);
   if (__ballot(hm != 0) == 0) continue;
   for (uint32_t u = 0; u < kGridScanU; ++u) {
    const uint32_t t = base0 + u * kWave + lane();
    const bool hit = (hm >> u) & 1u;
    const uint64_t hits = __ballot(hit);
    if (hits == 0) continue;
    uint32_t beg = 0, deg = 0;
    if (hit) {
      beg = a.in_ptr[t];
      deg = a.in_ptr[t + 1] - beg;
    }
    const uint32_t incl = wave_incl_scan_u32(deg);
    const uint32_t total = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
    if (a.trace_work && lane() == 0) {
      atomicAdd(&a.ctl->work[par].v[0], (uint32_t)__popcll(hits));
      atomicAdd(&a.ctl->work[par].v[1], total);
    }
    for (uint32_t e0 = 0; e0 < total; e0 += kWave) {
      const uint32_t e = e0 + lane();
      const bool valid = e < total;
      const uint32_t ee = valid ? e : total - 1;
      uint32_t j = 0;  // owner lane: the first with incl > ee
#pragma unroll
      for (uint32_t step = 32; step >= 1; step >>= 1) {
        const uint32_t probe = (uint32_t)__shfl((int)incl, (int)(j + step - 1), kWave);
        if (probe <= ee) j += step;
      }
      const uint32_t jb = (uint32_t)__shfl((int)beg, (int)j, kWave);
      const uint32_t ji = (uint32_t)__shfl((int)incl, (int)j, kWave);
      const uint32_t jd = (uint32_t)__shfl((int)deg, (int)j, kWave);
      const uint32_t edge = jb + (ee - (ji - jd));
      int32_t s = 0, o = 0;
      if (valid) {
        s = a.in_src[edge];
        o = a.in_ord[edge];
      }
      mark_slot(a, par, s, o, valid);
    }
   }
  }
}

__device__ __forceinline__ void bid(const Args& a, int32_t b, int32_t s, uint64_t epoch) {
  const uint64_t val = epoch | (uint64_t)(kNone - (uint32_t)s);
  const uint64_t cur = __hip_atomic_load(&a.nlw[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (cur < val) atomicMax((unsigned long long*)&a.nlw[b], (unsigned long long)val);
}

// B: compare with the leader and elect
__device__ void phase_b(const Args& a, uint32_t par, uint32_t k, const Part& p) {
  const uint64_t epoch = (uint64_t)(k + 1) << 32;
  const uint32_t nT = a.ctl->cntT[par].v[0];
  uint32_t* cntS = &a.ctl->cntS[par].v[0];
  for (uint32_t i0 = p.gwave * kWave; i0 < nT; i0 += p.gwaves * kWave) {
    const uint32_t i = i0 + lane();
    bool sp = false;
    int32_t s = 0, b = 0;
    if (i < nT) {
      s = a.tlist[i];
      b = a.block[s];
      if (s != b) {
        if (a.uniform) {
          sp = a.mw[s] != a.mw[b];
        } else {
          const uint32_t w0 = a.woff[s], w1 = a.woff[s + 1], wb = a.woff[b];
          for (uint32_t q = 0; q < w1 - w0; ++q)
            if (a.mw[w0 + q] != a.mw[wb + q]) {
              sp = true;
              break;
            }
        }
      }
    }
    if (sp) bid(a, b, s, epoch);
    wave_push(a.slist, cntS, s, sp);
  }
  if (a.ctl->ltany[par].v[0]) {
    const uint32_t n = (uint32_t)a.n;
    for (uint32_t base0 = p.gwave * kWave * kGridScanU; base0 < n;
         base0 += p.gwaves * kWave * kGridScanU) {
      int32_t bv[kGridScanU];
      uint64_t lw[kGridScanU], tw[kGridScanU];
#pragma unroll
      for (uint32_t u = 0; u < kGridScanU; ++u) {
        const uint32_t s = base0 + u * kWave + lane();
        bv[u] = s < n ? a.block[s] : 0;
      }
#pragma unroll
      for (uint32_t u = 0; u < kGridScanU; ++u) lw[u] = a.lt[(uint32_t)bv[u] >> 6];
#pragma unroll
      for (uint32_t u = 0; u < kGridScanU; ++u)
        tw[u] = base0 + u * kWave < n ? a.tb[(base0 + u * kWave) >> 6] : 0ull;
#pragma unroll
      for (uint32_t u = 0; u < kGridScanU; ++u) {
        const uint32_t s = base0 + u * kWave + lane();
        const int32_t b = bv[u];
        const bool sp =
            s < n && ((lw[u] >> (b & 63)) & 1ull) && !((tw[u] >> (s & 63)) & 1ull);
        if (sp) bid(a, b, (int32_t)s, epoch);
        wave_push(a.slist, cntS, (int32_t)s, sp);
      }
    }
  }
}

// C: relabel and update the unstable set (T: keep block features; L: learned
// policy bookkeeping)
template <bool L, bool T>
__device__ void phase_c(const Args& a, uint32_t par, uint32_t k, uint32_t C, const Part& p) {
  const uint32_t nS = a.ctl->cntS[par].v[0];
  const uint32_t nT = a.ctl->cntT[par].v[0];
  uint32_t best = kNone;
  for (uint32_t i0 = p.gwave * kWave; i0 < nS; i0 += p.gwaves * kWave) {
    const uint32_t i = i0 + lane();
    bool lead = false;
    int32_t old = 0, nl = 0;
    if (i < nS) {
      const int32_t s = a.slist[i];
      old = a.block[s];
      nl = (int32_t)(kNone - (uint32_t)a.nlw[old]);
      a.block[s] = nl;
      lead = (s == nl);
      if (T) {
        atomicAdd(&a.acc[(size_t)nl * 17], 1u);
        atomicSub(&a.acc[(size_t)old * 17], 1u);
        for (int q = 0; q < 16; ++q) {
          const uint32_t v = a.sfeat[(size_t)s * 16 + q];
          if (v) {
            atomicAdd(&a.acc[(size_t)nl * 17 + 1 + q], v);
            atomicSub(&a.acc[(size_t)old * 17 + 1 + q], v);
          }
        }
      }
      if (lead) {
        unstable_set(a, (uint32_t)old);
        unstable_set(a, (uint32_t)nl);
        best = min(best, (uint32_t)old);
        if (T) {
          a.born[old] = k + 1;
          a.born[nl] = k + 1;
        }
      }
    }
    if (L) {  // record (old, new) pairs for re-scoring
      const uint64_t bal = __ballot(lead);
      if (bal) {
        const int leader = __ffsll((unsigned long long)bal) - 1;
        uint32_t base = 0;
        if ((int)lane() == leader) base = atomicAdd(&a.ctl->cntC[par].v[0], (uint32_t)__popcll(bal));
        base = (uint32_t)__shfl((int)base, leader, kWave);
        if (lead) {
          const uint32_t idx = base + __popcll(bal & ((1ull << lane()) - 1ull));
          a.chg[2 * idx] = old;
          a.chg[2 * idx + 1] = nl;
        }
      }
    }
  }
  for (uint32_t i = p.gtid; i < nT; i += p.gthreads) {
    const int32_t s = a.tlist[i];
    if (a.uniform) {
      a.mw[s] = 0;
    } else {
      for (uint32_t q = a.woff[s]; q < a.woff[s + 1]; ++q) a.mw[q] = 0;
    }
    a.tb[s >> 6] = 0;
    a.lt[s >> 6] = 0;
  }
  if (!L) {
    best = wave_min_u32(best);
    if (lane() == 0 && best != kNone) atomicMin(&a.ctl->cand[par ^ 1].v[0], best);
  }
  if (p.gtid == 0) {
    if (nS > 0) unstable_set(a, C);
    if (!L) {
      if (nS > 0) atomicMin(&a.ctl->cand[par ^ 1].v[0], C);
      a.ctl->cand[par].v[0] = kNone;
    }
    if (a.trace_nsplit && k < a.trace_cap) a.trace_nsplit[k] = nS;
    if (a.trace_work && k < a.trace_cap) {
      int64_t* w = a.trace_work + 4 * (uint64_t)k;
      w[0] = a.ctl->work[par].v[0];
      w[1] = a.ctl->work[par].v[1];
      w[2] = nT;
      w[3] = a.ctl->ltany[par].v[0];
    }
  }
}

// ---------------------------------------------------------------------------
// Plain policy in two grid-wide steps per iteration.  The relabel of
// iteration k-1 is folded into iteration k's scan of block[]: a state whose
// split flag (k-1) is set takes the label its old block elected, read from
// the epoch-tagged bid (epoch k); the owner of the state writes it back, and
// every other reader in the same step applies the same rule, which gives the
// same answer whether or not the write-back has happened (a new label never
// carries a bid of epoch k).  The next splitter is known without the new
// leaders: each is larger than its block's old label, which becomes unstable
// in the same iteration.  Marks, touched lists and split flags alternate
// between two halves by iteration parity, so the step that needs a half
// clean clears what the iteration before last left in it.
//   X(k): head; relabel k-1's splits (new leaders min-reduced into the next
//         candidate and listed); re-mark the previous splitter if anything
//         split; clear C, search the next smallest unstable label; mark
//         (marks, touched and leader-touched bits; no lists).
//   Y(k): one pass over all states: compare touched states with their
//         leader, untouched members of leader-touched blocks split; elect;
//         split flags; old labels become unstable and, with C if anything
//         split, are min-reduced into the next candidate; k-1's marks are
//         cleared in the same pass; k-1's new leaders become unstable.
// ---------------------------------------------------------------------------
struct FPar {  // the half of iteration parity `par`
  uint64_t* mw;
  uint64_t* tb;
  uint64_t* lt;
  uint64_t* sb;
};
__device__ __forceinline__ FPar fpar(const Args& a, uint32_t par) {
  const size_t nwd = ((uint32_t)a.n + 63u) >> 6;
  return {a.mw + par * a.nwords, a.tb + par * nwd, a.lt + par * nwd, a.sb + par * nwd};
}

// label of s during iteration k: block[s], or its block's elected leader if s
// split in iteration k-1 and the write-back has not happened yet
__device__ __forceinline__ int32_t lazy_label(const Args& a, const uint64_t* prev_sb, uint32_t s,
                                              uint32_t k) {
  const int32_t b = a.block[s];
  if (!test_bit(prev_sb, s)) return b;
  const uint64_t v = a.nlw[b];
  return (uint32_t)(v >> 32) == k ? (int32_t)(kNone - (uint32_t)v) : b;
}

__device__ uint32_t head2(const Args& a, uint32_t k, const Part& p, uint32_t C) {
  const bool over = (k + 1 > a.iter_cap);
  if (p.gtid == 0) {
    Ctl* c = a.ctl;
    if (k > 0 && k - 1 < a.trace_cap) {  // iteration k-1's counters are final now
      const uint32_t q = (k - 1) % 3;
      if (a.trace_nsplit) a.trace_nsplit[k - 1] = c->fS[q].v[0];
      if (a.trace_work) {
        int64_t* w = a.trace_work + 4 * (uint64_t)(k - 1);
        w[0] = c->fW[q].v[0];
        w[1] = c->fW[q].v[1];
        w[2] = c->fW[q].v[2];
        w[3] = c->fL[q].v[0];
      }
    }
    if (C == kNone || over) {
      c->state.v[0] = k + 1;
      c->state.v[1] = 1;
      if (over && C != kNone) c->state.v[2] = 1;
      if (a.trace_C && k < a.trace_cap) a.trace_C[k] = -1;
      if (a.trace_nsplit && k < a.trace_cap) a.trace_nsplit[k] = 0;
      if (a.trace_work && k < a.trace_cap)
        for (int q = 0; q < 4; ++q) a.trace_work[4 * (uint64_t)k + q] = 0;
    } else {
      const uint32_t q = (k + 1) % 3;  // last used by iteration k-2
      c->state.v[3] = C;
      c->fC[k % 3].v[0] = C;
      c->fS[q].v[0] = 0;
      c->fL[q].v[0] = 0;
      c->fW[q].v[0] = 0;
      c->fW[q].v[1] = 0;
      c->fW[q].v[2] = 0;
      c->fN[q].v[0] = 0;
      if (a.trace_C && k < a.trace_cap) a.trace_C[k] = (int32_t)C;
    }
  }
  return (C == kNone || over) ? kNone : C;
}
__device__ uint32_t head2(const Args& a, uint32_t k, const Part& p) {
  return head2(a, k, p, a.ctl->cand[k & 1].v[0]);
}

// chunks of 64 states per wave and step of the two-step engine's scans; all
// their loads are issued before any is used
constexpr uint32_t kFusedU = 2;

// The loads of a wave's first scan step, which depend on nothing the step
// computes: the per-phase kernels issue them at entry, beside the control
// block's, so that they are not one more round trip on the kernel's chain.
struct XChunk {
  int32_t bv[kFusedU];  // block[] of the chunk's states
  uint64_t fw[kFusedU]; // their split flags of the previous iteration
};
// chunks per wave and step of X: the combining variant takes one, so that
// twice as many waves share the marks of a large splitter
template <bool Agg>
constexpr uint32_t x_chunks() {
  return Agg ? 1u : kFusedU;
}
template <uint32_t U>
__device__ __forceinline__ void load_xchunk(const Args& a, uint32_t k, uint32_t base0,
                                            XChunk& c) {
  const uint32_t n = (uint32_t)a.n;
  const uint64_t* prv_sb = fpar(a, (k & 1) ^ 1).sb;
#pragma unroll
  for (uint32_t u = 0; u < U; ++u) {
    const uint32_t base = base0 + u * kWave, t = base + lane();
    c.bv[u] = t < n ? a.block[t] : -1;
    c.fw[u] = base < n ? prv_sb[base >> 6] : 0ull;
  }
}
struct YChunk {
  int32_t bv[kFusedU];  // block[] of the chunk's states
  uint64_t tw[kFusedU]; // touched bits of this iteration
  uint64_t pw[kFusedU]; // touched bits of the previous one (marks to clear)
};
__device__ __forceinline__ void load_ychunk(const Args& a, uint32_t k, uint32_t base0,
                                            YChunk& c) {
  const uint32_t n = (uint32_t)a.n;
  const uint64_t* ctb = fpar(a, k & 1).tb;
  const uint64_t* ptb = fpar(a, (k & 1) ^ 1).tb;
#pragma unroll
  for (uint32_t u = 0; u < kFusedU; ++u) {
    const uint32_t base = base0 + u * kWave, s = base + lane();
    c.bv[u] = s < n ? a.block[s] : 0;
    c.tw[u] = base < n ? ctb[base >> 6] : 0ull;
    c.pw[u] = base < n ? ptb[base >> 6] : 0ull;
  }
}

// Marks of source s (slots `bits` of its word wi): the mark word, and the
// touched-leader bit when s leads its block.  Every atomic is fire-and-forget
// (the touched set is the tb bitmap, read back by the next step's scan).
__device__ __forceinline__ void mark_word(const Args& a, const FPar& cur, const uint64_t* prev_sb,
                                          uint32_t slot, uint32_t k, int32_t s, uint64_t wi,
                                          uint64_t bits) {
  const int32_t bl = a.block[s];
  const bool flagged = test_bit(prev_sb, (uint32_t)s);
  atomicOr((unsigned long long*)&cur.mw[wi], (unsigned long long)bits);
  int32_t lab = bl;  // lazy_label, with its loads issued before the atomic
  if (flagged) {
    const uint64_t v = a.nlw[bl];
    if ((uint32_t)(v >> 32) == k) lab = (int32_t)(kNone - (uint32_t)v);
  }
  if (lab == s) {  // a touched leader
    atomicOr((unsigned long long*)&cur.lt[s >> 6], 1ull << (s & 63));
    a.ctl->fL[slot].v[0] = 1;
  }
}

__device__ __forceinline__ void mark_state(const Args& a, const FPar& cur, const uint64_t* prev_sb,
                                           uint32_t slot, uint32_t k, int32_t s, uint64_t wi,
                                           uint64_t bits) {
  mark_word(a, cur, prev_sb, slot, k, s, wi, bits);
  atomicOr((unsigned long long*)&cur.tb[s >> 6], 1ull << (s & 63));
}

__device__ __forceinline__ uint64_t wave_or_u64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v |= (uint64_t)__shfl_xor((unsigned long long)v, d, kWave);
  return v;
}

// Set the touched bits of the sources of the lanes with `pend` (wave-uniform
// call).  When lanes share a bitmap word with the first such lane (sources
// that are neighbours, like a chain's), the words of the first two groups
// take one atomic each: consecutive words sit in few memory channels, where
// one atomic per lane would queue.
__device__ __forceinline__ void touch_lanes(const FPar& cur, int32_t s, bool pend) {
  const uint64_t pb0 = __ballot(pend);
  if (!pb0) return;
  const uint32_t w = (uint32_t)s >> 6;
  const uint32_t wf = (uint32_t)__shfl((int)w, __ffsll((unsigned long long)pb0) - 1, kWave);
  if (__popcll(__ballot(pend && w == wf)) > 1) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const uint64_t pb = __ballot(pend);
      if (!pb) return;
      const int f = __ffsll((unsigned long long)pb) - 1;
      const uint32_t w0 = (uint32_t)__shfl((int)w, f, kWave);
      const bool mine = pend && w == w0;
      const uint64_t bits = wave_or_u64(mine ? 1ull << (s & 63) : 0ull);
      if ((int)lane() == f) atomicOr((unsigned long long*)&cur.tb[w0], (unsigned long long)bits);
      pend = pend && !mine;
    }
  }
  if (pend) atomicOr((unsigned long long*)&cur.tb[w], 1ull << (s & 63));
}

// Per-workgroup table of sources whose marks are combined in LDS and written
// once, after the workgroup's last chunk.  The combining marking runs on LTSs
// with a state of at least kHotDegree outgoing transitions (one such state
// can fill a wave with the same source); elsewhere each lane marks its own.
constexpr int kHot = 4;
constexpr uint32_t kHotDegree = 64;
struct HotTab {
  int32_t* s;             // [kHot] source, -1 while free
  unsigned long long* b;  // [kHot] its slot bits
};

// Mark the transitions held by the lanes of a wave when a state's slots may
// span several words (valid lanes: source s, action rank o; wave-uniform
// call): one mark atomic per lane, touched bits combined per word.
__device__ __forceinline__ void mark_lanes_wide(const Args& a, const FPar& cur,
                                                const uint64_t* prev_sb, uint32_t slot, uint32_t k,
                                                int32_t s, int32_t o, bool valid) {
  if (valid)
    mark_word(a, cur, prev_sb, slot, k, s, (uint64_t)a.woff[s] + (uint32_t)(o >> 6),
              1ull << (o & 63));
  touch_lanes(cur, s, valid);
}

// Transition index of entry ee of a wave's in-transition list, whose lane l
// owns entries [incl_l - deg_l, incl_l) starting at in_ptr position beg_l
// (wave-uniform call: shuffles only).
__device__ __forceinline__ uint32_t edge_of(uint32_t incl, uint32_t beg, uint32_t deg,
                                            uint32_t ee) {
  uint32_t j = 0;  // owner lane: the first with incl > ee
#pragma unroll
  for (uint32_t step = 32; step >= 1; step >>= 1) {
    const uint32_t probe = (uint32_t)__shfl((int)incl, (int)(j + step - 1), kWave);
    if (probe <= ee) j += step;
  }
  const uint32_t jb = (uint32_t)__shfl((int)beg, (int)j, kWave);
  const uint32_t ji = (uint32_t)__shfl((int)incl, (int)j, kWave);
  const uint32_t jd = (uint32_t)__shfl((int)deg, (int)j, kWave);
  return jb + (ee - (ji - jd));
}

// Combining of recurring sources: lanes of the wave's first two
// sources, when the first recurs, go to the workgroup's table; returns
// whether this lane is still to be marked (wave-uniform call).
__device__ __forceinline__ bool take_recurring(const Args& a, const FPar& cur,
                                               const uint64_t* prev_sb, uint32_t slot, uint32_t k,
                                               int32_t s, int32_t o, bool valid, const HotTab& ht) {
  const uint64_t vb = __ballot(valid);
  if (!vb) return false;
  const int32_t sf = __shfl(s, __ffsll((unsigned long long)vb) - 1, kWave);
  bool pending = valid;
  if (__popcll(__ballot(valid && s == sf)) <= 1) return pending;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const uint64_t pb = __ballot(pending);
    if (!pb) break;
    const int f = __ffsll((unsigned long long)pb) - 1;
    const int32_t s0 = __shfl(s, f, kWave);
    const bool mine = pending && s == s0;
    const uint64_t bits = wave_or_u64(mine ? 1ull << (o & 63) : 0ull);
    if ((int)lane() == f) {
      bool put = false;
      for (int i = 0; i < kHot && !put; ++i) {
        const int32_t old = atomicCAS(&ht.s[i], -1, s0);
        if (old == -1 || old == s0) {
          atomicOr(&ht.b[i], (unsigned long long)bits);
          put = true;
        }
      }
      if (!put) mark_state(a, cur, prev_sb, slot, k, s0, (uint64_t)s0, bits);
    }
    pending = pending && !mine;
  }
  return pending;
}

// The combining marking of a chunk's in-transitions (uniform layout): up to
// kRounds wave-rounds at a time, with every load of the group (sources,
// ranks, labels) issued before any of its atomics.  On CDNA a load waits for
// the wave's earlier memory operations, atomics included, so marking round by
// round would put a full memory round trip per round on the wave's chain,
// and a large splitter gives a wave many rounds (wave-uniform call).
constexpr uint32_t kRounds = 4;
__device__ __forceinline__ void mark_rounds(const Args& a, const FPar& cur, const uint64_t* prev_sb,
                                            uint32_t slot, uint32_t k, uint32_t incl,
                                            uint32_t beg, uint32_t deg, uint32_t total,
                                            const HotTab& ht) {
  for (uint32_t e0 = 0; e0 < total; e0 += kWave * kRounds) {
    int32_t s[kRounds], o[kRounds], lab[kRounds];
    bool pend[kRounds], fl[kRounds];
#pragma unroll
    for (uint32_t g = 0; g < kRounds; ++g) {
      s[g] = 0;
      o[g] = 0;
      pend[g] = false;
      const uint32_t eg = e0 + g * kWave;
      if (eg >= total) continue;  // wave-uniform
      const uint32_t e = eg + lane();
      const bool valid = e < total;
      const uint32_t edge = edge_of(incl, beg, deg, valid ? e : total - 1);
      if (valid) {
        s[g] = a.in_src[edge];
        o[g] = a.in_ord[edge];
      }
      pend[g] = valid;
    }
#pragma unroll
    for (uint32_t g = 0; g < kRounds; ++g)
      if (e0 + g * kWave < total)
        pend[g] = take_recurring(a, cur, prev_sb, slot, k, s[g], o[g], pend[g], ht);
#pragma unroll
    for (uint32_t g = 0; g < kRounds; ++g) {
      lab[g] = pend[g] ? a.block[s[g]] : -1;
      fl[g] = pend[g] && test_bit(prev_sb, (uint32_t)s[g]);
    }
#pragma unroll
    for (uint32_t g = 0; g < kRounds; ++g) {
      if (fl[g]) {  // lazy_label
        const uint64_t v = a.nlw[lab[g]];
        if ((uint32_t)(v >> 32) == k) lab[g] = (int32_t)(kNone - (uint32_t)v);
      }
    }
#pragma unroll
    for (uint32_t g = 0; g < kRounds; ++g) {
      if (pend[g]) {
        atomicOr((unsigned long long*)&cur.mw[s[g]], 1ull << (o[g] & 63));
        if (lab[g] == s[g]) {  // a touched leader
          atomicOr((unsigned long long*)&cur.lt[s[g] >> 6], 1ull << (s[g] & 63));
          a.ctl->fL[slot].v[0] = 1;
        }
      }
      if (e0 + g * kWave < total) touch_lanes(cur, s[g], pend[g]);
    }
  }
}

template <bool Agg>
__device__ void phase_x(const Args& a, uint32_t k, uint32_t C, const Part& p,
                        const XChunk* first = nullptr) {
  const uint32_t par = k & 1, slot = k % 3;
  const FPar cur = fpar(a, par), prv = fpar(a, par ^ 1);
  uint32_t* cand = &a.ctl->cand[par ^ 1].v[0];
  const uint32_t n = (uint32_t)a.n, nwd = (n + 63u) >> 6;
  __shared__ int32_t hot_s[kHot];
  __shared__ unsigned long long hot_b[kHot];
  const HotTab ht{hot_s, hot_b};
  if (Agg) {
    if (threadIdx.x < (uint32_t)kHot) {
      hot_s[threadIdx.x] = -1;
      hot_b[threadIdx.x] = 0;
    }
    __syncthreads();
  }
  if (p.gwave == p.gwaves - 1) {  // clear C, search the next smallest unstable label
    // (on the last wave, which has the least scan work; the previous splitter
    // is unstable again if anything split, unless it is C itself; it is
    // folded in here, where nothing else writes the set)
    // all loads that do not depend on each other first: the previous
    // splitter's slots, C's word and the first window of summary words
    const uint32_t w0 = C >> 6;
    const uint32_t from = (k == 0) ? 0u : w0;  // a forced first splitter need not be the smallest
    const uint32_t nsw = (nwd + 63u) >> 6;
    const uint32_t q0 = from >> 6;
    const uint32_t fs1 = k > 0 ? a.ctl->fS[(k - 1) % 3].v[0] : 0u;
    const uint32_t fc1 = k > 0 ? a.ctl->fC[(k - 1) % 3].v[0] : kNone;
    const uint64_t ubw = a.ub[w0];
    const uint64_t sv0 = q0 + lane() < nsw ? a.us[q0 + lane()] : 0ull;
    uint32_t pc = kNone;
    if (k > 0 && !a.rcpp && fs1 != 0) pc = fc1;
    if (pc == C) pc = kNone;
    uint64_t bits = ubw & ~(1ull << (C & 63));
    if (pc != kNone && (pc >> 6) == w0) bits |= 1ull << (pc & 63);
    if (lane() == 0) {
      a.ub[w0] = bits;
      if (bits == 0) atomicAnd((unsigned long long*)&a.us[w0 >> 6], ~(1ull << (w0 & 63)));
      if (pc != kNone && (pc >> 6) != w0) {
        atomicOr((unsigned long long*)&a.ub[pc >> 6], 1ull << (pc & 63));
        atomicOr((unsigned long long*)&a.us[pc >> 12], 1ull << ((pc >> 6) & 63));
      }
    }
    uint32_t next = kNone;
    for (uint32_t q = q0; q < nsw; q += kWave) {
      const uint32_t qq = q + lane();
      uint64_t sv = q == q0 ? sv0 : (qq < nsw ? a.us[qq] : 0ull);
      if (qq == (from >> 6)) sv &= ~0ull << (from & 63);
      if (qq == (w0 >> 6)) {
        const uint64_t b0 = 1ull << (w0 & 63);
        sv = bits ? (sv | b0) : (sv & ~b0);
      }
      const uint64_t bal = __ballot(sv != 0);
      if (bal) {
        const int l = __ffsll((unsigned long long)bal) - 1;
        const uint64_t v = (uint64_t)__shfl((unsigned long long)sv, l, kWave);
        const uint32_t word = ((q + (uint32_t)l) << 6) + (uint32_t)(__ffsll((unsigned long long)v) - 1);
        const uint64_t wb = (word == w0) ? bits : a.ub[word];
        if (wb) next = (word << 6) + (uint32_t)(__ffsll((unsigned long long)wb) - 1);
        break;
      }
    }
    if (pc < next) next = pc;  // its bit may not be visible to this search yet
    if (lane() == 0 && next != kNone) atomicMin(cand, next);
  }
  constexpr uint32_t U = x_chunks<Agg>();
  const uint32_t b00 = p.gwave * kWave * U;
  for (uint32_t base0 = b00; base0 < n; base0 += p.gwaves * kWave * U) {
    XChunk ch;
    if (first && base0 == b00)
      ch = *first;
    else
      load_xchunk<U>(a, k, base0, ch);
#pragma unroll
    for (uint32_t u = 0; u < U; ++u) {
      const uint32_t base = base0 + u * kWave, t = base + lane();
      int32_t lab = ch.bv[u];
      bool lead = false;
      if (t < n && ((ch.fw[u] >> lane()) & 1ull)) {  // split in k-1: relabel now
        const uint64_t v = a.nlw[lab];
        if ((uint32_t)(v >> 32) == k) {
          lab = (int32_t)(kNone - (uint32_t)v);
          a.block[t] = lab;
          lead = (lab == (int32_t)t);
        }
      }
      if (base < n && lane() == 0) cur.sb[base >> 6] = 0;  // k-2's flags; Y(k) writes k's
      if (__ballot(lead)) {
        wave_push(a.nlist, &a.ctl->fN[slot].v[0], (int32_t)t, lead);
        const uint32_t mn = wave_min_u32(lead ? t : kNone);
        if (lane() == 0) atomicMin(cand, mn);
      }
      const bool hit = (uint32_t)lab == C;
      const uint64_t hits = __ballot(hit);
      if (hits == 0) continue;
      uint32_t beg = 0, deg = 0;
      if (hit) {
        beg = a.in_ptr[t];
        deg = a.in_ptr[t + 1] - beg;
      }
      const uint32_t incl = wave_incl_scan_u32(deg);
      const uint32_t total = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
      if (a.trace_work && lane() == 0) {
        atomicAdd(&a.ctl->fW[slot].v[0], (uint32_t)__popcll(hits));
        atomicAdd(&a.ctl->fW[slot].v[1], total);
      }
      if (Agg && a.uniform) {
        mark_rounds(a, cur, prv.sb, slot, k, incl, beg, deg, total, ht);
        continue;
      }
      for (uint32_t e0 = 0; e0 < total; e0 += kWave) {
        const uint32_t e = e0 + lane();
        const bool valid = e < total;
        const uint32_t edge = edge_of(incl, beg, deg, valid ? e : total - 1);
        int32_t s = 0, o = 0;
        if (valid) {
          s = a.in_src[edge];
          o = a.in_ord[edge];
        }
        if (Agg) {
          mark_lanes_wide(a, cur, prv.sb, slot, k, s, o, valid);
        } else if (valid) {
          mark_state(a, cur, prv.sb, slot, k, s,
                     a.uniform ? (uint64_t)s : (uint64_t)a.woff[s] + (uint32_t)(o >> 6),
                     1ull << (o & 63));
        }
      }
    }
  }
  if (!Agg) return;
  __syncthreads();  // write the workgroup's combined marks
  if (threadIdx.x < (uint32_t)kHot && hot_s[threadIdx.x] >= 0)
    mark_state(a, cur, prv.sb, slot, k, hot_s[threadIdx.x], (uint64_t)hot_s[threadIdx.x],
               hot_b[threadIdx.x]);
}

// Split states s = base + lane of one 64-state chunk of Y's scan (wave-uniform
// call; b = block[s]).  Atomics are aggregated per wave: one split-flag word,
// and one bid for the block of the first split lane (usually the only block:
// a large block that loses most of its states bids from every wave of the
// scan), with a read first so that later, larger bids are skipped.
__device__ __forceinline__ void split2(const Args& a, const FPar& cur, uint32_t slot, uint32_t par,
                                       uint32_t C, uint32_t base, int32_t b, bool sp,
                                       uint64_t epoch) {
  const uint64_t bal = __ballot(sp);
  if (!bal) return;
  const uint32_t s = base + lane();
  const int first = __ffsll((unsigned long long)bal) - 1;
  const int32_t b0 = __shfl(b, first, kWave);
  const uint32_t m0 = wave_min_u32(sp && b == b0 ? s : kNone);
  if ((int)lane() == first) {
    const uint64_t v = epoch | (uint64_t)(kNone - m0);
    if (__hip_atomic_load(&a.nlw[b0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < v)
      atomicMax((unsigned long long*)&a.nlw[b0], (unsigned long long)v);
    atomicOr((unsigned long long*)&cur.sb[base >> 6], (unsigned long long)bal);
  }
  if (sp && b != b0)
    atomicMax((unsigned long long*)&a.nlw[b],
              (unsigned long long)(epoch | (uint64_t)(kNone - s)));
  if (sp) {  // old label unstable (sets only in this step)
    const uint32_t w = (uint32_t)b >> 6;
    if (!((a.ub[w] >> (b & 63)) & 1ull)) {
      atomicOr((unsigned long long*)&a.ub[w], 1ull << (b & 63));
      atomicOr((unsigned long long*)&a.us[w >> 6], 1ull << (w & 63));
    }
  }
  const uint32_t mb = wave_min_u32(sp ? (uint32_t)b : kNone);
  if (lane() == 0) {
    atomicAdd(&a.ctl->fS[slot].v[0], (uint32_t)__popcll(bal));
    // anything split: C is a candidate again (its unstable bit is set by
    // the next step's selection) -- not in Algorithm 2
    atomicMin(&a.ctl->cand[par ^ 1].v[0], (mb < C || a.rcpp) ? mb : C);
  }
}

// Y(k): one pass over all states.  A touched state (tb) splits iff its marks
// differ from its leader's; an untouched one iff its leader was touched (lt).
// The same pass clears what iteration k-1 left in the other half.
__device__ void phase_y(const Args& a, uint32_t k, const Part& p, uint32_t C,
                        const YChunk* first = nullptr) {
  const uint32_t par = k & 1, slot = k % 3;
  const FPar cur = fpar(a, par), prv = fpar(a, par ^ 1);
  const uint64_t epoch = (uint64_t)(k + 1) << 32;
  const uint32_t n = (uint32_t)a.n;
  const uint32_t b00 = p.gwave * kWave * kFusedU;
  for (uint32_t base0 = b00; base0 < n; base0 += p.gwaves * kWave * kFusedU) {
    YChunk ch;
    if (first && base0 == b00)
      ch = *first;
    else
      load_ychunk(a, k, base0, ch);
    const int32_t* bv = ch.bv;
    const uint64_t* tw = ch.tw;
    const uint64_t* pw = ch.pw;
#pragma unroll
    for (uint32_t u = 0; u < kFusedU; ++u) {
      const uint32_t base = base0 + u * kWave, s = base + lane();
      const int32_t b = bv[u];
      const bool touched = (tw[u] >> lane()) & 1ull;
      bool sp = false;
      if (s < n) {
        if (touched) {
          if ((int32_t)s != b) {
            if (a.uniform) {
              sp = cur.mw[s] != cur.mw[b];
            } else {
              const uint32_t w0 = a.woff[s], w1 = a.woff[s + 1], wb = a.woff[b];
              for (uint32_t q = 0; q < w1 - w0; ++q)
                if (cur.mw[w0 + q] != cur.mw[wb + q]) {
                  sp = true;
                  break;
                }
            }
          }
        } else {
          sp = test_bit(cur.lt, (uint32_t)b);
        }
      }
      split2(a, cur, slot, par, C, base, b, sp, epoch);
      if (a.trace_work && lane() == 0 && tw[u])
        atomicAdd(&a.ctl->fW[slot].v[2], (uint32_t)__popcll(tw[u]));
      if (pw[u]) {  // iteration k-1's marks in this chunk
        if ((pw[u] >> lane()) & 1ull) {
          if (a.uniform) {
            prv.mw[s] = 0;
          } else {
            for (uint32_t q = a.woff[s]; q < a.woff[s + 1]; ++q) prv.mw[q] = 0;
          }
        }
        if (lane() == 0) {
          prv.tb[base >> 6] = 0;
          prv.lt[base >> 6] = 0;
        }
      }
    }
  }
  const uint32_t nN = a.ctl->fN[slot].v[0];  // new leaders of k-1
  for (uint32_t i = p.gtid; i < nN; i += p.gthreads) {
    const uint32_t t = (uint32_t)a.nlist[i], w = t >> 6;
    atomicOr((unsigned long long*)&a.ub[w], 1ull << (t & 63));
    atomicOr((unsigned long long*)&a.us[w >> 6], 1ull << (w & 63));
  }
  if (p.gtid == 0) a.ctl->cand[par].v[0] = kNone;  // read by X(k); reused by iteration k+2
}

// S (learned policy, one workgroup): re-score the labels that changed in this
// iteration (both labels of every split block, and C, whose "used" feature
// changed), move them between levels (all removals before all insertions, so
// the summaries stay exact), then pick the next splitter: the smallest label
// of the highest non-empty level.
__device__ void phase_s(const Args& a, const MlpLds& M, uint32_t par, uint32_t k) {
  const uint32_t nC = a.ctl->cntC[par].v[0];
  const uint32_t C = a.ctl->state.v[3];
  const uint32_t ne = 2 * nC + 1;
  const uint32_t wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
  for (uint32_t q = wid; q < ne; q += nw) {
    const uint32_t b = q < 2 * nC ? (uint32_t)a.chg[q] : C;
    const uint32_t lv = test_bit(a.ub, b) ? block_level(a, M, b, k + 1) : 0xFFu;
    if (lane() == 0) {
      lv_remove(a, b, a.lvl[b]);
      a.lvq[q] = (uint8_t)lv;
    }
  }
  __syncthreads();
  for (uint32_t q = threadIdx.x; q < ne; q += blockDim.x) {
    const uint32_t b = q < 2 * nC ? (uint32_t)a.chg[q] : C;
    const uint32_t lv = a.lvq[q];
    if (lv != 0xFFu) {
      lv_insert(a, b, lv);
      a.lvl[b] = (uint8_t)lv;
    }
  }
  __syncthreads();
  if (wid == 0) {
    const uint32_t nx = lv_search(a);
    if (lane() == 0) {
      a.ctl->cand[par ^ 1].v[0] = nx == kNone - 1 ? kNone : nx;
      if (nx == kNone - 1) a.ctl->state.v[4] = 1;
    }
  }
}

// Full re-scoring (every R iterations, before S): new levels of all unstable
// labels, and an empty structure (F1); then every unstable label inserted at
// its level (F2).
__device__ void phase_f1(const Args& a, const MlpLds& M, uint32_t kcur, const Part& p) {
  const LvDims d = lv_dims(a);
  for (uint32_t i = p.gtid; i < kLevels * d.nwd; i += p.gthreads) a.lvb[i] = 0;
  for (uint32_t i = p.gtid; i < kLevels * d.nsw; i += p.gthreads) a.lvs[i] = 0;
  for (uint32_t i = p.gtid; i < kLevels * d.ntw; i += p.gthreads) a.lvt[i] = 0;
  for (uint32_t w = p.gwave; w < d.nwd; w += p.gwaves) {
    uint64_t bits = a.ub[w];
    while (bits) {
      const uint32_t b = (w << 6) + (uint32_t)(__ffsll((unsigned long long)bits) - 1);
      bits &= bits - 1;
      const uint32_t lv = block_level(a, M, b, kcur);
      if (lane() == 0) a.lvl[b] = (uint8_t)lv;
    }
  }
}
__device__ void phase_f2(const Args& a, const Part& p) {
  const uint32_t nwd = ((uint32_t)a.n + 63u) >> 6;
  for (uint32_t w = p.gtid; w < nwd; w += p.gthreads) {
    uint64_t bits = a.ub[w];
    while (bits) {
      const uint32_t b = (w << 6) + (uint32_t)(__ffsll((unsigned long long)bits) - 1);
      bits &= bits - 1;
      lv_insert(a, b, a.lvl[b]);
    }
  }
}

// ---------------------------------------------------------------------------
// per-run initialisation
// ---------------------------------------------------------------------------
__global__ void k_init_run(Args a, const int32_t* __restrict__ pre, uint32_t first,
                           uint64_t nwords, uint32_t learned) {
  const Part p = part();
  const uint32_t n = (uint32_t)a.n;
  for (uint32_t s = p.gtid; s < n; s += p.gthreads) {
    a.block[s] = pre[s];
    a.nlw[s] = 0;
  }
  for (uint64_t w = p.gtid; w < 2 * nwords; w += p.gthreads) a.mw[w] = 0;
  const uint32_t nwd = (n + 63u) >> 6;
  for (uint32_t w = p.gtid; w < nwd; w += p.gthreads) {
    uint64_t bits = 0;
    const uint32_t s0 = w << 6;
    for (uint32_t j = 0; j < 64 && s0 + j < n; ++j)
      if ((uint32_t)pre[s0 + j] == s0 + j) bits |= 1ull << j;
    a.ub[w] = bits;
    a.tb[w] = a.tb[nwd + w] = 0;
    a.lt[w] = a.lt[nwd + w] = 0;
    a.sb[w] = a.sb[nwd + w] = 0;
  }
  if (blockIdx.x == 0) {
    uint32_t* c = reinterpret_cast<uint32_t*>(a.ctl);
    for (uint32_t i = threadIdx.x; i < sizeof(Ctl) / 4; i += blockDim.x) c[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
      a.ctl->cand[0].v[0] = (n == 0 || learned) ? kNone : first;
      a.ctl->cand[1].v[0] = kNone;
    }
  }
}

// summary level of the unstable bitmap (after k_init_run has written ub)
__global__ void k_init_summary(Args a) {
  const Part p = part();
  const uint32_t nwd = ((uint32_t)a.n + 63u) >> 6;
  const uint32_t nsw = (nwd + 63u) >> 6;
  for (uint32_t q = p.gtid; q < nsw; q += p.gthreads) {
    uint64_t bits = 0;
    for (uint32_t j = 0; j < 64 && (q << 6) + j < nwd; ++j)
      if (a.ub[(q << 6) + j]) bits |= 1ull << j;
    a.us[q] = bits;
  }
}

__global__ void k_zero_features(Args a) {
  const Part p = part();
  const uint64_t n = (uint32_t)a.n;
  for (uint64_t i = p.gtid; i < 17 * n; i += p.gthreads) a.acc[i] = 0;
  for (uint64_t i = p.gtid; i < n; i += p.gthreads) {
    a.born[i] = 0;
    a.used[i] = 0;
    if (a.lvl) a.lvl[i] = 0;
  }
}
__global__ void k_accumulate_features(Args a, const int32_t* __restrict__ pre) {
  const Part p = part();
  for (uint32_t s = p.gtid; s < (uint32_t)a.n; s += p.gthreads) {
    const size_t b = (size_t)pre[s];
    atomicAdd(&a.acc[b * 17], 1u);
    for (int q = 0; q < 16; ++q) {
      const uint32_t v = a.sfeat[(size_t)s * 16 + q];
      if (v) atomicAdd(&a.acc[b * 17 + 1 + q], v);
    }
  }
}
// learned policy: levels of all unstable labels (F1, F2) and the splitter of
// the first iteration
__global__ void k_levels_all(Args a, uint32_t kcur) {
  extern __shared__ float sw[];
  MlpLds M = mlp_lds_layout(sw, kPolicyF);
  mlp_stage(M, a.wbf, kPolicyF);
  __syncthreads();
  phase_f1(a, M, kcur, part());
}
__global__ void k_levels_insert(Args a) { phase_f2(a, part()); }
__global__ void k_learned_first(Args a) {
  if (threadIdx.x >= kWave) return;
  const uint32_t nx = lv_search(a);
  if (lane() == 0) {
    a.ctl->cand[0].v[0] = nx == kNone - 1 ? kNone : nx;
    if (nx == kNone - 1) a.ctl->state.v[4] = 1;
  }
}

__global__ void k_count_leaders(const int32_t* __restrict__ block, int32_t n,
                                unsigned long long* out) {
  const Part p = part();
  uint32_t c = 0;
  for (uint32_t s = p.gtid; s < (uint32_t)n; s += p.gthreads) c += (block[s] == (int32_t)s);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) c += (uint32_t)__shfl_xor((int)c, d, kWave);
  if (lane() == 0 && c) atomicAdd(out, (unsigned long long)c);
}

}  // namespace
}  // namespace bisim
