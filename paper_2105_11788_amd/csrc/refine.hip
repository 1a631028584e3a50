// The refinement loop of the labelled PRAM algorithm (Algorithm 3, section 4),
// as three data-parallel phases per iteration with a grid-wide dependency
// between them (the paper's GPU port also needs synchronisation points after
// the mark and the leader election; section 5):
//
//   A  select + mark    C is the smallest unstable block label (priority
//                       CRCW, computed as a min-reduction in the previous
//                       iteration).  Clear C's unstable bit; min-reduce the
//                       remaining unstable labels into the next iteration's
//                       candidate; for every state t with block[t] == C visit
//                       t's in-transitions (source s, action rank o) and set
//                       mark slot o of s.  The first touch of a state appends
//                       it to the touched list T; a touched leader sets its
//                       bit in the leader-touched bitmap.
//   B  compare + elect  A state splits iff its marks differ from its
//                       leader's.  Only two kinds of state can differ:
//                       touched states (compared word by word), and untouched
//                       members of blocks whose leader was touched (their
//                       marks are all zero, the leader's are not).  Each
//                       split state bids (epoch, ~s) with a 64-bit atomic max
//                       on new_leader[block], so the smallest state wins and
//                       stale bids of earlier iterations lose without a reset.
//   C  relabel          block[s] := new_leader[block[s]] for split states; the
//                       new leader marks its old and new block unstable, and
//                       C is re-marked unstable if anything split.  New
//                       unstable labels are min-reduced into the candidate.
//                       Marks and touched bits of T are cleared.
//
// Marks: each state's slots (one per distinct outgoing action, section 4.1)
// are bits of 64-bit words; with <= 64 actions per state the word index is
// the state itself.  The paper's "mark[off(s) + order_i]" is bit order_i of
// word off64(s) + order_i / 64.
//
// Engines: (1) one cooperative launch whose workgroups run all iterations,
// separated by grid barriers (agent-scope release/acquire, so the 8 XCDs'
// L2s see each other's writes); (2) one kernel per phase, enqueued in
// batches with a device-side done flag, where kernel boundaries are the
// barriers.
#include "internal.h"

namespace bisim {

namespace {
constexpr int kT = 256;            // per-phase kernels
constexpr int kPT = 512;           // persistent kernel
constexpr uint64_t kBarrierTimeoutTicks = 10ull * 100000000ull;  // 10 s at 100 MHz

struct Args {
  int32_t n;
  int uniform;
  const uint32_t* __restrict__ in_ptr;
  const int32_t* __restrict__ in_src;
  const int32_t* __restrict__ in_ord;
  const uint32_t* __restrict__ woff;
  int32_t* block;
  uint64_t* mw;
  uint64_t* tb;
  uint64_t* lt;
  uint64_t* ub;
  uint64_t* nlw;
  int32_t* tlist;
  int32_t* slist;
  Ctl* ctl;
  uint32_t iter_cap;
  int32_t* trace_C;
  int64_t* trace_nsplit;
  int64_t* trace_work;
  uint32_t trace_cap;
};

struct Part {
  uint32_t gtid, gthreads, gwave, gwaves;
};

__device__ __forceinline__ Part part() {
  const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t gthreads = gridDim.x * blockDim.x;
  return {gtid, gthreads, gtid / kWave, gthreads / kWave};
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
      c->state.v[3] = C;
      c->cntT[(k & 1) ^ 1].v[0] = 0;
      c->cntS[(k & 1) ^ 1].v[0] = 0;
      c->ltany[(k & 1) ^ 1].v[0] = 0;
      c->work[(k & 1) ^ 1].v[0] = 0;
      c->work[(k & 1) ^ 1].v[1] = 0;
      if (a.trace_C && k < a.trace_cap) a.trace_C[k] = (int32_t)C;
    }
  }
  return (C == kNone || over) ? kNone : C;
}

// A: clear C, reduce the other unstable labels into next iteration's candidate
__device__ void phase_a_select(const Args& a, uint32_t par, uint32_t C, const Part& p) {
  const uint32_t nwd = ((uint32_t)a.n + 63u) >> 6;
  uint32_t best = kNone;
  for (uint32_t w = p.gtid; w < nwd; w += p.gthreads) {
    uint64_t bits = a.ub[w];
    if (w == (C >> 6)) {
      bits &= ~(1ull << (C & 63));
      a.ub[w] = bits;
    }
    if (bits) best = min(best, (w << 6) + (uint32_t)(__ffsll((unsigned long long)bits) - 1));
  }
  best = wave_min_u32(best);
  if (lane() == 0 && best != kNone) atomicMin(&a.ctl->cand[par ^ 1].v[0], best);
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
  for (uint32_t base = p.gwave * kWave; base < n; base += p.gwaves * kWave) {
    const uint32_t t = base + lane();
    const bool hit = t < n && (uint32_t)a.block[t] == C;
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
    for (uint32_t base = p.gwave * kWave; base < n; base += p.gwaves * kWave) {
      const uint32_t s = base + lane();
      bool sp = false;
      int32_t b = 0;
      if (s < n) {
        b = a.block[s];
        sp = test_bit(a.lt, (uint32_t)b) && !test_bit(a.tb, s);
      }
      if (sp) bid(a, b, (int32_t)s, epoch);
      wave_push(a.slist, cntS, (int32_t)s, sp);
    }
  }
}

// C: relabel and update the unstable set
__device__ void phase_c(const Args& a, uint32_t par, uint32_t k, uint32_t C, const Part& p) {
  const uint32_t nS = a.ctl->cntS[par].v[0];
  const uint32_t nT = a.ctl->cntT[par].v[0];
  uint32_t best = kNone;
  for (uint32_t i = p.gtid; i < nS; i += p.gthreads) {
    const int32_t s = a.slist[i];
    const int32_t old = a.block[s];
    const int32_t nl = (int32_t)(kNone - (uint32_t)a.nlw[old]);
    a.block[s] = nl;
    if (s == nl) {
      atomicOr((unsigned long long*)&a.ub[old >> 6], 1ull << (old & 63));
      atomicOr((unsigned long long*)&a.ub[nl >> 6], 1ull << (nl & 63));
      best = min(best, (uint32_t)old);
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
  best = wave_min_u32(best);
  if (lane() == 0 && best != kNone) atomicMin(&a.ctl->cand[par ^ 1].v[0], best);
  if (p.gtid == 0) {
    if (nS > 0) {
      atomicOr((unsigned long long*)&a.ub[C >> 6], 1ull << (C & 63));
      atomicMin(&a.ctl->cand[par ^ 1].v[0], C);
    }
    a.ctl->cand[par].v[0] = kNone;
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
// per-run initialisation
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kT) k_init_run(Args a, const int32_t* __restrict__ pre,
                                                 uint32_t first, uint64_t nwords) {
  const Part p = part();
  const uint32_t n = (uint32_t)a.n;
  for (uint32_t s = p.gtid; s < n; s += p.gthreads) {
    a.block[s] = pre[s];
    a.nlw[s] = 0;
  }
  for (uint64_t w = p.gtid; w < nwords; w += p.gthreads) a.mw[w] = 0;
  const uint32_t nwd = (n + 63u) >> 6;
  for (uint32_t w = p.gtid; w < nwd; w += p.gthreads) {
    uint64_t bits = 0;
    const uint32_t s0 = w << 6;
    for (uint32_t j = 0; j < 64 && s0 + j < n; ++j)
      if ((uint32_t)pre[s0 + j] == s0 + j) bits |= 1ull << j;
    a.ub[w] = bits;
    a.tb[w] = 0;
    a.lt[w] = 0;
  }
  if (blockIdx.x == 0) {
    uint32_t* c = reinterpret_cast<uint32_t*>(a.ctl);
    for (uint32_t i = threadIdx.x; i < sizeof(Ctl) / 4; i += blockDim.x) c[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
      a.ctl->cand[0].v[0] = (n == 0) ? kNone : first;
      a.ctl->cand[1].v[0] = kNone;
    }
  }
}

__global__ void __launch_bounds__(kT) k_count_leaders(const int32_t* __restrict__ block, int32_t n,
                                                      unsigned long long* out) {
  const Part p = part();
  uint32_t c = 0;
  for (uint32_t s = p.gtid; s < (uint32_t)n; s += p.gthreads) c += (block[s] == (int32_t)s);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) c += (uint32_t)__shfl_xor((int)c, d, kWave);
  if (lane() == 0 && c) atomicAdd(out, (unsigned long long)c);
}

// ---------------------------------------------------------------------------
// engine 2: one kernel per phase
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kT) k_phase_a(Args a, uint32_t k) {
  if (a.ctl->state.v[1]) return;
  const Part p = part();
  const uint32_t C = head(a, k, p);
  if (C == kNone) return;
  phase_a_select(a, k & 1, C, p);
  phase_a_mark(a, k & 1, C, p);
}
__global__ void __launch_bounds__(kT) k_phase_b(Args a, uint32_t k) {
  if (a.ctl->state.v[1]) return;
  phase_b(a, k & 1, k, part());
}
__global__ void __launch_bounds__(kT) k_phase_c(Args a, uint32_t k) {
  if (a.ctl->state.v[1]) return;
  phase_c(a, k & 1, k, a.ctl->state.v[3], part());
}

// ---------------------------------------------------------------------------
// engine 1: persistent cooperative kernel
// ---------------------------------------------------------------------------
__device__ bool grid_barrier(Ctl* ctl, uint32_t& gen) {
  __shared__ uint32_t ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t g = gen;
    __threadfence();
    const uint32_t arrived = atomicAdd(&ctl->bar.v[0], 1u);
    if (arrived == gridDim.x - 1) {
      atomicExch(&ctl->bar.v[0], 0u);
      __threadfence();
      atomicExch(&ctl->bar.v[1], g + 1);
    } else {
      const uint64_t t0 = wall_clock64();
      while (__hip_atomic_load(&ctl->bar.v[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (__hip_atomic_load(&ctl->bar.v[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        if (wall_clock64() - t0 > kBarrierTimeoutTicks) {
          atomicExch(&ctl->bar.v[2], 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __threadfence();
    gen = g + 1;
    ok = __hip_atomic_load(&ctl->bar.v[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
  }
  __syncthreads();
  return ok != 0;
}

__global__ void __launch_bounds__(kPT) k_persistent(Args a) {
  const Part p = part();
  uint32_t gen = 0;
  for (uint32_t k = 0;; ++k) {
    const uint32_t C = head(a, k, p);
    if (C == kNone) break;
    phase_a_select(a, k & 1, C, p);
    phase_a_mark(a, k & 1, C, p);
    if (!grid_barrier(a.ctl, gen)) break;
    phase_b(a, k & 1, k, p);
    if (!grid_barrier(a.ctl, gen)) break;
    phase_c(a, k & 1, k, C, p);
    if (!grid_barrier(a.ctl, gen)) break;
  }
}

template <class T>
bisim_status dalloc(T** p, size_t count, hipStream_t s) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMallocAsync((void**)p, sizeof(T) * count, s);
  if (e != hipSuccess) {
    set_error("device allocation of %zu bytes failed: %s", sizeof(T) * count, hipGetErrorString(e));
    return BISIM_E_NOMEM;
  }
  return BISIM_OK;
}
}  // namespace

bisim_status refine_alloc(bisim_lts* h) {
  const size_t n = (size_t)h->n;
  const size_t nwd = (n + 63) / 64;
  hipStream_t s = h->stream;
  BISIM_TRY(dalloc(&h->block, n, s));
  BISIM_TRY(dalloc(&h->mw, (size_t)h->nwords, s));
  BISIM_TRY(dalloc(&h->tb, nwd, s));
  BISIM_TRY(dalloc(&h->lt, nwd, s));
  BISIM_TRY(dalloc(&h->ub, nwd, s));
  BISIM_TRY(dalloc(&h->nlw, n, s));
  BISIM_TRY(dalloc(&h->tlist, n, s));
  BISIM_TRY(dalloc(&h->slist, n, s));
  BISIM_TRY(dalloc(&h->ctl, 1, s));
  BISIM_TRY_HIP(hipHostMalloc((void**)&h->ctl_host, sizeof(Ctl), hipHostMallocDefault));
  return BISIM_OK;
}

bisim_status refine_run(bisim_lts* h, int32_t* block_id) {
  hipStream_t st = h->stream;
  const int32_t n = h->n;
  int64_t cap = 3 * (int64_t)n - h->pre_blocks + 1;
  if (cap < 1) cap = 1;
  if (h->iter_limit > 0 && h->iter_limit < cap) cap = h->iter_limit;
  if (cap > 0xFFFFFFF0ll) cap = 0xFFFFFFF0ll;

  uint32_t first = 0;
  if (h->first_splitter >= 0) {
    if (h->first_splitter >= n) {
      set_error("first splitter %lld is not a state", (long long)h->first_splitter);
      return BISIM_E_INVALID;
    }
    int32_t lead = -1;
    BISIM_TRY_HIP(hipMemcpyAsync(&lead, h->pre_block + h->first_splitter, sizeof(int32_t),
                                 hipMemcpyDeviceToHost, st));
    BISIM_TRY_HIP(hipStreamSynchronize(st));
    if (lead != h->first_splitter) {
      set_error("first splitter %lld is not a block label of the preprocessed partition",
                (long long)h->first_splitter);
      return BISIM_E_INVALID;
    }
    first = (uint32_t)h->first_splitter;
  }

  Args a{};
  a.n = n;
  a.uniform = h->uniform;
  a.in_ptr = h->in_ptr;
  a.in_src = h->in_src;
  a.in_ord = h->in_ord;
  a.woff = h->woff;
  a.block = h->block;
  a.mw = h->mw;
  a.tb = h->tb;
  a.lt = h->lt;
  a.ub = h->ub;
  a.nlw = h->nlw;
  a.tlist = h->tlist;
  a.slist = h->slist;
  a.ctl = h->ctl;
  a.iter_cap = (uint32_t)cap;
  a.trace_C = h->trace_C;
  a.trace_nsplit = h->trace_nsplit;
  a.trace_work = h->trace_work;
  a.trace_cap = (uint32_t)(h->trace_cap > 0xFFFFFFFFll ? 0xFFFFFFFFll : h->trace_cap);

  const int cu = h->num_cu > 0 ? h->num_cu : 1;
  int64_t g_init = ((int64_t)n + kT - 1) / kT;
  if (g_init > cu * 8) g_init = cu * 8;
  if (g_init < 1) g_init = 1;
  hipLaunchKernelGGL(k_init_run, dim3((unsigned)g_init), dim3(kT), 0, st, a, h->pre_block, first,
                     h->nwords);
  BISIM_TRY_HIP(hipGetLastError());
  BISIM_TRY_HIP(hipEventRecord(h->ev0, st));

  int engine = h->engine;
  if (engine == 0) engine = 1;
  if (engine == 1) {
    int per_cu = 0;
    BISIM_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent, kPT, 0));
    if (per_cu < 1) {
      set_error("persistent kernel cannot be resident");
      return BISIM_E_DEVICE;
    }
    int grid = h->grid > 0 ? h->grid : cu;
    if (grid > per_cu * cu) grid = per_cu * cu;
    void* args[] = {&a};
    BISIM_TRY_HIP(hipLaunchCooperativeKernel((const void*)k_persistent, dim3(grid), dim3(kPT),
                                             args, 0, st));
  } else {
    int grid = h->grid > 0 ? h->grid : cu * 4;
    uint32_t k = 0, chunk = 8;
    for (;;) {
      for (uint32_t j = 0; j < chunk; ++j, ++k) {
        hipLaunchKernelGGL(k_phase_a, dim3(grid), dim3(kT), 0, st, a, k);
        hipLaunchKernelGGL(k_phase_b, dim3(grid), dim3(kT), 0, st, a, k);
        hipLaunchKernelGGL(k_phase_c, dim3(grid), dim3(kT), 0, st, a, k);
      }
      BISIM_TRY_HIP(hipGetLastError());
      BISIM_TRY_HIP(hipMemcpyAsync(&h->ctl_host->state, &h->ctl->state, sizeof(Line),
                                   hipMemcpyDeviceToHost, st));
      BISIM_TRY_HIP(hipStreamSynchronize(st));
      if (h->ctl_host->state.v[1]) break;
      if (k >= (uint32_t)cap + 1) break;  // the head's cap check has fired or will
      if (chunk < 256) chunk *= 2;
    }
  }
  BISIM_TRY_HIP(hipGetLastError());
  BISIM_TRY_HIP(hipEventRecord(h->ev1, st));
  BISIM_TRY_HIP(hipMemcpyAsync(h->ctl_host, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  BISIM_TRY_HIP(hipStreamSynchronize(st));
  float ms = 0.f;
  BISIM_TRY_HIP(hipEventElapsedTime(&ms, h->ev0, h->ev1));
  h->t_alg_ms = ms;
  const Ctl& c = *h->ctl_host;
  if (c.bar.v[2]) {
    set_error("grid barrier timed out");
    return BISIM_E_DEVICE;
  }
  if (!c.state.v[1]) {
    set_error("refinement did not finish");
    return BISIM_E_DEVICE;
  }
  h->last_iters = c.state.v[0];
  if (c.state.v[2]) {
    set_error("iteration cap %lld exceeded", (long long)cap);
    return BISIM_E_ITERCAP;
  }
  if (block_id && n > 0)
    BISIM_TRY_HIP(hipMemcpyAsync(block_id, h->block, sizeof(int32_t) * (size_t)n,
                                 hipMemcpyDeviceToDevice, st));
  unsigned long long* cnt = nullptr;
  BISIM_TRY(dalloc(&cnt, 1, st));
  BISIM_TRY_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), st));
  hipLaunchKernelGGL(k_count_leaders, dim3((unsigned)g_init), dim3(kT), 0, st, h->block, n, cnt);
  unsigned long long nb = 0;
  BISIM_TRY_HIP(hipMemcpyAsync(&nb, cnt, sizeof(nb), hipMemcpyDeviceToHost, st));
  BISIM_TRY_HIP(hipFreeAsync(cnt, st));
  BISIM_TRY_HIP(hipStreamSynchronize(st));
  h->last_blocks = (int64_t)nb;
  return BISIM_OK;
}

}  // namespace bisim
