// The refinement loop of the labelled PRAM algorithm (Algorithm 3, section 4),
// as three data-parallel phases per iteration with a grid-wide dependency
// between them (the paper's GPU port also needs synchronisation points after
// the mark and the leader election; section 5):
//
//   A  select + mark    C is the unstable block chosen by the policy (plain:
//                       the smallest label, the priority-CRCW reading of the
//                       concurrent write; learned: the smallest label of the
//                       highest priority level).  Clear C's unstable bit; for
//                       the plain policy, find the next smallest unstable
//                       label for the next iteration's candidate; for every
//                       state t with block[t] == C visit t's in-transitions
//                       (source s, action rank o) and set mark slot o of s.
//                       The first touch of a state appends it to the touched
//                       list T; a touched leader sets its bit in the
//                       leader-touched bitmap.
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
//                       unstable labels are reduced into the candidate.
//                       Marks and touched bits of T are cleared.
//   S  (learned policy, one workgroup) re-score the blocks created or split
//                       in C and C itself with the network, move them between
//                       priority levels, and pick the next splitter.  Every R
//                       iterations all unstable blocks are re-scored first.
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
#include <hip/hip_ext.h>

#include <sys/stat.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <new>
#include <string>
#include <vector>

#include "internal.h"
#include "mlp_dev.h"
#include "refine_dev.h"

namespace bisim {

namespace {
constexpr int kT = 256;   // per-phase kernels
constexpr int kPT = 512;  // persistent kernel
constexpr uint64_t kBarrierTimeoutTicks = 10ull * 100000000ull;  // 10 s at 100 MHz

// ---------------------------------------------------------------------------
// engine 2: one kernel per phase
// ---------------------------------------------------------------------------
template <bool L, bool T>
__global__ void __launch_bounds__(kT) k_phase_a(Args a, uint32_t k) {
  if (a.ctl->state.v[1]) return;
  const Part p = part();
  const uint32_t C = head(a, k, p);
  if (C == kNone) return;
  phase_a_select<L>(a, k & 1, C, k, p);
  phase_a_mark(a, k & 1, C, p);
}
template <bool L, bool T>
__global__ void __launch_bounds__(kT) k_phase_b(Args a, uint32_t k) {
  if (a.ctl->state.v[1]) return;
  phase_b(a, k & 1, k, part());
}
template <bool L, bool T>
__global__ void __launch_bounds__(kT) k_phase_c(Args a, uint32_t k) {
  if (a.ctl->state.v[1]) return;
  phase_c<L, T>(a, k & 1, k, a.ctl->state.v[3], part());
}
// plain policy: two kernels per iteration
// The per-phase kernels load the control words and their first scan chunk
// together, before any branch.
template <bool Agg>
__global__ void __launch_bounds__(kT) k_fused_x(Args a, uint32_t k) {
  const Part p = part();
  XChunk ch;
  load_xchunk<x_chunks<Agg>()>(a, k, p.gwave * kWave * x_chunks<Agg>(), ch);
  const uint32_t done = a.ctl->state.v[1];
  const uint32_t cand = a.ctl->cand[k & 1].v[0];
  if (done) return;
  const uint32_t C = head2(a, k, p, cand);
  if (C == kNone) return;
  phase_x<Agg>(a, k, C, p, &ch);
}
__global__ void __launch_bounds__(kT) k_fused_y(Args a, uint32_t k) {
  const Part p = part();
  YChunk ch;
  load_ychunk(a, k, p.gwave * kWave * kFusedU, ch);
  const uint32_t done = a.ctl->state.v[1];
  const uint32_t C = a.ctl->state.v[3];
  if (done) return;
  phase_y(a, k, p, C, &ch);
}

constexpr int kST = 1024;  // re-scoring + selection workgroup (learned policy)
__global__ void __launch_bounds__(kST) k_phase_s(Args a, uint32_t k) {
  if (a.ctl->state.v[1]) return;
  extern __shared__ float sw[];
  MlpLds M = mlp_lds_layout(sw, kPolicyF);
  mlp_stage(M, a.wbf, kPolicyF);
  __syncthreads();
  phase_s(a, M, k & 1, k);
}
__global__ void __launch_bounds__(kT) k_phase_f1(Args a, uint32_t k) {
  if (a.ctl->state.v[1]) return;
  extern __shared__ float sw[];
  MlpLds M = mlp_lds_layout(sw, kPolicyF);
  mlp_stage(M, a.wbf, kPolicyF);
  __syncthreads();
  phase_f1(a, M, k + 1, part());
}
__global__ void __launch_bounds__(kT) k_phase_f2(Args a, uint32_t k) {
  if (a.ctl->state.v[1]) return;
  phase_f2(a, part());
}

// ---------------------------------------------------------------------------
// engine 1: persistent cooperative kernel
// ---------------------------------------------------------------------------
// Grid barrier.  Arrival is two-level: workgroups are grouped by
// blockIdx % 8 (the hardware deals consecutive workgroups round-robin to the
// 8 XCDs), the last arriver of each group arrives at the top counter, and the
// last of those advances the generation.  Every arrival is preceded by an
// agent-scope release (this workgroup's writes reach memory visible to all
// XCDs); waiting polls the generation with relaxed loads and issues a single
// acquire fence once it has moved, so polling does not keep invalidating the
// caches the other workgroups of the XCD are using.  The wait is bounded:
// after the timeout every workgroup leaves through the abort flag.
__device__ bool grid_barrier(Ctl* ctl, uint32_t& gen) {
  __shared__ uint32_t ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t g = gen;
    const uint32_t groups = gridDim.x < 8 ? gridDim.x : 8;
    const uint32_t grp = blockIdx.x % groups;
    const uint32_t members = (gridDim.x - grp + groups - 1) / groups;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    uint32_t* gcount = &ctl->barg[grp].v[0];
    const uint32_t a1 = __hip_atomic_fetch_add(gcount, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool last = false;
    if (a1 == members - 1) {
      // the group counter is reset before (release) the arrival that can
      // let the generation advance
      __hip_atomic_store(gcount, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t a2 =
          __hip_atomic_fetch_add(&ctl->bar.v[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (a2 == groups - 1) {
        __hip_atomic_store(&ctl->bar.v[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctl->bar.v[1], g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        last = true;
      }
    }
    if (!last) {
      const uint64_t t0 = wall_clock64();
      while (__hip_atomic_load(&ctl->bar.v[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (__hip_atomic_load(&ctl->bar.v[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
        if (wall_clock64() - t0 > kBarrierTimeoutTicks) {
          atomicExch(&ctl->bar.v[2], 1u);
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    gen = g + 1;
    ok = __hip_atomic_load(&ctl->bar.v[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
  }
  __syncthreads();
  return ok != 0;
}

template <bool L>
__global__ void __launch_bounds__(kPT) k_persistent(Args a) {
  extern __shared__ float sw[];
  MlpLds M{};
  if (L) {
    M = mlp_lds_layout(sw, kPolicyF);
    mlp_stage(M, a.wbf, kPolicyF);
    __syncthreads();
  }
  const Part p = part();
  uint32_t gen = 0;
  if (!L) {  // plain policy: two steps per iteration
    for (uint32_t k = 0;; ++k) {
      const uint32_t C = head2(a, k, p);
      if (C == kNone) break;
      if (a.hot)
        phase_x<true>(a, k, C, p);
      else
        phase_x<false>(a, k, C, p);
      if (!grid_barrier(a.ctl, gen)) break;
      phase_y(a, k, p, a.ctl->state.v[3]);
      if (!grid_barrier(a.ctl, gen)) break;
    }
    return;
  }
  for (uint32_t k = 0;; ++k) {
    const uint32_t C = head(a, k, p);
    if (C == kNone) break;
    phase_a_select<L>(a, k & 1, C, k, p);
    phase_a_mark(a, k & 1, C, p);
    if (!grid_barrier(a.ctl, gen)) break;
    phase_b(a, k & 1, k, p);
    if (!grid_barrier(a.ctl, gen)) break;
    phase_c<L, L>(a, k & 1, k, C, p);
    if (!grid_barrier(a.ctl, gen)) break;
    if (L) {
      if (a.rescore && (k + 1) % a.rescore == 0) {
        phase_f1(a, M, k + 1, p);
        if (!grid_barrier(a.ctl, gen)) break;
        phase_f2(a, p);
        if (!grid_barrier(a.ctl, gen)) break;
      }
      if (blockIdx.x == 0) phase_s(a, M, k & 1, k);
      if (!grid_barrier(a.ctl, gen)) break;
    }
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

int grid_cap(int cu) { return cu * 8; }
}  // namespace

bisim_status refine_alloc(bisim_lts* h) {
  const size_t n = (size_t)h->n;
  const size_t nwd = (n + 63) / 64;
  hipStream_t s = h->stream;
  BISIM_TRY(dalloc(&h->block, n, s));
  BISIM_TRY(dalloc(&h->mw, 2 * (size_t)h->nwords, s));
  BISIM_TRY(dalloc(&h->tb, 2 * nwd, s));
  BISIM_TRY(dalloc(&h->lt, 2 * nwd, s));
  BISIM_TRY(dalloc(&h->sb, 2 * nwd, s));
  BISIM_TRY(dalloc(&h->nlist, n, s));
  BISIM_TRY(dalloc(&h->ub, nwd, s));
  BISIM_TRY(dalloc(&h->us, (nwd + 63) / 64, s));
  BISIM_TRY(dalloc(&h->nlw, n, s));
  BISIM_TRY(dalloc(&h->tlist, n, s));
  BISIM_TRY(dalloc(&h->slist, n, s));
  BISIM_TRY(dalloc(&h->ctl, 1, s));
  if (!h->ctl_host)  // the allocation-free entry point brings its own host mirror
    BISIM_TRY_HIP(hipHostMalloc((void**)&h->ctl_host, sizeof(Ctl), hipHostMallocDefault));
  return BISIM_OK;
}

// feature / policy state, allocated on first use
bisim_status refine_alloc_features(bisim_lts* h) {
  if (h->acc) return BISIM_OK;
  const size_t n = (size_t)h->n;
  hipStream_t s = h->stream;
  const size_t nwd = (n + 63) / 64, nsw = (nwd + 63) / 64, ntw = (nsw + 63) / 64;
  BISIM_TRY(dalloc(&h->acc, 17 * n, s));
  BISIM_TRY(dalloc(&h->born, n, s));
  BISIM_TRY(dalloc(&h->used, n, s));
  BISIM_TRY(dalloc(&h->chg, 2 * n, s));
  BISIM_TRY(dalloc(&h->lvl, n, s));
  BISIM_TRY(dalloc(&h->lvb, kLevels * nwd, s));
  BISIM_TRY(dalloc(&h->lvs, kLevels * nsw, s));
  BISIM_TRY(dalloc(&h->lvt, kLevels * ntw, s));
  BISIM_TRY(dalloc(&h->lvq, 2 * n + 1, s));
  return BISIM_OK;
}

Args make_args(bisim_lts* h, uint32_t cap, bool learned, bool track) {
  Args a{};
  a.n = h->n;
  a.uniform = h->uniform;
  a.hot = h->max_out >= kHotDegree;
  a.in_ptr = h->in_ptr;
  a.in_src = h->in_src;
  a.in_ord = h->in_ord;
  a.woff = h->woff;
  a.block = h->block;
  a.mw = h->mw;
  a.tb = h->tb;
  a.lt = h->lt;
  a.ub = h->ub;
  a.us = h->us;
  a.nlw = h->nlw;
  a.tlist = h->tlist;
  a.sb = h->sb;
  a.nlist = h->nlist;
  a.nwords = h->nwords;
  a.slist = h->slist;
  a.ctl = h->ctl;
  a.iter_cap = cap;
  a.trace_C = h->trace_C;
  a.trace_nsplit = h->trace_nsplit;
  a.trace_work = h->trace_work;
  a.trace_cap = (uint32_t)(h->trace_cap > 0xFFFFFFFFll ? 0xFFFFFFFFll : h->trace_cap);
  if (track || learned) {
    a.sfeat = h->sfeat;
    a.acc = h->acc;
    a.born = h->born;
    a.used = h->used;
    a.chg = h->chg;
  }
  if (learned) {
    a.lvl = h->lvl;
    a.lvb = h->lvb;
    a.lvs = h->lvs;
    a.lvt = h->lvt;
    a.lvq = h->lvq;
  }
  a.wbf = learned ? h->policy_w : nullptr;
  a.rescore = (uint32_t)(h->rescore_every > 0 ? h->rescore_every : 64);
  return a;
}

// per-run initialisation, shared with the training-data collector
bisim_status refine_init(bisim_lts* h, const Args& a, uint32_t first, bool learned, bool track,
                         const int32_t* start) {
  hipStream_t st = h->stream;
  const int cu = h->num_cu > 0 ? h->num_cu : 1;
  int64_t g = ((int64_t)h->n + kT - 1) / kT;
  g = g > grid_cap(cu) ? grid_cap(cu) : (g < 1 ? 1 : g);
  hipLaunchKernelGGL(k_init_run, dim3((unsigned)g), dim3(kT), 0, st, a, start, first,
                     h->nwords, learned ? 1u : 0u);
  hipLaunchKernelGGL(k_init_summary, dim3((unsigned)g), dim3(kT), 0, st, a);
  BISIM_TRY_HIP(hipGetLastError());
  if (track || learned) {
    hipLaunchKernelGGL(k_zero_features, dim3((unsigned)g), dim3(kT), 0, st, a);
    hipLaunchKernelGGL(k_accumulate_features, dim3((unsigned)g), dim3(kT), 0, st, a,
                       h->pre_block);
    BISIM_TRY_HIP(hipGetLastError());
  }
  if (learned) {
    hipLaunchKernelGGL(k_levels_all, dim3((unsigned)g), dim3(kT),
                       mlp_lds_floats(kPolicyF) * sizeof(float), st, a, 0u);
    hipLaunchKernelGGL(k_levels_insert, dim3((unsigned)g), dim3(kT), 0, st, a);
    hipLaunchKernelGGL(k_learned_first, dim3(1), dim3(kWave), 0, st, a);
    BISIM_TRY_HIP(hipGetLastError());
  }
  return BISIM_OK;
}

// number of block labels (states that are their block's label) of a partition
bisim_status count_labels(bisim_lts* h, const int32_t* block, int64_t* out) {
  hipStream_t st = h->stream;
  const int cu = h->num_cu > 0 ? h->num_cu : 1;
  unsigned long long* cnt = nullptr;
  BISIM_TRY(dalloc(&cnt, 1, st));
  BISIM_TRY_HIP(hipMemsetAsync(cnt, 0, sizeof(unsigned long long), st));
  int64_t g = ((int64_t)h->n + kT - 1) / kT;
  g = g > grid_cap(cu) ? grid_cap(cu) : (g < 1 ? 1 : g);
  if (h->n > 0)
    hipLaunchKernelGGL(k_count_leaders, dim3((unsigned)g), dim3(kT), 0, st, block, h->n, cnt);
  unsigned long long nb = 0;
  BISIM_TRY_HIP(hipMemcpyAsync(&nb, cnt, sizeof(nb), hipMemcpyDeviceToHost, st));
  BISIM_TRY_HIP(dev_free(cnt, st));
  BISIM_TRY_HIP(hipStreamSynchronize(st));
  *out = (int64_t)nb;
  return BISIM_OK;
}

static bisim_status refine_run_impl(bisim_lts* h, int32_t* block_id);

namespace {
// ---------------------------------------------------------------------------
// automatic engine choice: a cached tuner over (engine, grid)
// ---------------------------------------------------------------------------
constexpr int32_t kTuneMinStates = 200000;  // smaller LTSs: per-phase kernels, no trials
constexpr int64_t kTuneIters = 96;          // iterations per trial

std::string lts_tune_key(const bisim_lts* h) {
  hipDeviceProp_t p;
  std::string arch = "gpu";
  if (hipGetDeviceProperties(&p, h->device) == hipSuccess) arch = p.gcnArchName;
  for (char& c : arch)
    if (c == ' ' || c == ':') c = '_';
  int ln = 0, lm = 0;
  for (int64_t v = h->n; v > 1; v >>= 1) ++ln;
  for (int64_t v = h->m; v > 1; v >>= 1) ++lm;
  char buf[256];
  snprintf(buf, sizeof buf, "lts_%s_cu%d_n%d_m%d_u%d", arch.c_str(), h->num_cu, ln, lm,
           h->uniform);
  return buf;
}

std::string lts_tune_path() {
  const char* e = getenv("BISIM_TUNE_CACHE");
  if (e && *e) return e;
  const char* home = getenv("HOME");
  return std::string(home && *home ? home : "/tmp") + "/.cache/bisim_tune.txt";
}

bool lts_tune_lookup(const std::string& key, int* engine, int* grid) {
  FILE* f = fopen(lts_tune_path().c_str(), "r");
  if (!f) return false;
  char line[512];
  bool found = false;
  while (fgets(line, sizeof line, f)) {
    char k[256];
    int e = 0, g = 0;
    float us = 0.f;
    if (sscanf(line, "%255s %d %d %f", k, &e, &g, &us) == 4 && key == k && (e == 2 || e == 3) &&
        g > 0) {
      *engine = e;
      *grid = g;
      found = true;
    }
  }
  fclose(f);
  return found;
}

void lts_tune_store(const std::string& key, int engine, int grid, float us) {
  const std::string path = lts_tune_path();
  const std::string dir = path.substr(0, path.find_last_of('/'));
  for (size_t i = 1; i <= dir.size(); ++i)
    if (i == dir.size() || dir[i] == '/') (void)mkdir(dir.substr(0, i).c_str(), 0755);
  FILE* f = fopen(path.c_str(), "a");
  if (!f) return;
  fprintf(f, "%s %d %d %.4f\n", key.c_str(), engine, grid, us);
  fclose(f);
}
}  // namespace

// Engine and grid of an automatic run: the per-phase kernels for small LTSs
// (and for the learned policy, Algorithm 2, traced runs and the
// allocation-free entry point); otherwise the cached choice for this device
// and size class, else the fastest of a few candidates timed on the first
// kTuneIters iterations of this LTS (each timed twice, the second kept).
static bisim_status choose_engine(bisim_lts* h, int* engine, int* grid) {
  const int cu = h->num_cu > 0 ? h->num_cu : 1;
  *engine = 2;
  *grid = h->grid;
  const bool learned = h->policy == 1 && h->policy_w;
  if (h->n < kTuneMinStates || learned || h->algorithm == 2 || h->trace_cap > 0 ||
      h->first_splitter >= 0 || h->iter_limit > 0 || h->profile_every > 0 || arena_active() ||
      h->start_override)
    return BISIM_OK;
  const std::string key = lts_tune_key(h);
  int e = 0, g = 0;
  if (lts_tune_lookup(key, &e, &g)) {
    *engine = e;
    *grid = h->grid > 0 ? h->grid : g;
    return BISIM_OK;
  }
  struct Cand {
    int engine, grid;
  };
  const Cand cands[] = {{2, cu * 4}, {2, cu * 8}, {2, cu * 16}, {3, cu * 4}, {3, cu * 8}};
  const int saved_engine = h->engine, saved_grid = h->grid;
  const int64_t saved_limit = h->iter_limit;
  float best = 1e30f;
  int be = 2, bg = cu * 8;
  bisim_status rc = BISIM_OK;
  for (const Cand& c : cands) {
    h->engine = c.engine;
    h->grid = c.grid;
    h->iter_limit = kTuneIters;
    float us = 0.f;
    for (int rep = 0; rep < 2; ++rep) {
      const bisim_status r = refine_run_impl(h, nullptr);
      if (r != BISIM_OK && r != BISIM_E_ITERCAP) {
        rc = r;
        break;
      }
      const int64_t its = r == BISIM_OK ? h->last_iters : kTuneIters;
      us = (float)(h->t_alg_ms * 1000.0 / (double)(its > 0 ? its : 1));
    }
    if (rc != BISIM_OK) break;
    if (us < best) {
      best = us;
      be = c.engine;
      bg = c.grid;
    }
  }
  h->engine = saved_engine;
  h->grid = saved_grid;
  h->iter_limit = saved_limit;
  if (rc != BISIM_OK) return rc;
  clear_error();
  lts_tune_store(key, be, bg, best);
  *engine = be;
  *grid = h->grid > 0 ? h->grid : bg;
  return BISIM_OK;
}

bisim_status refine_run(bisim_lts* h, int32_t* block_id) {
  if (h->engine != 0) {
    h->run_engine = h->engine;
    return refine_run_impl(h, block_id);
  }
  int engine = 2, grid = 0;
  BISIM_TRY(choose_engine(h, &engine, &grid));
  const int saved_grid = h->grid;
  h->engine = engine;
  h->grid = grid;
  h->run_engine = engine;
  const bisim_status rc = refine_run_impl(h, block_id);
  h->engine = 0;
  h->grid = saved_grid;
  return rc;
}

static bisim_status refine_run_impl(bisim_lts* h, int32_t* block_id) {
  hipStream_t st = h->stream;
  const int32_t n = h->n;
  const bool learned = h->policy == 1 && h->policy_w;
  const bool rcpp = h->algorithm == 2;
  if (rcpp && learned) {
    set_error("coarsest_partition: Algorithm 2 runs with the plain splitter policy only");
    return BISIM_E_UNSUPPORTED;
  }
  // Algorithm 2 starts from pi_0 itself, Algorithm 3 from the preprocessed partition
  const int32_t* start = rcpp ? h->init_block : h->pre_block;
  h->run_pre_blocks = h->pre_blocks;
  if (rcpp) BISIM_TRY(count_labels(h, start, &h->run_pre_blocks));
  if (h->start_override && !rcpp && !learned) {  // a refinement of pi_pre (hybrid runs)
    start = h->start_override;
    h->run_pre_blocks = h->start_override_blocks;
  }
  int64_t cap = 3 * (int64_t)n - h->run_pre_blocks + 1;
  if (cap < 1) cap = 1;
  if (h->iter_limit > 0 && h->iter_limit < cap) cap = h->iter_limit;
  if (cap > 0xFFFFFFF0ll) cap = 0xFFFFFFF0ll;

  uint32_t first = 0;
  if (h->first_splitter >= 0 && !learned) {
    if (h->first_splitter >= n) {
      set_error("first splitter %lld is not a state", (long long)h->first_splitter);
      return BISIM_E_INVALID;
    }
    int32_t lead = -1;
    BISIM_TRY_HIP(hipMemcpyAsync(&lead, start + h->first_splitter, sizeof(int32_t),
                                 hipMemcpyDeviceToHost, st));
    BISIM_TRY_HIP(hipStreamSynchronize(st));
    if (lead != h->first_splitter) {
      set_error("first splitter %lld is not a block label of the preprocessed partition",
                (long long)h->first_splitter);
      return BISIM_E_INVALID;
    }
    first = (uint32_t)h->first_splitter;
  }
  const int engine = h->engine == 0 ? 2 : h->engine;  // per-phase kernels: the default
  if (engine == 3 && (learned || rcpp)) {
    set_error("coarsest_partition: the member-list engine runs Algorithm 3 with the plain "
              "splitter policy only");
    return BISIM_E_UNSUPPORTED;
  }
  if (learned) BISIM_TRY(refine_alloc_features(h));
  Args a = make_args(h, (uint32_t)cap, learned, learned);
  a.rcpp = rcpp ? 1u : 0u;
  BISIM_TRY(refine_init(h, a, first, learned, learned, start));
  BISIM_TRY_HIP(hipEventRecord(h->ev0, st));

  const int cu = h->num_cu > 0 ? h->num_cu : 1;
  const size_t lds = learned ? mlp_lds_floats(kPolicyF) * sizeof(float) : 0;
  std::vector<uint32_t> sampled;
  std::vector<hipEvent_t> sample_start;
  if (engine == 3) {
    BISIM_TRY(lists_loop(h, (uint32_t)cap, h->count_work != 0));
  } else if (engine == 1) {
    int per_cu = 0;
    if (learned)
      BISIM_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<true>, kPT, lds));
    else
      BISIM_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<false>, kPT, lds));
    if (per_cu < 1) {
      set_error("persistent kernel cannot be resident");
      return BISIM_E_DEVICE;
    }
    int grid = h->grid > 0 ? h->grid : cu;
    h->run_grid = grid;
    if (grid > per_cu * cu) grid = per_cu * cu;
    void* args[] = {&a};
    const void* fn = learned ? (const void*)k_persistent<true> : (const void*)k_persistent<false>;
    BISIM_TRY_HIP(hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kPT), args, lds, st));
  } else {
    int grid = h->grid > 0 ? h->grid : cu * 8;  // 2048 workgroups on MI355X: best of a 128..2048 sweep
    h->run_grid = grid;
    const bool prof = h->profile_every > 0;
    if (prof && !h->pev) {
      h->pev = new (std::nothrow) hipEvent_t[8 * 256];
      if (!h->pev) return BISIM_E_NOMEM;
      for (int i = 0; i < 8 * 256; ++i) BISIM_TRY_HIP(hipEventCreate(&h->pev[i]));
      h->pev_slots = 256;
    }
    sampled.clear();
    sample_start.clear();
    // Sampled iterations bind an event to the end of each phase kernel (and of
    // the previous iteration's last kernel).  Kernels of one stream run back to
    // back, so a phase's duration is the distance between consecutive ends; no
    // start marker is put between the kernels.
    auto go = [&](auto kern, hipEvent_t stop, size_t shm, uint32_t k) {
      if (stop)
        hipExtLaunchKernelGGL(kern, dim3(grid), dim3(kT), (uint32_t)shm, st, nullptr, stop, 0, a, k);
      else
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kT), shm, st, a, k);
    };
    const int nph = learned ? 4 : 2;
    const uint64_t pe = prof ? (uint64_t)h->profile_every : 0;
    hipEvent_t carry = nullptr;  // end of the previous iteration, if the current one is sampled
    uint32_t k = 0, chunk = 8;
    for (;;) {
      for (uint32_t j = 0; j < chunk; ++j, ++k) {
        hipEvent_t ends[4] = {nullptr, nullptr, nullptr, nullptr};
        const size_t slot = sampled.size();
        const bool samp = prof && carry && slot < (size_t)h->pev_slots;
        if (samp) {
          for (int q = 0; q < nph; ++q) ends[q] = h->pev[8 * slot + 1 + q];
          sampled.push_back(k);
          sample_start.push_back(carry);
        }
        carry = nullptr;
        if (prof && (k + 1) % pe == 0 && sampled.size() < (size_t)h->pev_slots) {
          if (!ends[nph - 1]) ends[nph - 1] = h->pev[8 * sampled.size()];
          carry = ends[nph - 1];
        }
        if (learned) {
          go(k_phase_a<true, true>, ends[0], 0, k);
          go(k_phase_b<true, true>, ends[1], 0, k);
          go(k_phase_c<true, true>, ends[2], 0, k);
          if (a.rescore && (k + 1) % a.rescore == 0) {
            go(k_phase_f1, nullptr, lds, k);
            go(k_phase_f2, nullptr, 0, k);
          }
          if (ends[3])
            hipExtLaunchKernelGGL(k_phase_s, dim3(1), dim3(kST), (uint32_t)lds, st, nullptr,
                                  ends[3], 0, a, k);
          else
            hipLaunchKernelGGL(k_phase_s, dim3(1), dim3(kST), lds, st, a, k);
        } else {
          if (a.hot)
            go(k_fused_x<true>, ends[0], 0, k);
          else
            go(k_fused_x<false>, ends[0], 0, k);
          go(k_fused_y, ends[1], 0, k);
        }
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
  if (c.state.v[4]) {
    set_error(engine == 3 ? "member-list engine: inconsistent block ranges"
                          : "learned splitter policy: priority structure inconsistent");
    return BISIM_E_DEVICE;
  }
  if (!c.state.v[1]) {
    set_error("refinement did not finish");
    return BISIM_E_DEVICE;
  }
  h->last_iters = c.state.v[0];
  for (int q = 0; q < 4 && engine != 3; ++q) {  // engine 3 keeps its own
    h->phase_ms[q] = 0;
    h->phase_cnt[q] = 0;
  }
  for (size_t i = 0; i < sampled.size(); ++i) {
    if ((int64_t)sampled[i] + 1 >= h->last_iters) continue;  // no splitter: early-exit kernels
    hipEvent_t prev = sample_start[i];
    for (int q = 0; q < (learned ? 4 : 2); ++q) {
      hipEvent_t cur = h->pev[8 * i + 1 + q];
      float pm = 0.f;
      if (hipEventElapsedTime(&pm, prev, cur) == hipSuccess) {
        h->phase_ms[q] += pm;
        h->phase_cnt[q] += 1;
      }
      prev = cur;
    }
  }
  if (c.state.v[2]) {
    set_error("iteration cap %lld exceeded", (long long)cap);
    return BISIM_E_ITERCAP;
  }
  if (block_id && n > 0)
    BISIM_TRY_HIP(hipMemcpyAsync(block_id, h->block, sizeof(int32_t) * (size_t)n,
                                 hipMemcpyDeviceToDevice, st));
  return count_labels(h, h->block, &h->last_blocks);
}

// one iteration of the per-phase engine with feature tracking (training-data
// collection steps the loop from the host)
bisim_status refine_step_tracked(bisim_lts* h, const Args& a, uint32_t k) {
  hipStream_t st = h->stream;
  const int cu = h->num_cu > 0 ? h->num_cu : 1;
  const int grid = cu * 4;
  hipLaunchKernelGGL((k_phase_a<false, true>), dim3(grid), dim3(kT), 0, st, a, k);
  hipLaunchKernelGGL((k_phase_b<false, true>), dim3(grid), dim3(kT), 0, st, a, k);
  hipLaunchKernelGGL((k_phase_c<false, true>), dim3(grid), dim3(kT), 0, st, a, k);
  BISIM_TRY_HIP(hipGetLastError());
  return BISIM_OK;
}

}  // namespace bisim

// ---------------------------------------------------------------------------
// training data for the learned splitter policy
// ---------------------------------------------------------------------------
namespace bisim {
namespace {
// One workgroup per sampled candidate X (evenly spaced among the unstable
// labels in label order): its features, and log(1 + the number of blocks that
// would split if X were the splitter now) from a what-if mark + compare in LDS.
__global__ void __launch_bounds__(256) k_collect(Args a, uint32_t k, uint32_t limit,
                                                 float* __restrict__ feat,
                                                 float* __restrict__ tgt,
                                                 int32_t* __restrict__ meta, uint32_t* written) {
  extern __shared__ uint64_t lds[];
  __shared__ uint32_t wsum[256 / kWave];
  __shared__ uint32_t sx[2];
  const uint32_t n = (uint32_t)a.n, nwd = (n + 63u) >> 6;
  const uint32_t tid = threadIdx.x, wid = tid / kWave;
  uint32_t c = 0;
  for (uint32_t q = tid; q < nwd; q += blockDim.x) c += (uint32_t)__popcll(a.ub[q]);
  for (int d = 32; d >= 1; d >>= 1) c += (uint32_t)__shfl_xor((int)c, d, kWave);
  if (lane() == 0) wsum[wid] = c;
  __syncthreads();
  if (tid == 0) {
    uint32_t nU = 0;
    for (uint32_t q = 0; q < blockDim.x / kWave; ++q) nU += wsum[q];
    sx[0] = nU;
  }
  __syncthreads();
  const uint32_t nU = sx[0];
  const uint32_t total = min(limit, nU);
  if (blockIdx.x >= total) return;
  const uint32_t idx = blockIdx.x * (nU / total);
  if (tid == 0) {
    uint32_t r = idx, X = 0;
    for (uint32_t q = 0; q < nwd; ++q) {
      uint64_t bits = a.ub[q];
      const uint32_t pc = (uint32_t)__popcll(bits);
      if (r < pc) {
        for (uint32_t j = 0; j < r; ++j) bits &= bits - 1;
        X = (q << 6) + (uint32_t)(__ffsll((unsigned long long)bits) - 1);
        break;
      }
      r -= pc;
    }
    sx[1] = X;
    if (blockIdx.x == 0) *written = total;
  }
  __syncthreads();
  const uint32_t X = sx[1];
  if (tid < kPolicyF) feat[(size_t)blockIdx.x * kPolicyF + tid] = block_feature(a, X, tid, k);
  if (meta && tid == 0) {
    meta[2 * (size_t)blockIdx.x] = (int32_t)k;
    meta[2 * (size_t)blockIdx.x + 1] = (int32_t)X;
  }
  uint64_t* mask = lds;
  uint8_t* flag = reinterpret_cast<uint8_t*>(lds + n);
  for (uint32_t s = tid; s < n; s += blockDim.x) {
    mask[s] = 0;
    flag[s] = 0;
  }
  __syncthreads();
  for (uint32_t t = tid; t < n; t += blockDim.x)
    if ((uint32_t)a.block[t] == X)
      for (uint32_t e = a.in_ptr[t]; e < a.in_ptr[t + 1]; ++e)
        atomicOr((unsigned long long*)&mask[a.in_src[e]], 1ull << (a.in_ord[e] & 63));
  __syncthreads();
  for (uint32_t s = tid; s < n; s += blockDim.x) {
    const int32_t b = a.block[s];
    if (mask[s] != mask[b]) flag[b] = 1;
  }
  __syncthreads();
  uint32_t cnt = 0;
  for (uint32_t s = tid; s < n; s += blockDim.x) cnt += flag[s];
  for (int d = 32; d >= 1; d >>= 1) cnt += (uint32_t)__shfl_xor((int)cnt, d, kWave);
  __syncthreads();
  if (lane() == 0) wsum[wid] = cnt;
  __syncthreads();
  if (tid == 0) {
    uint32_t s = 0;
    for (uint32_t q = 0; q < blockDim.x / kWave; ++q) s += wsum[q];
    tgt[blockIdx.x] = log1pf((float)s);
  }
}
}  // namespace
}  // namespace bisim

using namespace bisim;

extern "C" {

bisim_status bisim_set_splitter_policy(bisim_lts* h, int32_t policy, const bisim_mlp* w,
                                       int32_t rescore_every) {
  if (!h || (policy != 0 && policy != 1) || rescore_every < 1 ||
      (policy == 1 && (!w || mlp_features(w) != kPolicyF))) {
    set_error("bisim_set_splitter_policy: policy 0 or 1, rescore_every >= 1, and a 19-input "
              "network for policy 1");
    return BISIM_E_INVALID;
  }
  h->policy = policy;
  h->policy_w = policy ? mlp_weights_bf16(w) : nullptr;
  h->rescore_every = rescore_every;
  return BISIM_OK;
}

bisim_status bisim_collect_training(bisim_lts* h, int64_t sample_every, int32_t max_cands,
                                    float* feat, float* target, int32_t* meta, int64_t cap,
                                    int64_t* rows) {
  if (!h || sample_every < 1 || max_cands < 1 || cap < 0 || !rows ||
      (cap > 0 && (!feat || !target))) {
    set_error("bisim_collect_training: bad arguments");
    return BISIM_E_INVALID;
  }
  *rows = 0;
  int lds_max = 0;
  BISIM_TRY_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock,
                                      h->device));
  const size_t lds = 9 * (size_t)h->n + 64;
  if (!h->uniform || h->n > 16384 || lds + 1024 > (size_t)lds_max) {
    set_error("bisim_collect_training: needs <= 64 actions per state and n <= 16384");
    return BISIM_E_UNSUPPORTED;
  }
  hipStream_t st = h->stream;
  (void)hipFuncSetAttribute((const void*)k_collect, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  (void)hipGetLastError();
  BISIM_TRY(refine_alloc_features(h));
  int64_t cap_it = 3 * (int64_t)h->n - h->pre_blocks + 1;
  if (cap_it < 1) cap_it = 1;
  Args a = make_args(h, (uint32_t)cap_it, false, true);
  a.trace_C = nullptr;
  a.trace_nsplit = nullptr;
  a.trace_work = nullptr;
  BISIM_TRY(refine_init(h, a, 0, false, true, h->pre_block));
  uint32_t* written = nullptr;
  BISIM_TRY_HIP(hipMallocAsync((void**)&written, sizeof(uint32_t), st));
  int64_t r = 0;
  bisim_status rc = BISIM_OK;
  for (uint32_t k = 0;; ++k) {
    if (k % (uint64_t)sample_every == 0 && r < cap) {
      const uint32_t limit = (uint32_t)std::min<int64_t>(max_cands, cap - r);
      hipError_t e = hipMemsetAsync(written, 0, sizeof(uint32_t), st);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_collect, dim3(limit), dim3(256), lds, st, a, k, limit,
                           feat + r * kPolicyF, target + r, meta ? meta + 2 * r : nullptr,
                           written);
        e = hipGetLastError();
      }
      uint32_t w = 0;
      if (e == hipSuccess) e = hipMemcpyAsync(&w, written, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        set_error("bisim_collect_training: %s", hipGetErrorString(e));
        rc = BISIM_E_DEVICE;
        break;
      }
      r += w;
    }
    rc = refine_step_tracked(h, a, k);
    if (rc != BISIM_OK) break;
    hipError_t e = hipMemcpyAsync(&h->ctl_host->state, &h->ctl->state, sizeof(Line),
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
      set_error("bisim_collect_training: %s", hipGetErrorString(e));
      rc = BISIM_E_DEVICE;
      break;
    }
    if (h->ctl_host->state.v[1]) break;
    if ((int64_t)k > cap_it + 1) {
      set_error("bisim_collect_training: refinement did not finish");
      rc = BISIM_E_DEVICE;
      break;
    }
  }
  (void)hipFreeAsync(written, st);
  (void)hipStreamSynchronize(st);
  *rows = r;
  return rc;
}

}  // extern "C"
