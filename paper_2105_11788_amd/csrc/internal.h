// Internal declarations shared by the library's translation units: the
// handle layout, the device control block, wave-level helpers for wave64
// (CDNA4), and the host entry points of each stage.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bisim.h"

namespace bisim {

constexpr uint32_t kNone = 0xFFFFFFFFu;  // "no splitter" / +infinity for labels
constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const char* fmt, ...);

#define BISIM_TRY_HIP(expr)                                                                    \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      ::bisim::set_error("%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
      return BISIM_E_DEVICE;                                                                   \
    }                                                                                          \
  } while (0)

#define BISIM_TRY(expr)                \
  do {                                 \
    bisim_status s_ = (expr);          \
    if (s_ != BISIM_OK) return s_;     \
  } while (0)

// ---------------------------------------------------------------------------
// device memory of the library's buffers.  dev_alloc takes stream-ordered
// memory (hipMallocAsync), or, while an ArenaScope is open on the calling
// thread, a 256-byte aligned piece of the scope's region (bump allocation,
// nothing is returned before the scope closes); dev_free releases the former
// and ignores the latter.
// ---------------------------------------------------------------------------
hipError_t dev_alloc(void** p, size_t bytes, hipStream_t s);
hipError_t dev_free(void* p, hipStream_t s);
class ArenaScope {
 public:
  ArenaScope(char* base, size_t capacity);
  ~ArenaScope();
  size_t used() const { return used_; }
  ArenaScope(const ArenaScope&) = delete;
  ArenaScope& operator=(const ArenaScope&) = delete;

 private:
  friend hipError_t dev_alloc(void**, size_t, hipStream_t);
  friend hipError_t dev_free(void*, hipStream_t);
  char* base_;
  size_t cap_, used_ = 0;
  ArenaScope* outer_;
};
// true while an ArenaScope is open on this thread (allocation-free calls)
bool arena_active();

// ---------------------------------------------------------------------------
// device control block of one refinement run.  Fields written by atomics from
// many workgroups sit on their own 128-byte lines.
// ---------------------------------------------------------------------------
struct alignas(128) Line {
  uint32_t v[32];
};
struct Ctl {
  Line cand[2];   // v[0]: splitter for iterations of this parity (min-reduced)
  Line cntT[2];   // v[0]: touched-state list length
  Line cntS[2];   // v[0]: split-state list length
  Line ltany[2];  // v[0]: some block leader was touched
  Line work[2];   // traced runs only: v[0] members of C, v[1] in-transitions of C
  Line cntC[2];   // learned policy: changed (old, new) block pairs this iteration
  // plain policy, two kernels per iteration: counters of iteration k in slot
  // k % 3 (a slot is read up to the iteration after and reset two later)
  Line fS[3];     // v[0]: split states
  Line fL[3];     // v[0]: some block leader was touched
  Line fW[3];     // traced runs only: v[0] members of C, v[1] in-transitions of C,
                  // v[2] touched states
  Line fN[3];     // v[0]: new leaders of the previous iteration's splits
  Line fC[3];     // v[0]: the splitter
  Line state;     // v[0] iterations done, v[1] done flag, v[2] iteration cap hit,
                  // v[3] current splitter, v[4] learned priority structure inconsistent
  Line bar;       // v[0] group arrivals, v[1] generation, v[2] abort
  Line barg[8];   // v[0]: arrivals within workgroup group g (blockIdx % 8)
};

// ---------------------------------------------------------------------------
// wave helpers (wave64)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t lane() { return __lane_id(); }

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, d, kWave));
  return v;
}

__device__ __forceinline__ uint32_t wave_incl_scan_u32(uint32_t v) {
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    uint32_t t = (uint32_t)__shfl_up((int)v, d, kWave);
    if ((int)lane() >= d) v += t;
  }
  return v;
}

// Append `val` to list for every lane with pred; one atomic per wave.  Must
// be reached by all active lanes of the wave.
__device__ __forceinline__ void wave_push(int32_t* list, uint32_t* counter, int32_t val,
                                          bool pred) {
  uint64_t bal = __ballot(pred);
  if (bal == 0) return;
  int leader = __ffsll((unsigned long long)bal) - 1;
  uint32_t base = 0;
  if ((int)lane() == leader) base = atomicAdd(counter, (uint32_t)__popcll(bal));
  base = (uint32_t)__shfl((int)base, leader, kWave);
  if (pred) list[base + __popcll(bal & ((1ull << lane()) - 1ull))] = val;
}

__device__ __forceinline__ bool test_bit(const uint64_t* bm, uint32_t i) {
  return (bm[i >> 6] >> (i & 63)) & 1ull;
}

// Scans of block[] over all states take U chunks of 64 states per wave and
// step, loading all of them before testing any (U > 1 pays where one
// workgroup scans a large instance in global memory).
// bit u set: state base0 + 64u + lane exists (< n) and block[state] == C
template <uint32_t U>
__device__ __forceinline__ uint32_t hit_mask(const int32_t* blk, uint32_t base0, uint32_t n,
                                             uint32_t C) {
  int32_t v[U];
#pragma unroll
  for (uint32_t u = 0; u < U; ++u) {
    const uint32_t t = base0 + u * kWave + lane();
    v[u] = t < n ? blk[t] : -1;
  }
  uint32_t m = 0;
#pragma unroll
  for (uint32_t u = 0; u < U; ++u) m |= ((uint32_t)v[u] == C ? 1u : 0u) << u;
  return m;
}

// ---------------------------------------------------------------------------
// the handle
// ---------------------------------------------------------------------------
}  // namespace bisim

// device arrays of the member-list engine (engine 3), allocated on first use
struct bisim_lists {
  int32_t *perm = nullptr, *pos = nullptr, *bs = nullptr, *be = nullptr;
  int32_t *cnt = nullptr, *fc = nullptr, *gc = nullptr, *tcn = nullptr;
  uint64_t* tmp64 = nullptr;
  uint64_t* pin = nullptr;  // in-transition range by member-list position
  uint32_t* pf = nullptr;   // the next splitter, prefetched (two slots)
  int32_t *lb = nullptr, *lo = nullptr, *lh = nullptr;
  int32_t *ts = nullptr, *tbk = nullptr;
  int32_t *ss = nullptr, *sbk = nullptr, *sr = nullptr, *sfi = nullptr, *sne = nullptr,
          *sps = nullptr, *sse = nullptr;
  uint64_t* work = nullptr;
  // the captured graph of a chunk of iterations and the arguments it holds
  hipGraphExec_t gexec = nullptr;
  unsigned char gargs[512] = {};
  int ggrid = 0;
  hipStream_t own = nullptr;  // capture stream when the handle's stream is the null stream
};

struct bisim_lts {
  int32_t n = 0;
  int64_t m = 0;
  int32_t K = 1;
  hipStream_t stream = nullptr;
  int device = 0;
  int num_cu = 0;

  // preprocessed, immutable after load
  int32_t* pre_block = nullptr;  // [n] pi_pre, canonical
  int32_t* init_block = nullptr; // [n] leader-normalised pi_0 (one-action LTSs: Algorithm 2)
  int32_t* nr_marks = nullptr;   // [n] distinct outgoing actions per state
  uint32_t* in_ptr = nullptr;    // [n+1] transitions grouped by target
  int32_t* in_src = nullptr;     // [m] source of each grouped transition
  int32_t* in_ord = nullptr;     // [m] its action's rank among the source's actions
  uint32_t* woff = nullptr;      // [n+1] mark-word offsets (only when !uniform)
  int uniform = 1;               // every state has <= 64 actions: word index = state
  uint32_t max_out = 0;          // largest number of outgoing transitions of a state
  bool one_pass = false;         // pi_pre and the action ranks came from the one-pass kernels
  uint32_t max_ranks = 0;        // largest number of distinct actions of a state
  uint64_t nwords = 0;
  int64_t pre_blocks = 0;
  int64_t mark_length = 0;

  // per-run working set
  // (mw, tb, lt and sb hold two halves, one per iteration parity, for the
  // two-step plain engine; the three-step path uses the first half)
  int32_t* block = nullptr;  // [n]
  uint64_t* mw = nullptr;    // [2][nwords] packed marks
  uint64_t* tb = nullptr;    // [2][ceil(n/64)] touched states
  uint64_t* lt = nullptr;    // [2][ceil(n/64)] touched leaders
  uint64_t* sb = nullptr;    // [2][ceil(n/64)] split states (two-kernel engine)
  uint64_t* ub = nullptr;    // [ceil(n/64)] unstable block labels
  uint64_t* us = nullptr;    // [ceil(n/4096)] summary: bit w set iff ub[w] != 0
  uint64_t* nlw = nullptr;   // [n] (epoch << 32) | ~state, max-reduced
  int32_t* tlist = nullptr;  // [n]
  int32_t* slist = nullptr;  // [n]
  int32_t* nlist = nullptr;  // [n] new leaders (two-kernel engine)
  bisim::Ctl* ctl = nullptr;
  bisim::Ctl* ctl_host = nullptr;  // pinned mirror

  // options
  int engine = 0;
  int algorithm = 3;  // 3: labelled (Algorithm 3); 2: one-action RCPP (Algorithm 2)
  int64_t run_pre_blocks = 0;  // blocks the last run started from
  const int32_t* start_override = nullptr;  // device: a partition refining pi_pre to start from
  int64_t start_override_blocks = 0;
  int64_t first_splitter = -1;
  int64_t iter_limit = 0;
  int grid = 0;
  int32_t* trace_C = nullptr;
  int64_t* trace_nsplit = nullptr;
  int64_t* trace_work = nullptr;
  int64_t trace_cap = 0;

  // block features and the learned splitter policy
  uint32_t* sfeat = nullptr;  // [n][16] out/in transitions of each state by label mod 8
  uint32_t* acc = nullptr;    // [n][17] per block label: size, out[8], in[8]
  uint32_t* born = nullptr;   // [n] iteration the block was created / last split
  uint32_t* used = nullptr;   // [n] iteration the block was last the splitter
  int32_t* chg = nullptr;     // [2n] (old, new) label pairs of this iteration's splits
  uint8_t* lvl = nullptr;     // [n] priority level of each unstable label (learned policy)
  uint64_t* lvb = nullptr;    // [16][ceil(n/64)] unstable labels by level
  uint64_t* lvs = nullptr;    // [16][ceil(n/4096)] non-empty words of lvb
  uint64_t* lvt = nullptr;    // [16][ceil(n/262144)] non-empty words of lvs
  uint8_t* lvq = nullptr;     // [2n+1] scratch of the re-scoring step
  int policy = 0;
  const uint16_t* policy_w = nullptr;  // bf16 network parameters (18 inputs)
  int rescore_every = 64;

  // sampled phase timing (per-phase engine)
  int64_t profile_every = 0;
  hipEvent_t* pev = nullptr;  // 8 events per sampled iteration
  int pev_slots = 0;
  double phase_ms[4] = {0, 0, 0, 0};
  int64_t phase_cnt[4] = {0, 0, 0, 0};

  // engine and grid of the last run (engine 0 resolves to the tuner's choice)
  int run_engine = 0;
  int run_grid = 0;

  // signature rounds: the run's device buffers, kept from the first such run
  // to lts_free (slot k holds the k-th buffer a run asks for; a slot too
  // small for a request is reallocated)
  static constexpr int kSigSlots = 24;
  void* sig_buf[kSigSlots] = {};
  size_t sig_bytes[kSigSlots] = {};

  // member-list engine
  bisim_lists lists;
  int count_work = 0;            // accumulate the engine's work totals
  uint64_t lists_work[8] = {0, 0, 0, 0, 0, 0, 0, 0};

  double t_pre_ms = 0.0;
  double t_alg_ms = 0.0;
  int64_t last_iters = 0;
  int64_t last_blocks = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace bisim {
// abi.hip
void clear_error();
bisim_status check_load_args(const int32_t* src, const int32_t* label, const int32_t* dst,
                             int32_t n, int64_t m, int32_t num_actions, const char* who);
bisim_status load_into(bisim_lts* h, const int32_t* src, const int32_t* label,
                       const int32_t* dst, const int32_t* init_partition, bool with_run_state);
// scan.hip: out[0..count] = exclusive prefix sums of in[0..count), out[count] = total
bisim_status exclusive_scan_u32(const uint32_t* in, uint32_t* out, int64_t count,
                                hipStream_t stream);
// upper bound of the device memory exclusive_scan_u32 takes for `count`
// values (as dev_alloc counts it: each piece rounded up to 256 bytes)
size_t exclusive_scan_scratch_bytes(int64_t count);
// sort.hip: stable least-significant-digit radix sort of 64-bit keys by bits
// [begin_bit, end_bit), carrying 32-bit values when vals_in is not NULL
// (keys_in and vals_in are left as they were; temp holds
// radix_sort_temp_bytes(count, vals_in != NULL) bytes), and an inclusive
// max-scan over uint32
size_t radix_sort_temp_bytes(int64_t count, bool with_values);
bisim_status radix_sort_u64(void* temp, size_t temp_bytes, const uint64_t* keys_in,
                            uint64_t* keys_out, const uint32_t* vals_in, uint32_t* vals_out,
                            int64_t count, int begin_bit, int end_bit, hipStream_t stream);
bisim_status inclusive_max_scan_u32(const uint32_t* in, uint32_t* out, int64_t count,
                                    hipStream_t stream);
// setup.hip
bisim_status setup_load(bisim_lts* h, const int32_t* src, const int32_t* lab,
                        const int32_t* dst, const int32_t* init);
// refine.hip
bisim_status refine_run(bisim_lts* h, int32_t* block_id);
bisim_status refine_alloc(bisim_lts* h);
// signature.hip: multi-way signature refinement (baseline), or signature
// rounds followed by Algorithm 3 (hybrid)
bisim_status signature_run(bisim_lts* h, int32_t* block_id, bool hybrid);
// lists.hip: the member-list engine (engine 3)
bisim_status lists_alloc(bisim_lts* h);
bisim_status lists_loop(bisim_lts* h, uint32_t cap, bool count_work_totals);
void lists_free(bisim_lts* h);
}  // namespace bisim

struct bisim_mlp;
namespace bisim {
// mlp.hip
const uint16_t* mlp_weights_bf16(const bisim_mlp* w);
int mlp_features(const bisim_mlp* w);
}  // namespace bisim
