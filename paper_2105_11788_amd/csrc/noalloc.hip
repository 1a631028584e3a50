// Allocation-free form of lts_load + coarsest_partition + lts_free, for
// callers that cannot allocate device memory.  Every buffer the loading and
// refinement kernels use (preprocessed arrays, temporaries, the run's
// working set) is carved out of one file-scope device array, `scratch`, of a
// fixed size; each GPU holds its own copy of it until the process ends.  The
// same kernels run as for the handle-based calls.
#include <mutex>

#include "internal.h"

namespace bisim {
namespace {

constexpr size_t kScratchBytes = (size_t)BISIM_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
struct DevScratch {
  char* ptr = nullptr;  // the device's address of `scratch`
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};
DevScratch g_dev[kMaxDevices];
std::mutex g_mu;

// Once per device, with that device current: the device address of the
// array (its name in host code is a host-side stand-in), and two timing
// events.
bisim_status scratch_for(int dev, DevScratch** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  DevScratch& d = g_dev[dev];
  if (!d.ptr) {
    void* p = nullptr;
    BISIM_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || ((uintptr_t)p & 255)) {
      set_error("coarsest_partition_noalloc: bad scratch address");
      return BISIM_E_DEVICE;
    }
    if (!d.ev0) BISIM_TRY_HIP(hipEventCreate(&d.ev0));
    if (!d.ev1) BISIM_TRY_HIP(hipEventCreate(&d.ev1));
    d.ptr = (char*)p;
  }
  *out = &d;
  return BISIM_OK;
}

// Upper bound of what loading and one plain refinement take from the region
// for n states, m transitions and K actions: every allocation of the
// preprocessing (section 4.1) and of the run state, each rounded up to 256
// bytes as dev_alloc places it.  Data-dependent sizes take their maxima (the
// mark-word offsets of states with more than 64 actions, at most n + m/64
// mark words).
size_t noalloc_bytes(int64_t n, int64_t m, int64_t K) {
  size_t need = 0;
  auto add = [&](int64_t bytes) { need += ((size_t)(bytes > 0 ? bytes : 1) + 255) / 256 * 256; };
  const int64_t nwd = (n + 63) / 64;
  // preprocessing: validation flag, persistent arrays, temporaries
  add(4);
  add(4 * n);            // pre_block
  add(4 * n);            // nr_marks
  add(4 * (n + 1));      // in_ptr
  add(4 * m);            // in_src
  add(4 * m);            // in_ord
  add(4 * m);            // action ranks
  add(4 * K);            // bucket counts
  add(4 * (K + 1));      // bucket offsets
  add(4 * ((K > n ? K : n) + 1));  // cursors
  add(4 * m);            // transitions by action
  add(4 * n);            // leaders of pi_0
  add(16);
  add(8);
  add(n);                // has an a-transition
  add(n);                // split flags
  add(8 * n);            // bids
  need += exclusive_scan_scratch_bytes(K);
  if (K == 1) add(4 * n);  // pi_0 kept for Algorithm 2
  add(4 * n);            // mark words per state
  add(4 * (n + 1));      // mark-word offsets
  need += exclusive_scan_scratch_bytes(n);
  add(4 * n);            // degrees
  need += exclusive_scan_scratch_bytes(n);
  // run state
  const int64_t nwords = n + m / 64 + 1;
  add(4 * n);            // block
  add(16 * nwords);      // marks, two halves
  add(16 * nwd);         // touched
  add(16 * nwd);         // touched leaders
  add(16 * nwd);         // split flags
  add(4 * n);            // new leaders
  add(8 * nwd);          // unstable labels
  add(8 * ((nwd + 63) / 64));
  add(8 * n);            // bids
  add(4 * n);            // touched list
  add(4 * n);            // split list
  add((int64_t)sizeof(Ctl));
  for (int i = 0; i < 4; ++i) add(8);  // block counts
  return need;
}

}  // namespace
}  // namespace bisim

using namespace bisim;

extern "C" bisim_status coarsest_partition_noalloc(const int32_t* src, const int32_t* label,
                                                   const int32_t* dst, int32_t n, int64_t m,
                                                   int32_t num_actions,
                                                   const int32_t* init_partition,
                                                   int32_t* block_id, bisim_stats* st,
                                                   void* hip_stream) {
  clear_error();
  const char* who = "coarsest_partition_noalloc";
  BISIM_TRY(check_load_args(src, label, dst, n, m, num_actions, who));
  if (!block_id && n > 0) {
    set_error("%s: NULL block_id", who);
    return BISIM_E_INVALID;
  }
  const size_t need = noalloc_bytes(n, m, num_actions);
  if (need > kScratchBytes) {
    set_error("%s: an LTS of n=%d, m=%lld, K=%d needs up to %zu bytes of working memory; the "
              "static region holds %zu (use lts_load + coarsest_partition)",
              who, n, (long long)m, num_actions, need, kScratchBytes);
    return BISIM_E_UNSUPPORTED;
  }
  int dev = 0;
  BISIM_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("%s: device %d beyond the supported %d", who, dev, kMaxDevices);
    return BISIM_E_UNSUPPORTED;
  }
  DevScratch* d = nullptr;
  BISIM_TRY(scratch_for(dev, &d));

  // a handle on the stack whose memory all comes from the region; nothing in
  // it is freed (the region is reused by the next call on this device)
  bisim_lts h;
  Ctl mirror;  // host copy of the control block (pageable)
  h.n = n;
  h.m = m;
  h.K = num_actions;
  h.stream = (hipStream_t)hip_stream;
  h.ev0 = d->ev0;
  h.ev1 = d->ev1;
  h.ctl_host = &mirror;
  bisim_status rc;
  {
    ArenaScope arena(d->ptr, kScratchBytes);
    rc = load_into(&h, src, label, dst, init_partition, true);
    const double t_pre = h.t_pre_ms;
    if (rc == BISIM_OK) rc = refine_run(&h, block_id);
    h.t_pre_ms = t_pre;
    if (arena.used() > need && rc == BISIM_OK) {  // the bound above must hold
      set_error("%s: working memory %zu exceeded its bound %zu", who, arena.used(), need);
      rc = BISIM_E_DEVICE;
    }
  }
  if (rc == BISIM_E_NOMEM) {
    set_error("%s: the static region (%zu bytes) was exhausted", who, kScratchBytes);
    rc = BISIM_E_UNSUPPORTED;
  }
  if (st) {
    st->iterations = h.last_iters;
    st->blocks = h.last_blocks;
    st->pre_blocks = h.run_pre_blocks;
    st->mark_length = h.mark_length;
    st->t_pre_ms = h.t_pre_ms;
    st->t_alg_ms = h.t_alg_ms;
  }
  return rc;
}
