// extern "C" entry points declared in include/bisim.h: argument validation,
// handle lifetime, error text, options.
#include <cstdarg>
#include <cstdio>
#include <new>

#include "internal.h"

namespace bisim {
static thread_local char g_err[512] = "";
void clear_error() { g_err[0] = 0; }

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

static void free_handle(bisim_lts* h) {
  if (!h) return;
  hipStream_t s = h->stream;
  lists_free(h);
  void* ptrs[] = {h->init_block, h->pre_block, h->nr_marks, h->in_ptr, h->in_src, h->in_ord, h->woff,
                  h->block,     h->mw,       h->tb,     h->lt,     h->ub,     h->nlw,
                  h->tlist,     h->slist,    h->ctl,    h->sfeat,  h->acc,    h->born,
                  h->used,      h->chg,      h->us,     h->lvl,    h->lvb,    h->lvs,
                  h->lvt,       h->lvq,      h->sb,     h->nlist};
  for (void* p : ptrs)
    if (p) (void)hipFreeAsync(p, s);
  for (void* p : h->sig_buf)
    if (p) (void)hipFreeAsync(p, s);
  (void)hipStreamSynchronize(s);
  if (h->ctl_host) (void)hipHostFree(h->ctl_host);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  for (int i = 0; i < 8 * h->pev_slots; ++i) (void)hipEventDestroy(h->pev[i]);
  delete[] h->pev;
  delete h;
}
// argument checks of lts_load (and of the allocation-free entry point)
bisim_status check_load_args(const int32_t* src, const int32_t* label, const int32_t* dst,
                                    int32_t n, int64_t m, int32_t num_actions, const char* who) {
  if (n < 0 || m < 0 || num_actions < 1) {
    set_error("%s: need n >= 0, m >= 0, num_actions >= 1 (got %d, %lld, %d)", who, n,
              (long long)m, num_actions);
    return BISIM_E_INVALID;
  }
  if (m > 0 && (!src || !label || !dst)) {
    set_error("%s: NULL transition array", who);
    return BISIM_E_INVALID;
  }
  if (m >= 0xFFFFFFFFll || n >= 0x7FFFFFFF) {
    set_error("%s: sizes beyond n < 2^31-1, m < 2^32-1", who);
    return BISIM_E_UNSUPPORTED;
  }
  return BISIM_OK;
}

// Fill a handle whose sizes and stream are set: device and CU count, timing
// events (unless given), preprocessing, and the run state.  Records T_pre.
bisim_status load_into(bisim_lts* h, const int32_t* src, const int32_t* label,
                       const int32_t* dst, const int32_t* init_partition, bool with_run_state) {
  hipError_t e = hipGetDevice(&h->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&h->num_cu, hipDeviceAttributeMultiprocessorCount, h->device);
  if (e == hipSuccess && !h->ev0) e = hipEventCreate(&h->ev0);
  if (e == hipSuccess && !h->ev1) e = hipEventCreate(&h->ev1);
  if (e != hipSuccess) {
    set_error("lts_load: no usable HIP device (%s)", hipGetErrorString(e));
    return BISIM_E_DEVICE;
  }
  BISIM_TRY_HIP(hipEventRecord(h->ev0, h->stream));
  BISIM_TRY(setup_load(h, src, label, dst, init_partition));
  if (with_run_state) BISIM_TRY(refine_alloc(h));
  float ms = 0.f;
  if (hipEventRecord(h->ev1, h->stream) != hipSuccess ||
      hipEventSynchronize(h->ev1) != hipSuccess ||
      hipEventElapsedTime(&ms, h->ev0, h->ev1) != hipSuccess) {
    set_error("lts_load: %s", hipGetErrorString(hipGetLastError()));
    return BISIM_E_DEVICE;
  }
  h->t_pre_ms = ms;
  return BISIM_OK;
}

static bisim_status load_impl(const int32_t* src, const int32_t* label, const int32_t* dst,
                              int32_t n, int64_t m, int32_t num_actions,
                              const int32_t* init_partition, void* hip_stream, bisim_lts** out,
                              bool with_run_state) {
  g_err[0] = 0;
  if (!out) {
    set_error("lts_load: out is NULL");
    return BISIM_E_INVALID;
  }
  *out = nullptr;
  BISIM_TRY(check_load_args(src, label, dst, n, m, num_actions, "lts_load"));
  bisim_lts* h = new (std::nothrow) bisim_lts;
  if (!h) {
    set_error("lts_load: host allocation failed");
    return BISIM_E_NOMEM;
  }
  h->n = n;
  h->m = m;
  h->K = num_actions;
  h->stream = (hipStream_t)hip_stream;
  const bisim_status st = load_into(h, src, label, dst, init_partition, with_run_state);
  if (st != BISIM_OK) {
    free_handle(h);
    return st;
  }
  *out = h;
  return BISIM_OK;
}

// preprocessing only (used by the batched loader for the union of instances)
bisim_status lts_create_union(int32_t n, int64_t m, int32_t K, const int32_t* src,
                              const int32_t* lab, const int32_t* dst, const int32_t* init,
                              hipStream_t stream, bisim_lts** out) {
  return load_impl(src, lab, dst, n, m, K, init, stream, out, false);
}
void lts_destroy(bisim_lts* h) { free_handle(h); }
}  // namespace bisim

using namespace bisim;

extern "C" {

const char* bisim_last_error(void) { return g_err; }

bisim_status lts_load(const int32_t* src, const int32_t* label, const int32_t* dst, int32_t n,
                      int64_t m, int32_t num_actions, const int32_t* init_partition,
                      void* hip_stream, bisim_lts** out) {
  return load_impl(src, label, dst, n, m, num_actions, init_partition, hip_stream, out, true);
}

bisim_status coarsest_partition(bisim_lts* h, int32_t* block_id, bisim_stats* st) {
  g_err[0] = 0;
  if (!h || (!block_id && h->n > 0)) {
    set_error("coarsest_partition: NULL handle or output");
    return BISIM_E_INVALID;
  }
  bisim_status rc = (h->algorithm == BISIM_ALGORITHM_SIGNATURE ||
                     h->algorithm == BISIM_ALGORITHM_HYBRID)
                        ? signature_run(h, block_id, h->algorithm == BISIM_ALGORITHM_HYBRID)
                        : refine_run(h, block_id);
  if (st) {
    st->iterations = h->last_iters;
    st->blocks = h->last_blocks;
    st->pre_blocks = h->run_pre_blocks;
    st->mark_length = h->mark_length;
    st->t_pre_ms = h->t_pre_ms;
    st->t_alg_ms = h->t_alg_ms;
  }
  return rc;
}

void lts_free(bisim_lts* h) { free_handle(h); }

bisim_status bisim_set_option(bisim_lts* h, int32_t option, int64_t value) {
  if (!h) {
    set_error("bisim_set_option: NULL handle");
    return BISIM_E_INVALID;
  }
  switch (option) {
    case BISIM_OPT_ENGINE:
      if (value < 0 || value > 3) break;
      h->engine = (int)value;
      return BISIM_OK;
    case BISIM_OPT_COUNT_WORK:
      if (value != 0 && value != 1) break;
      h->count_work = (int)value;
      return BISIM_OK;
    case BISIM_OPT_FIRST_SPLITTER:
      if (value < -1 || value >= h->n) break;
      h->first_splitter = value;
      return BISIM_OK;
    case BISIM_OPT_ITER_LIMIT:
      if (value < 0) break;
      h->iter_limit = value;
      return BISIM_OK;
    case BISIM_OPT_GRID:
      if (value < 0 || value > (1 << 20)) break;
      h->grid = (int)value;
      return BISIM_OK;
    case BISIM_OPT_PROFILE_EVERY:
      if (value < 0) break;
      h->profile_every = value;
      return BISIM_OK;
    case BISIM_OPT_ALGORITHM:
      if (value != BISIM_ALGORITHM_RCPP && value != BISIM_ALGORITHM_LABELLED &&
          value != BISIM_ALGORITHM_SIGNATURE && value != BISIM_ALGORITHM_HYBRID)
        break;
      if (value == 2 && (h->K != 1 || (h->n > 0 && !h->init_block))) {
        set_error("bisim_set_option: Algorithm 2 needs a one-action LTS (num_actions = 1)");
        return BISIM_E_UNSUPPORTED;
      }
      h->algorithm = (int)value;
      return BISIM_OK;
    default:
      break;
  }
  set_error("bisim_set_option: bad option %d or value %lld", option, (long long)value);
  return BISIM_E_INVALID;
}

bisim_status bisim_set_trace(bisim_lts* h, int32_t* trace_C, int64_t* trace_nsplit,
                             int64_t* trace_work, int64_t cap) {
  if (!h || cap < 0 || (cap > 0 && !trace_C)) {
    set_error("bisim_set_trace: bad arguments");
    return BISIM_E_INVALID;
  }
  h->trace_C = cap ? trace_C : nullptr;
  h->trace_nsplit = cap ? trace_nsplit : nullptr;
  h->trace_work = cap ? trace_work : nullptr;
  h->trace_cap = cap;
  return BISIM_OK;
}

bisim_status bisim_get_phase_times(bisim_lts* h, double* avg_ms, int64_t* samples) {
  if (!h || !avg_ms) {
    set_error("bisim_get_phase_times: NULL argument");
    return BISIM_E_INVALID;
  }
  for (int q = 0; q < 4; ++q) {
    avg_ms[q] = h->phase_cnt[q] ? h->phase_ms[q] / (double)h->phase_cnt[q] : 0.0;
    if (samples) samples[q] = h->phase_cnt[q];
  }
  return BISIM_OK;
}

bisim_status bisim_get_run_config(bisim_lts* h, int32_t* engine, int32_t* grid) {
  if (!h || !engine || !grid) {
    set_error("bisim_get_run_config: NULL argument");
    return BISIM_E_INVALID;
  }
  *engine = h->run_engine;
  *grid = h->run_grid;
  return BISIM_OK;
}

bisim_status bisim_get_work(bisim_lts* h, int64_t* out) {
  if (!h || !out) {
    set_error("bisim_get_work: NULL handle or output");
    return BISIM_E_INVALID;
  }
  for (int i = 0; i < 8; ++i) out[i] = (int64_t)h->lists_work[i];
  return BISIM_OK;
}

bisim_status bisim_get_preprocessed(bisim_lts* h, int32_t* block_id, int32_t* nr_marks) {
  if (!h || (!block_id && h->n > 0)) {
    set_error("bisim_get_preprocessed: NULL handle or output");
    return BISIM_E_INVALID;
  }
  if (h->n > 0) {
    BISIM_TRY_HIP(hipMemcpyAsync(block_id, h->pre_block, sizeof(int32_t) * (size_t)h->n,
                                 hipMemcpyDeviceToDevice, h->stream));
    if (nr_marks)
      BISIM_TRY_HIP(hipMemcpyAsync(nr_marks, h->nr_marks, sizeof(int32_t) * (size_t)h->n,
                                   hipMemcpyDeviceToDevice, h->stream));
  }
  BISIM_TRY_HIP(hipStreamSynchronize(h->stream));
  return BISIM_OK;
}

bisim_status bisim_get_preprocess_method(bisim_lts* h, int32_t* method) {
  if (!h || !method) {
    set_error("bisim_get_preprocess_method: NULL handle or output");
    return BISIM_E_INVALID;
  }
  *method = h->one_pass ? 1 : 0;
  return BISIM_OK;
}

}  // extern "C"
