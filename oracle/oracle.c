/*
 * Sequential CPU oracle for strong bisimulation (relational coarsest partition).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP implementation.
 *
 * Problem (section 2): given an LTS (S, Act, ->) and an initial partition
 * pi_0, the result is the coarsest refinement of pi_0 whose induced relation
 * is a strong bisimulation (Definition 2).  It is unique, and every routine
 * below that produces a partition emits it canonically: the block id of a
 * state is the smallest state of its block.
 *
 * Routines
 *   orc_ks_coarsest   Kanellakis-Smolka refinement with an explicit set of
 *                     possibly-unstable splitters (section 3.1, Algorithm 1),
 *                     generalised to labels by splitting on every action's
 *                     pre-image of the splitter.  Reading of Algorithm 1: the
 *                     block removed from pi when B' splits is B' itself, not
 *                     the splitter B.  This is the timed CPU baseline.
 *   orc_preprocess    The preprocessing of section 4.1 for the labelled
 *                     algorithm: transitions sorted by (source, action),
 *                     action_switch (Algorithm 5), order (inclusive segmented
 *                     scan of action_switch), nr_marks (last order + 1, or 0
 *                     for a state with no transitions), off (exclusive scan of
 *                     nr_marks) and mark_length; plus pi_pre, the split of the
 *                     leader-normalised pi_0 by outgoing action sets done one
 *                     action at a time (Algorithm 4).
 *   orc_alg3          Lock-step simulation of the labelled PRAM algorithm
 *                     (Algorithm 3) after that preprocessing, or of the
 *                     unlabelled one (Algorithm 2, section 3.2), under these
 *                     readings of the concurrent writes:
 *                       - priority CRCW: the splitter C is the smallest
 *                         unstable block label, a concurrent new_leader write
 *                         is won by the smallest state, and the initial leader
 *                         of a pi_0 block is its smallest member;
 *                       - within one step every "unstable := false" write
 *                         precedes every "unstable := true" write;
 *                       - the iteration count includes the final pass that
 *                         finds no splitter (Table 1's #It).
 *                     Emits the iteration count, the splitter sequence, the
 *                     number of states split per iteration and optionally the
 *                     partition after every iteration.
 *   orc_check_*       Checkers: stability (section 2, "stable"), refinement
 *                     of pi_0, canonical labelling.
 *
 * Parity pins (see tests): brute-force greatest-fixpoint bisimulation and
 * exhaustive partition enumeration on tiny LTSs, the arrays printed for
 * Figure 2, the single iteration drawn in Figure 1, hand-derived closed forms
 * for Fan_out_n and the tail-labelled chain, the iteration bounds of
 * Theorems 2 and 3, and lifted planted quotients.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_E_INVALID (-1)
#define ORC_E_RANGE (-2)
#define ORC_E_NOMEM (-3)

static int validate(int32_t n, int64_t m, int32_t K, const int32_t* src, const int32_t* lab,
                    const int32_t* dst, const int32_t* init) {
  if (n < 0 || m < 0 || K < 1) return ORC_E_INVALID;
  if (m > 0 && (!src || !lab || !dst)) return ORC_E_INVALID;
  for (int64_t i = 0; i < m; ++i) {
    if (src[i] < 0 || src[i] >= n || dst[i] < 0 || dst[i] >= n) return ORC_E_RANGE;
    if (lab[i] < 0 || lab[i] >= K) return ORC_E_RANGE;
  }
  if (init)
    for (int32_t s = 0; s < n; ++s)
      if (init[s] < 0 || init[s] >= n) return ORC_E_RANGE;
  return 0;
}

/* ======================================================================== */
/* Kanellakis-Smolka with a splitter worklist                                */
/* ======================================================================== */
int64_t orc_ks_coarsest(int32_t n, int64_t m, int32_t K, const int32_t* src, const int32_t* lab,
                        const int32_t* dst, const int32_t* init, int32_t* out_block) {
  int rc = validate(n, m, K, src, lab, dst, init);
  if (rc) return rc;
  if (n == 0) return 0;

  /* reverse index: transitions grouped by target */
  int64_t* rptr = calloc((size_t)n + 1, sizeof(int64_t));
  int32_t* rsrc = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
  int32_t* rlab = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
  /* refinable partition: each block's states are contiguous in elems */
  int32_t* blk = malloc(sizeof(int32_t) * (size_t)n);
  int32_t* elems = malloc(sizeof(int32_t) * (size_t)n);
  int64_t* pos = malloc(sizeof(int64_t) * (size_t)n);
  int64_t* bbeg = malloc(sizeof(int64_t) * (size_t)n);
  int64_t* bend = malloc(sizeof(int64_t) * (size_t)n);
  int64_t* mcnt = calloc((size_t)n, sizeof(int64_t));
  int32_t* idmap = malloc(sizeof(int32_t) * (size_t)n);
  int32_t* work = malloc(sizeof(int32_t) * (size_t)n);
  char* inwork = calloc((size_t)n, 1);
  int32_t* snap = malloc(sizeof(int32_t) * (size_t)n);
  int32_t* plab = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
  int32_t* psrc = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
  int32_t* gsrc = malloc(sizeof(int32_t) * (size_t)(m ? m : 1));
  int64_t* lcnt = calloc((size_t)K, sizeof(int64_t));
  int32_t* touched_lab = malloc(sizeof(int32_t) * (size_t)(K < m ? K : (m ? m : 1)));
  int64_t* tl_beg = malloc(sizeof(int64_t) * (size_t)(K < m ? K : (m ? m : 1)));
  int64_t* stamp = calloc((size_t)n, sizeof(int64_t));
  int32_t* touched_blk = malloc(sizeof(int32_t) * (size_t)n);
  int32_t* minm = malloc(sizeof(int32_t) * (size_t)n);
  if (!rptr || !rsrc || !rlab || !blk || !elems || !pos || !bbeg || !bend || !mcnt || !idmap ||
      !work || !inwork || !snap || !plab || !psrc || !gsrc || !lcnt || !touched_lab || !tl_beg ||
      !stamp || !touched_blk || !minm) {
    rc = ORC_E_NOMEM;
    goto done;
  }
  for (int64_t i = 0; i < m; ++i) rptr[dst[i] + 1]++;
  for (int32_t s = 0; s < n; ++s) rptr[s + 1] += rptr[s];
  {
    int64_t* cur = malloc(sizeof(int64_t) * (size_t)n);
    if (!cur) { rc = ORC_E_NOMEM; goto done; }
    memcpy(cur, rptr, sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < m; ++i) {
      int64_t p = cur[dst[i]]++;
      rsrc[p] = src[i];
      rlab[p] = lab[i];
    }
    free(cur);
  }

  /* pi_0: one block per distinct init value */
  int32_t nb = 0;
  for (int32_t v = 0; v < n; ++v) idmap[v] = -1;
  for (int32_t s = 0; s < n; ++s) {
    int32_t v = init ? init[s] : 0;
    if (idmap[v] < 0) idmap[v] = nb++;
    blk[s] = idmap[v];
  }
  for (int32_t b = 0; b < nb; ++b) bbeg[b] = 0;
  for (int32_t s = 0; s < n; ++s) bbeg[blk[s]]++;
  {
    int64_t acc = 0;
    for (int32_t b = 0; b < nb; ++b) {
      int64_t c = bbeg[b];
      bbeg[b] = acc;
      bend[b] = acc;
      acc += c;
    }
  }
  for (int32_t s = 0; s < n; ++s) {
    int64_t p = bend[blk[s]]++;
    elems[p] = s;
    pos[s] = p;
  }

  int64_t nwork = 0;
  for (int32_t b = 0; b < nb; ++b) {
    work[nwork++] = b;
    inwork[b] = 1;
  }
  int64_t cur_stamp = 0;

  while (nwork > 0) {
    int32_t B = work[--nwork];
    inwork[B] = 0;
    /* snapshot of the splitter's members: its later splits do not change
       the set being split on */
    int64_t bs = bend[B] - bbeg[B];
    memcpy(snap, elems + bbeg[B], sizeof(int32_t) * (size_t)bs);
    /* in-transitions of the splitter, grouped by action */
    int64_t x = 0;
    for (int64_t k = 0; k < bs; ++k) {
      int32_t t = snap[k];
      for (int64_t j = rptr[t]; j < rptr[t + 1]; ++j) {
        plab[x] = rlab[j];
        psrc[x] = rsrc[j];
        ++x;
      }
    }
    int64_t ntl = 0;
    for (int64_t i = 0; i < x; ++i)
      if (lcnt[plab[i]]++ == 0) touched_lab[ntl++] = plab[i];
    {
      int64_t acc = 0;
      for (int64_t k = 0; k < ntl; ++k) {
        int32_t a = touched_lab[k];
        int64_t c = lcnt[a];
        lcnt[a] = acc;
        tl_beg[k] = acc;
        acc += c;
      }
    }
    for (int64_t i = 0; i < x; ++i) gsrc[lcnt[plab[i]]++] = psrc[i];

    for (int64_t k = 0; k < ntl; ++k) {
      int32_t a = touched_lab[k];
      int64_t g0 = tl_beg[k], g1 = lcnt[a];
      lcnt[a] = 0;
      /* S' = sources reaching the splitter with action a; move each to the
         front of its block */
      ++cur_stamp;
      int64_t ntb = 0;
      for (int64_t i = g0; i < g1; ++i) {
        int32_t s = gsrc[i];
        if (stamp[s] == cur_stamp) continue;
        stamp[s] = cur_stamp;
        int32_t b = blk[s];
        int64_t to = bbeg[b] + mcnt[b];
        int32_t other = elems[to];
        int64_t from = pos[s];
        elems[to] = s;
        pos[s] = to;
        elems[from] = other;
        pos[other] = from;
        if (mcnt[b]++ == 0) touched_blk[ntb++] = b;
      }
      /* split every B' with empty < B' n S' < B' */
      for (int64_t i = 0; i < ntb; ++i) {
        int32_t b = touched_blk[i];
        int64_t c = mcnt[b];
        mcnt[b] = 0;
        if (c == bend[b] - bbeg[b]) continue;
        int32_t nbk = nb++;
        bbeg[nbk] = bbeg[b];
        bend[nbk] = bbeg[b] + c;
        bbeg[b] += c;
        for (int64_t p = bbeg[nbk]; p < bend[nbk]; ++p) blk[elems[p]] = nbk;
        if (!inwork[b]) {
          work[nwork++] = b;
          inwork[b] = 1;
        }
        work[nwork++] = nbk;
        inwork[nbk] = 1;
      }
    }
  }

  for (int32_t b = 0; b < nb; ++b) minm[b] = n;
  for (int32_t s = 0; s < n; ++s)
    if (s < minm[blk[s]]) minm[blk[s]] = s;
  for (int32_t s = 0; s < n; ++s) out_block[s] = minm[blk[s]];
  rc = 0;

done:
  free(rptr); free(rsrc); free(rlab); free(blk); free(elems); free(pos); free(bbeg); free(bend);
  free(mcnt); free(idmap); free(work); free(inwork); free(snap); free(plab); free(psrc);
  free(gsrc); free(lcnt); free(touched_lab); free(tl_beg); free(stamp); free(touched_blk);
  free(minm);
  return rc ? rc : nb;
}

/* ======================================================================== */
/* Preprocessing of section 4.1                                              */
/* ======================================================================== */
/* Stable counting sort of the permutation `idx` by key[idx[i]] in [0, range). */
static int stable_count_sort(int64_t m, int32_t range, const int32_t* key, int32_t* idx,
                             int32_t* tmp) {
  int64_t* cnt = calloc((size_t)range + 1, sizeof(int64_t));
  if (!cnt) return ORC_E_NOMEM;
  for (int64_t i = 0; i < m; ++i) cnt[key[idx[i]] + 1]++;
  for (int32_t r = 0; r < range; ++r) cnt[r + 1] += cnt[r];
  for (int64_t i = 0; i < m; ++i) tmp[cnt[key[idx[i]]]++] = idx[i];
  memcpy(idx, tmp, sizeof(int32_t) * (size_t)m);
  free(cnt);
  return 0;
}

/*
 * Outputs (all caller-allocated; any may be NULL):
 *   s_src, s_lab, s_dst [m]  transitions sorted by (source, action)
 *   action_switch, order [m]
 *   nr_marks [n], off [n]    (off = exclusive prefix sum of nr_marks)
 *   mark_length [1]
 *   pre_block [n]            pi_pre (canonical)
 * Returns the number of blocks of pi_pre, or < 0 on error.
 */
int64_t orc_preprocess(int32_t n, int64_t m, int32_t K, const int32_t* src, const int32_t* lab,
                       const int32_t* dst, const int32_t* init, int32_t* s_src, int32_t* s_lab,
                       int32_t* s_dst, int32_t* action_switch, int32_t* order, int32_t* nr_marks,
                       int64_t* off, int64_t* mark_length, int32_t* pre_block) {
  int rc = validate(n, m, K, src, lab, dst, init);
  if (rc) return rc;
  size_t mm = (size_t)(m ? m : 1), nn = (size_t)(n ? n : 1);
  int32_t* idx = malloc(sizeof(int32_t) * mm);
  int32_t* tmp = malloc(sizeof(int32_t) * mm);
  int32_t* sw = malloc(sizeof(int32_t) * mm);
  int32_t* ord = malloc(sizeof(int32_t) * mm);
  int32_t* nrm = calloc(nn, sizeof(int32_t));
  int32_t* block = malloc(sizeof(int32_t) * nn);
  int32_t* newl = malloc(sizeof(int32_t) * nn);
  char* has = calloc(nn, 1);
  char* spl = calloc(nn, 1);
  int64_t nblocks = 0;
  if (!idx || !tmp || !sw || !ord || !nrm || !block || !newl || !has || !spl) {
    rc = ORC_E_NOMEM;
    goto done;
  }
  for (int64_t i = 0; i < m; ++i) idx[i] = (int32_t)i;
  /* sort by (source, action): stable sort by action, then by source */
  if (m && ((rc = stable_count_sort(m, K, lab, idx, tmp)) || (rc = stable_count_sort(m, n, src, idx, tmp))))
    goto done;
  /* Algorithm 5 (loop over 0 <= i < m) */
  for (int64_t i = 0; i < m; ++i) {
    int32_t s = src[idx[i]], a = lab[idx[i]];
    if (i == 0 || s != src[idx[i - 1]] || a == lab[idx[i - 1]])
      sw[i] = 0;
    else
      sw[i] = 1;
  }
  /* order: inclusive scan of action_switch, restarted at every source */
  for (int64_t i = 0; i < m; ++i) {
    int new_seg = (i == 0 || src[idx[i]] != src[idx[i - 1]]);
    ord[i] = new_seg ? sw[i] : ord[i - 1] + sw[i];
  }
  /* nr_marks: 1 + (sum of action_switch over the source's transitions), i.e.
     the number of distinct actions; 0 for a state without transitions */
  for (int64_t i = 0; i < m; ++i) nrm[src[idx[i]]] = ord[i] + 1;
  {
    int64_t acc = 0;
    for (int32_t s = 0; s < n; ++s) {
      if (off) off[s] = acc;
      acc += nrm[s];
    }
    if (mark_length) *mark_length = acc;
  }
  for (int64_t i = 0; i < m; ++i) {
    if (s_src) s_src[i] = src[idx[i]];
    if (s_lab) s_lab[i] = lab[idx[i]];
    if (s_dst) s_dst[i] = dst[idx[i]];
    if (action_switch) action_switch[i] = sw[i];
    if (order) order[i] = ord[i];
  }
  if (nr_marks) memcpy(nr_marks, nrm, sizeof(int32_t) * (size_t)n);

  /* leaders of pi_0: new_leader[I_i] := i with the smallest i winning */
  for (int32_t v = 0; v < n; ++v) newl[v] = n;
  for (int32_t s = 0; s < n; ++s) {
    int32_t v = init ? init[s] : 0;
    if (s < newl[v]) newl[v] = s;
  }
  for (int32_t s = 0; s < n; ++s) block[s] = newl[init ? init[s] : 0];
  /* Algorithm 4: one split round per action a = 0..K-1 */
  for (int32_t a = 0; a < K; ++a) {
    memset(has, 0, (size_t)n);
    for (int64_t i = 0; i < m; ++i)
      if (lab[i] == a) has[src[i]] = 1;
    for (int32_t s = 0; s < n; ++s) newl[s] = n;
    for (int32_t s = 0; s < n; ++s) {
      spl[s] = has[s] != has[block[s]];
      if (spl[s] && s < newl[block[s]]) newl[block[s]] = s;
    }
    for (int32_t s = 0; s < n; ++s)
      if (spl[s]) block[s] = newl[block[s]];
  }
  for (int32_t s = 0; s < n; ++s) nblocks += (block[s] == s);
  if (pre_block) memcpy(pre_block, block, sizeof(int32_t) * (size_t)n);
  rc = 0;
done:
  free(idx); free(tmp); free(sw); free(ord); free(nrm); free(block); free(newl); free(has);
  free(spl);
  return rc ? rc : nblocks;
}

/* ======================================================================== */
/* Lock-step simulation of Algorithm 3 (variant 3) or Algorithm 2 (variant 2) */
/* ======================================================================== */
/*
 * out_block [n]      final partition (canonical under the priority reading)
 * out_pre_blocks     number of blocks the loop starts from
 * trace_cap          capacity of the trace arrays (iterations)
 * trace_C            splitter per iteration (-1 for the final pass)
 * trace_nsplit       states split per iteration
 * trace_blocks       trace_cap x n partition after each iteration (nullable)
 * force_first_C      >= 0: use this unstable block label as the first splitter
 * max_iters          > 0: stop after this many iterations (returns -4 if hit)
 * variant            3 = Algorithm 3 (labelled, with preprocessing);
 *                    2 = Algorithm 2 (labels ignored, one mark per state)
 * Returns the iteration count #It (including the final pass), or < 0.
 */
int64_t orc_alg3(int32_t n, int64_t m, int32_t K, const int32_t* src, const int32_t* lab,
                 const int32_t* dst, const int32_t* init, int32_t* out_block,
                 int64_t* out_pre_blocks, int64_t trace_cap, int32_t* trace_C,
                 int64_t* trace_nsplit, int32_t* trace_blocks, int32_t force_first_C,
                 int64_t max_iters, int32_t variant) {
  int rc = validate(n, m, K, src, lab, dst, init);
  if (rc) return rc;
  if (variant != 2 && variant != 3) return ORC_E_INVALID;
  size_t mm = (size_t)(m ? m : 1), nn = (size_t)(n ? n : 1);
  int32_t* ssrc = malloc(sizeof(int32_t) * mm);
  int32_t* sdst = malloc(sizeof(int32_t) * mm);
  int32_t* ord = malloc(sizeof(int32_t) * mm);
  int64_t* off = malloc(sizeof(int64_t) * nn);
  int32_t* block = malloc(sizeof(int32_t) * nn);
  int32_t* newl = malloc(sizeof(int32_t) * nn);
  char* unstable = calloc(nn, 1);
  char* split = calloc(nn, 1);
  char* mark = NULL;
  int64_t L = 0, iters = 0;
  if (!ssrc || !sdst || !ord || !off || !block || !newl || !unstable || !split) {
    rc = ORC_E_NOMEM;
    goto done;
  }
  if (variant == 3) {
    int64_t nbp = orc_preprocess(n, m, K, src, lab, dst, init, ssrc, NULL, sdst, NULL, ord, NULL,
                                 off, &L, block);
    if (nbp < 0) { rc = (int)nbp; goto done; }
  } else {
    /* Algorithm 2: mark_i per state; initial leaders by priority */
    for (int64_t i = 0; i < m; ++i) { ssrc[i] = src[i]; sdst[i] = dst[i]; ord[i] = 0; }
    for (int32_t s = 0; s < n; ++s) off[s] = s;
    L = n;
    for (int32_t v = 0; v < n; ++v) newl[v] = n;
    for (int32_t s = 0; s < n; ++s) {
      int32_t v = init ? init[s] : 0;
      if (s < newl[v]) newl[v] = s;
    }
    for (int32_t s = 0; s < n; ++s) block[s] = newl[init ? init[s] : 0];
  }
  mark = calloc((size_t)(L ? L : 1), 1);
  if (!mark) { rc = ORC_E_NOMEM; goto done; }
  /* initialisation: unstable_i := false; unstable_{block_i} := true */
  for (int32_t s = 0; s < n; ++s) unstable[s] = 0;
  for (int32_t s = 0; s < n; ++s) unstable[block[s]] = 1;
  if (out_pre_blocks) {
    int64_t c = 0;
    for (int32_t s = 0; s < n; ++s) c += (block[s] == s);
    *out_pre_blocks = c;
  }

  for (;;) {
    ++iters;
    if (max_iters > 0 && iters > max_iters) { rc = -4; goto done; }
    /* C := bot; C := i for an unstable i (priority: the smallest) */
    int32_t C = -1;
    for (int32_t s = 0; s < n; ++s)
      if (unstable[s]) { C = s; break; }
    if (iters == 1 && force_first_C >= 0) {
      if (force_first_C >= n || !unstable[force_first_C]) { rc = ORC_E_INVALID; goto done; }
      C = force_first_C;
    }
    int64_t it_idx = iters - 1;
    if (C < 0) {
      if (trace_C && it_idx < trace_cap) trace_C[it_idx] = -1;
      if (trace_nsplit && it_idx < trace_cap) trace_nsplit[it_idx] = 0;
      if (trace_blocks && it_idx < trace_cap)
        memcpy(trace_blocks + it_idx * (int64_t)n, block, sizeof(int32_t) * (size_t)n);
      break;
    }
    /* reset marks and split flags */
    memset(mark, 0, (size_t)L);
    memset(split, 0, (size_t)n);
    /* mark: transitions whose target is in block C */
    for (int64_t i = 0; i < m; ++i)
      if (block[sdst[i]] == C) mark[off[ssrc[i]] + ord[i]] = 1;
    if (variant == 3) {
      /* tag states whose mark for some action differs from their leader's */
      for (int64_t i = 0; i < m; ++i)
        if (mark[off[ssrc[i]] + ord[i]] != mark[off[block[ssrc[i]]] + ord[i]]) split[ssrc[i]] = 1;
    } else {
      for (int32_t s = 0; s < n; ++s) split[s] = mark[s] != mark[block[s]];
    }
    /* unstable_C := false precedes every := true of this step */
    unstable[C] = 0;
    /* leader election: the smallest split state of each block wins */
    int64_t nsplit = 0;
    for (int32_t s = 0; s < n; ++s) newl[s] = n;
    for (int32_t s = 0; s < n; ++s)
      if (split[s] && s < newl[block[s]]) newl[block[s]] = s;
    for (int32_t s = 0; s < n; ++s) {
      if (!split[s]) continue;
      ++nsplit;
      int32_t old = block[s];
      unstable[old] = 1;
      block[s] = newl[old];
      unstable[block[s]] = 1;
      if (variant == 3) unstable[C] = 1;
    }
    if (trace_C && it_idx < trace_cap) trace_C[it_idx] = C;
    if (trace_nsplit && it_idx < trace_cap) trace_nsplit[it_idx] = nsplit;
    if (trace_blocks && it_idx < trace_cap)
      memcpy(trace_blocks + it_idx * (int64_t)n, block, sizeof(int32_t) * (size_t)n);
  }
  if (out_block) memcpy(out_block, block, sizeof(int32_t) * (size_t)n);
  rc = 0;
done:
  free(ssrc); free(sdst); free(ord); free(off); free(block); free(newl); free(unstable);
  free(split); free(mark);
  return rc ? rc : iters;
}

/* ======================================================================== */
/* Checkers                                                                   */
/* ======================================================================== */
typedef struct {
  int32_t s, a, b;
} sig_t;

static int cmp_sig(const void* x, const void* y) {
  const sig_t* p = x;
  const sig_t* q = y;
  if (p->s != q->s) return p->s < q->s ? -1 : 1;
  if (p->a != q->a) return p->a < q->a ? -1 : 1;
  if (p->b != q->b) return p->b < q->b ? -1 : 1;
  return 0;
}

/* 1 iff every block is stable under every block: all members of a block
   reach the same set of (action, block) pairs.  Block labels need not be
   canonical.  < 0 on error. */
int orc_check_stable(int32_t n, int64_t m, const int32_t* src, const int32_t* lab,
                     const int32_t* dst, const int32_t* block) {
  for (int32_t s = 0; s < n; ++s)
    if (block[s] < 0 || block[s] >= n) return ORC_E_RANGE;
  sig_t* sg = malloc(sizeof(sig_t) * (size_t)(m ? m : 1));
  int64_t* beg = calloc((size_t)n + 1, sizeof(int64_t));
  int32_t* rep = malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
  int ok = 1;
  if (!sg || !beg || !rep) { ok = ORC_E_NOMEM; goto done; }
  for (int64_t i = 0; i < m; ++i) {
    sg[i].s = src[i];
    sg[i].a = lab[i];
    sg[i].b = block[dst[i]];
  }
  qsort(sg, (size_t)m, sizeof(sig_t), cmp_sig);
  /* dedupe into per-state unique lists */
  int64_t u = 0;
  for (int64_t i = 0; i < m; ++i)
    if (u == 0 || cmp_sig(&sg[u - 1], &sg[i]) != 0) sg[u++] = sg[i];
  for (int64_t i = 0; i < u; ++i) beg[sg[i].s + 1]++;
  for (int32_t s = 0; s < n; ++s) beg[s + 1] += beg[s];
  for (int32_t s = 0; s < n; ++s) rep[s] = -1;
  for (int32_t s = 0; s < n && ok == 1; ++s) {
    int32_t b = block[s];
    if (rep[b] < 0) { rep[b] = s; continue; }
    int32_t r = rep[b];
    int64_t ls = beg[s + 1] - beg[s], lr = beg[r + 1] - beg[r];
    if (ls != lr) { ok = 0; break; }
    for (int64_t k = 0; k < ls; ++k)
      if (sg[beg[s] + k].a != sg[beg[r] + k].a || sg[beg[s] + k].b != sg[beg[r] + k].b) {
        ok = 0;
        break;
      }
  }
done:
  free(sg); free(beg); free(rep);
  return ok;
}

/* 1 iff the partition `block` refines the partition `init` (init NULL = {S}). */
int orc_check_refines(int32_t n, const int32_t* block, const int32_t* init) {
  if (!init) return 1;
  int32_t* val = malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
  if (!val) return ORC_E_NOMEM;
  for (int32_t s = 0; s < n; ++s) val[s] = -1;
  int ok = 1;
  for (int32_t s = 0; s < n && ok; ++s) {
    int32_t b = block[s];
    if (b < 0 || b >= n) { ok = ORC_E_RANGE; break; }
    if (val[b] < 0) val[b] = init[s];
    else if (val[b] != init[s]) ok = 0;
  }
  free(val);
  return ok;
}

/* 1 iff every block id is the smallest member of its block. */
int orc_check_canonical(int32_t n, const int32_t* block) {
  for (int32_t s = 0; s < n; ++s) {
    int32_t b = block[s];
    if (b < 0 || b > s) return 0;
    if (block[b] != b) return 0;
  }
  return 1;
}
