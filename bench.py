#!/usr/bin/env python3
"""Benchmark: strong-bisimulation refinement on one MI355X.

A step is one full fixpoint of the refinement loop (every iteration of
select -> mark -> compare/elect -> relabel until no block is unstable) on an
LTS already loaded in HBM.  The metric is transitions x iterations per
second, m * #It / (seconds per step); for a batch, sum_k m_k * #It_k over
the wall time of the batch.

Forms (--form):
  batched  (default) 4096 independent LTSs in one launch, sizes log-uniform
           in [100, n_hi] (n_hi = 200,000 by default: ~108M states and
           ~648M transitions in all), Poisson(6) out-degree, K ~ U{1..32},
           half with planted quotients; against running each instance alone
           with the plain engine (timed on a sample of instances and scaled);
  plain    the plain method, smallest-label splitter, on one LTS (default
           the planted quotient with ~1.03M states / ~8.2M transitions;
           --workload planted-quotient-10M is the ~10M-state one);
  learned  the learned splitter policy (network trained on the GPU first)
           against the plain policy on the same LTS;
  signature  the multi-way signature baseline (or --hybrid).

Prints one JSON line.  Extra fields: `roofline` for the dominant kernel
(bytes it moves per launch, from a byte model of its loads and stores and
per-iteration work counters, over its HIP-event-timed duration, against
8 TB/s, with the measured copy bandwidth beside it), and `cpu_baseline` (the
Kanellakis-Smolka CPU oracle built -O3 -march=native, timed to the fixpoint
on one thread, and for the batch also over the host's cores).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ENGINE_NAMES = {0: "automatic", 1: "persistent", 2: "per-phase kernels",
                3: "member-list kernels"}

WORKLOADS = {
    "planted-quotient-1M": dict(
        desc="planted quotient: 50k quotient nodes, Poisson(8) out-degree, Zipf(1.1) over 16 "
             "actions, U{1..40} copies, pi_0={S}, seed 1",
        make=lambda g: g.planted_quotient(q=50_000, deg_mean=8.0, K=16, seed=1)),
    "kripke-1k": dict(
        desc="Kripke structure n=1000 m=5000, uniform src/dst, |Act|=1, pi_0 by a Bernoulli(0.5) "
             "proposition, seed 1",
        make=lambda g: g.kripke_uniform(1000, 5000, seed=1)),
    "chain-100k": dict(
        desc="labelled chain of 100k states with a distinct tail label",
        make=lambda g: g.chain_tail(100_000)),
    "product-810k": dict(
        desc="synchronised product of 4 cyclic processes of 30 states over 8 actions, 2 shared",
        make=lambda g: g.sync_product(seed=1)),
    "distinct-actions-25k": dict(
        desc="chain of 25,217 states whose 25,216 transitions each have an action of their "
             "own (the shape of Table 1's row with as many actions as transitions)",
        make=lambda g: g.chain_distinct(25_217)),
    "planted-quotient-10M": dict(
        desc="planted quotient: 487,805 quotient nodes, Poisson(10), Zipf(1.1) over 64 actions, "
             "U{1..40} copies, pi_0={S}, seed 1",
        make=lambda g: g.planted_quotient(q=487_805, deg_mean=10.0, K=64, seed=1)),
}


def workload(name: str):
    """A named workload, or the family fan-out-<n> (Fan_out_n of section 5,
    Figure 3: #It = 2n - 4)."""
    if name.startswith("fan-out-"):
        n = int(name[len("fan-out-"):])
        return dict(desc=f"Fan_out_n with n={n} (section 5, Figure 3)",
                    make=lambda g: g.fan_out(n))
    return WORKLOADS[name]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def phase_bytes(n: int, work: np.ndarray, nsplit: np.ndarray):
    """Bytes each kernel of each iteration touches with this layout (int32
    ids, 64-bit mark words and bids, 1-bit flags):
      X (relabel + select + mark)
                     4n block[] scan + n/4 split-flag words (read k-1's,
                     clear k-2's) + 20 per split state of k-1 (bid read,
                     block write, new-leader list)
                     + 8 per member of C (in_ptr pair)
                     + 40 per in-transition of C (source, rank, block and
                       split flag of the source, mark-word and touched-word RMW)
      Y (compare + elect, clear k-1's marks)
                     4n block[] scan + n/4 touched words (this and the other
                     half) + n/8 leader-touched words
                     + 16 per touched state (own and leader mark words)
                     + 20 per split state (bid, split flag, unstable bit)
                     + 24 per touched state of k-1 (mark word, flag words)
    Returns an array [iterations, 2]; the final pass (no splitter) is zero."""
    members, edges, touched = (work[:, i].astype(np.float64) for i in range(3))
    s = nsplit.astype(np.float64)
    s_prev = np.concatenate([[0.0], s[:-1]])
    t_prev = np.concatenate([[0.0], touched[:-1]])
    out = np.stack([4 * n + n / 4 + 20 * s_prev + 8 * members + 40 * edges,
                    4 * n + n / 4 + n / 8 + 16 * touched + 20 * s + 24 * t_prev], axis=1)
    out[-1] = 0.0
    return out


LISTS_KERNELS = ["k_l_mark (select+mark)", "k_l_compare (compare+elect+rank, prefetch)",
                 "k_l_split (relabel+tail+swaps+ranges, clear marks)"]


def lists_bytes(n: int, iters: int, w: dict):
    """Bytes each kernel of the member-list engine moves per launch, averaged
    over the iterations: the byte model of its loads, stores and atomics
    (int32 ids, 64-bit mark words, bids and bitmap words; an atomic counts
    its read and its write) times the run's work totals:
      mark     8 (range of C) + 8 per member (its in-transition range)
               + 52 per in-transition (source, rank, the source's block and
                 range, mark-word and touched-word atomics) + 16 per touched
                 state (list entry, its block's touched-count atomic)
                 + 12 per listed segment (entry)
      compare  24 per touched state (list entry, own and leader mark
               words) + 56 per split state (bid, rank and split-flag
               atomics, list entry) + 24 per segment (entry, its block's
               touched count and range) + 12 per member visited (perm,
               touched word; only blocks with an untouched member)
               + the prefetch of the next splitter: 28 (candidate, range,
               slot header) + 16 per member prefetched (range loaded and
               stored; min(64, the mean splitter size) per iteration)
      split    32 per touched state (list entry and its block; mark word,
               touched word and touched count cleared) + 96 per split state
               (list entry, its block's bid, range and count, position, label
               store, front/tail counters, tail state and its flag, pair
               store, four list stores) + 8 per iteration that splits
               (the arrival counter; one relabelling workgroup per 256 split
               states, one in most such iterations) + 76 per split state
               (seven list loads, pair load, four perm/pos stores, two
               in-transition ranges loaded and stored, split flag; counted
               for every split state though only those in front of the tail
               swap) + 64 per split block (ranges, counters, unstable bits)
    Returns a list of three floats (bytes per launch)."""
    it = max(1, iters - 1)  # the final pass does no work
    mark = 8 * it + 8 * w["members"] + 52 * w["in_transitions"] + 16 * w["touched"] \
        + 12 * w["segments"]
    pref = it * (28 + 16 * min(64.0, w["members"] / it))
    comp = 24 * w["touched"] + 56 * w["split_states"] + 24 * w["segments"] \
        + 12 * w["member_visits"] + pref
    spl = 32 * w["touched"] + 96 * w["split_states"] + 8 * w["split_iterations"] \
        + 76 * w["split_states"] + 64 * w["split_blocks"]
    return [mark / it, comp / it, spl / it]


def batch_bytes(sizes, st, mask_bytes: int):
    """Bytes the batched kernel moves in one launch, from its work totals
    (st["work"], per tier) and a byte model of its global-memory loads,
    stores and atomics (an atomic counts its read and its write):
      both tiers   8 per state (preprocessed label in, result out)
      LDS tier     per iteration only the in-transitions of the splitter
                   leave LDS: 8 per splitter member (in_ptr pair) + 8 per
                   in-transition (source, action rank)
      member lists 72 + mask per state at set-up (labels, marks, bids,
                   counters, ranges, member list, positions, in-transition
                   ranges by position)
                   + per iteration 8 (splitter range) + 8 per member (its
                   in-transition range; those of the next splitter's first 64
                   members are prefetched and not loaded again unless the
                   iteration split something, which is not counted)
                   + (8 + 2 mask) per in-transition (source, rank, mark
                   atomic) + (12 + 3 mask) per touched state (block and the
                   range it would lead; own and leader marks; marks cleared)
                   + 4 per member visited (perm) + 132 per split state (bid
                   and rank atomics; bid, range end, count, position, tail
                   state, counters, pair, label; swap of the states and of
                   their two in-transition ranges, counted for every split
                   state though only those in front of the tail swap)
                   + 24 per split block (ranges and counters)
    Bitmaps and per-iteration lists live in LDS for the member-list tier too
    (when they fit) and count nothing.  sizes: instance sizes; the member-list
    tier holds the st["global_instances"] largest."""
    sz = np.sort(np.asarray(sizes, np.float64))[::-1]
    g = int(st["global_instances"])
    n_list = float(sz[:g].sum())
    n_all = float(sz.sum())
    w0, w1 = st["work"][0], st["work"][1]
    lds = 8.0 * w0[1] + 8.0 * w0[2]
    mk = float(mask_bytes)
    lists = (72 + mk) * n_list + 8.0 * w1[0] + 8.0 * w1[1] + (8 + 2 * mk) * w1[2] \
        + (12 + 3 * mk) * w1[3] + 4.0 * w1[5] + 132.0 * w1[6] + 24.0 * w1[7]
    return 8.0 * n_all + lds + lists


def method_bytes(n: int, m: int, mark_length: int, work: np.ndarray, nsplit: np.ndarray):
    """Bytes one iteration of the method as specified moves (Algorithm 3 with
    int32 ids and byte flags, each pass over all transitions or states),
    assigned to the kernel that does that pass's work here:
      X  select + reset: n/8 unstable bits + L mark zeroing + n split flags;
         mark: 4m targets + 4m block[target] gather + 5 per transition into C;
         the previous iteration's relabel: 2n split flags + 23 per split state
      Y  compare: 4n block + 8n slot offsets + 4n leader offsets + 2L marks
         + n split flags
    L is the mark length (section 4.1).  The kernels skip most of this work;
    the ratio of these bytes to kernel time is therefore the rate at which the
    method's passes are completed, and can exceed the memory bandwidth."""
    edges = work[:, 1].astype(np.float64)
    s = nsplit.astype(np.float64)
    s_prev = np.concatenate([[0.0], s[:-1]])
    n, m, L = float(n), float(m), float(mark_length)
    out = np.stack([np.full_like(s, n / 8 + L + n + 2 * n) + 8 * m + 5 * edges + 23 * s_prev,
                    np.full_like(s, 17 * n + 2 * L)], axis=1)
    out[-1] = 0.0
    return out


def stored_traffic(kernel: str, workload: str):
    """Memory traffic per launch measured with rocprofv3 counters (FETCH_SIZE
    + WRITE_SIZE, calibrated on a plain copy) and kept under profiles/; None
    when absent or when the kernel sources have changed since."""
    from paper_2105_11788_amd import profsum
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(("#", " ", "|")):
                key, val = line.split(":", 1)
                kv[key.strip()] = val.strip()
    src = os.path.join(ROOT, "paper_2105_11788_amd", "csrc")
    files = [f for f in kv.get("source_files", "").split(",") if f] or None
    if kv.get("source_sha1") != profsum.source_digest(src, files):
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(L, iterations: int, gpu_block=None, target_s: float = 12.0):
    """The Kanellakis-Smolka CPU oracle (compiled -O3 -march=native on this
    host, one thread) solving the same LTS to its fixpoint, repeated until
    about target_s seconds have passed (at least once).  Its time includes
    building the reverse transition index (its preprocessing).  The value is
    expressed in the benchmark's unit: m * #It (the GPU method's iteration
    count on this LTS) over the oracle's seconds per solve, so that the ratio
    of the two values is the ratio of the times to the fixpoint.  When the
    GPU's partition is given it is compared with the oracle's, element by
    element."""
    import oracle
    ks = oracle.native_ks()
    times, blk = [], None
    while not times or sum(times) < target_s:
        t = time.perf_counter()
        blk, nb = ks(L.n, L.K, L.src, L.lab, L.dst, L.init)
        times.append(time.perf_counter() - t)
    per = float(np.mean(times))
    res = {
        "value": L.m * iterations / per,
        "unit": "transition*iterations/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"Kanellakis-Smolka refinement (the CPU oracle, gcc -O3 -march=native) on the "
                  f"whole workload, {len(times)} solve(s) of {per:.2f} s each (reverse index "
                  f"included), single thread; value = m x the GPU method's #It / seconds per "
                  f"solve",
        "seconds_to_fixpoint": per,
        "seconds_sem": sem(times),
        "blocks": nb,
        "host": host_cpu(),
        "note": "a single LTS is one sequential fixpoint: no multi-core figure",
    }
    if gpu_block is not None:
        res["partition_equal_to_gpu"] = bool((np.asarray(gpu_block) == blk).all())
    return res


def _ks_job(job):
    """One batch instance through the native Kanellakis-Smolka oracle:
    (k, seconds)."""
    import oracle
    from paper_2105_11788_amd import gen
    k, count, n_lo, n_hi, seed = job
    L = gen.batch_instance(k, count=count, n_lo=n_lo, n_hi=n_hi, seed=seed)
    ks = oracle.native_ks()
    t = time.perf_counter()
    ks(L.n, L.K, L.src, L.lab, L.dst, L.init)
    return k, time.perf_counter() - t


def cpu_baseline_batch(insts, its, count, n_hi, target_s: float = 12.0, workers: int = 16,
                       gpu_blocks=None):
    """The Kanellakis-Smolka oracle (-O3 -march=native) on a seeded sample of
    the batch's instances: one instance after another on one thread until
    about target_s seconds, then the same sample over a pool of up to
    `workers` host processes (each regenerates its instances from the batch
    seed; the pool's wall time includes that and the process start).  Values
    are sum over the sample of m_k * #It_k (the GPU method's counts) per
    second, comparable with the GPU's whole-batch figure.  When the GPU's
    per-instance partitions are given, every sampled instance's is compared
    with the oracle's, element by element."""
    import multiprocessing as mp
    import oracle
    ks = oracle.native_ks()
    rng = np.random.default_rng(7)
    order = rng.permutation(len(insts))
    sample, done, el, equal = [], 0.0, 0.0, 0
    for k in order:
        L = insts[int(k)]
        t = time.perf_counter()
        blk, _ = ks(L.n, L.K, L.src, L.lab, L.dst, L.init)
        el += time.perf_counter() - t
        if gpu_blocks is not None:
            equal += int(bool((np.asarray(gpu_blocks[int(k)]) == blk).all()))
        done += L.m * float(its[int(k)])
        sample.append(int(k))
        if el >= target_s:
            break
    frac = sum(insts[k].m for k in sample) / max(1, sum(x.m for x in insts))
    cores = max(1, min(workers, os.cpu_count() or 1))
    t = time.perf_counter()
    # fresh interpreters: the workers import only numpy, the generator and
    # the oracle, and never touch the GPU this process has opened
    with mp.get_context("spawn").Pool(cores) as pool:
        list(pool.imap_unordered(_ks_job, [(k, count, 100, n_hi, 1) for k in sample]))
    el_all = time.perf_counter() - t
    desc = (f"Kanellakis-Smolka refinement (the CPU oracle, gcc -O3 -march=native) to the "
            f"fixpoint of {len(sample)} randomly chosen instances of the batch "
            f"({100 * frac:.1f} % of its transitions)")
    check = {}
    if gpu_blocks is not None:
        check = {"partition_equal_to_gpu": equal == len(sample),
                 "instances_equal_to_gpu": f"{equal} of {len(sample)}"}
    return {**check,
            "value": done / el, "unit": "transition*iterations/s", "cores": 1, "kind": "oracle",
            "sample": desc + f"; {el:.1f} s on one thread; value = sum m_k x #It_k (the GPU "
                             f"method's counts) / seconds",
            "seconds_whole_batch_estimate": el / frac if frac > 0 else None,
            "host": host_cpu(),
            "all_cores": {"value": done / el_all, "cores": cores,
                          "sample": f"the same instances over {cores} processes, "
                                    f"{el_all:.1f} s wall (process start and instance "
                                    f"generation included)",
                          "seconds_whole_batch_estimate": el_all / frac if frac > 0 else None}}


def host_cpu():
    """CPU model, clock (as /proc/cpuinfo reports it) and logical core count
    of the host that ran the baseline."""
    model, mhz = "unknown", None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name") and model == "unknown":
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("cpu MHz") and mhz is None:
                    mhz = float(line.split(":", 1)[1])
    except (OSError, ValueError):
        pass
    return {"model": model, "mhz": mhz, "logical_cpus": os.cpu_count()}


def sem(xs):
    """Standard error of the mean (None for fewer than two samples)."""
    if len(xs) < 2:
        return None
    return float(np.std(xs, ddof=1) / np.sqrt(len(xs)))


def upload(bisim, L):
    to = lambda a: bisim.DeviceArray.from_numpy(a, np.int32)
    return to(L.src), to(L.lab), to(L.dst), (None if L.init is None else to(L.init))


def base_record(args, metric, value, ms_per_step, config):
    return {
        "metric": metric,
        "value": value,
        "unit": "transition*iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": config,
    }


def run_single(bisim, L, args, engine, mlp=None, trace=True):
    """Time `steps` fixpoints of one LTS; returns a dict of measurements."""
    src, lab, dst, init = upload(bisim, L)
    h = bisim.LTS(src, lab, dst, L.n, L.K, init)
    h.set_option(bisim.OPT_ENGINE, engine)
    if args.grid:
        h.set_option(bisim.OPT_GRID, args.grid)
    if getattr(args, "algorithm", 3) != 3 and mlp is None:
        h.set_option(bisim.OPT_ALGORITHM, args.algorithm)
    if mlp is not None:
        bisim.set_splitter_policy(h, bisim.POLICY_LEARNED, mlp, args.rescore)
    out = bisim.DeviceArray(L.n, np.int32)
    st = None
    for w in range(max(1, args.warmup) if engine == 0 else args.warmup):
        _, st = h.run(out)
        log(f"warmup {w}: #It={st.iterations} blocks={st.blocks} t_alg={st.t_alg_ms:.1f} ms")
    if engine == 0:  # what the automatic choice (cached tuner) resolved to, kept fixed
        engine, grid = h.run_config()
        h.set_option(bisim.OPT_ENGINE, engine)
        h.set_option(bisim.OPT_GRID, grid)
        log(f"automatic engine choice: engine {engine}, {grid} workgroups")
    if engine == 2:  # sample ~200 iterations' phase kernels per step
        h.set_option(bisim.OPT_PROFILE_EVERY,
                     max(1, st.iterations // 200) if st is not None else 256)
    bisim.synchronize()
    t0 = time.perf_counter()
    alg_ms, step_ms = [], []
    for _ in range(args.steps):
        ts = time.perf_counter()
        _, st = h.run(out)  # returns after the fixpoint is on the host
        step_ms.append((time.perf_counter() - ts) * 1000.0)
        alg_ms.append(st.t_alg_ms)
    bisim.synchronize()
    t1 = time.perf_counter()
    res = {"ms_per_step": (t1 - t0) * 1000.0 / args.steps, "stats": st,
           "run_config": h.run_config(),
           "kern_ms": float(np.mean(alg_ms)), "block": out.numpy(),
           "ms_per_step_sem": sem(step_ms), "t_alg_ms_sem": sem(alg_ms)}
    if engine == 2:
        res["phase_ms"], res["phase_samples"] = h.phase_times()
        h.set_option(bisim.OPT_PROFILE_EVERY, 0)
    elif engine == 3:
        # the timed runs replay captured graphs; kernel durations come from one
        # more run launched kernel by kernel with end events (~200 sampled
        # iterations); that run's fixpoint time is reported beside them
        h.set_option(bisim.OPT_PROFILE_EVERY, max(1, st.iterations // 200))
        t1 = time.perf_counter()
        _, st_p = h.run(out)
        res["eager_ms_per_step"] = (time.perf_counter() - t1) * 1000.0
        res["phase_ms"], res["phase_samples"] = h.phase_times()
        h.set_option(bisim.OPT_PROFILE_EVERY, 0)
        assert st_p.iterations == st.iterations
    if trace and engine == 3:
        h.set_option(bisim.OPT_COUNT_WORK, 1)
        _, st_w = h.run(out)
        h.set_option(bisim.OPT_COUNT_WORK, 0)
        assert st_w.iterations == st.iterations
        res["work_totals"] = h.work()
        tr_ = h.set_trace(st.iterations + 1)
        h.run(out)
        res["nsplit"] = tr_[1].numpy()[:st.iterations]
        h.set_trace(0)
    elif trace:
        iters = st.iterations
        tr = h.set_trace(iters + 1, work=True)
        _, st_tr = h.run(out)
        assert st_tr.iterations == iters
        h.set_trace(0)
        res["work"] = tr[2].numpy().reshape(-1, 4)[:iters]
        res["nsplit"] = tr[1].numpy()[:iters]
    h.close()
    return res


def form_plain(bisim, gen, args):
    wl = workload(args.workload)
    t = time.perf_counter()
    L = wl["make"](gen)
    log(f"workload {args.workload}: n={L.n} m={L.m} K={L.K} ({time.perf_counter() - t:.1f}s)")
    r = run_single(bisim, L, args, args.engine)
    st = r["stats"]
    iters = st.iterations
    eng, grid = r["run_config"]
    copy_gbs = bisim.copy_bandwidth(1 << 30)
    names = ["k_fused_x (relabel+select+mark)", "k_fused_y (compare+elect)"]
    if eng == 3:
        lb = lists_bytes(L.n, iters, r["work_totals"])
        ms = r["phase_ms"][:3]
        q = int(np.argmax(ms))
        kernel = LISTS_KERNELS[q]
        touched_launch = float(lb[q])
        kern_ms = float(ms[q])
        # the method's bytes of a whole iteration (its passes over all
        # transitions and states), against the time of all four kernels
        edges = np.zeros((iters, 4))
        edges[:-1, 1] = r["work_totals"]["in_transitions"] / max(1, iters - 1)
        mb_it = method_bytes(L.n, L.m, st.mark_length, edges, r["nsplit"]).sum(axis=1)
        bytes_launch = float(mb_it[:-1].mean()) * kern_ms / max(float(ms.sum()), 1e-12)
        per_phase = {LISTS_KERNELS[i]: {"avg_us": float(ms[i] * 1e3),
                                        "bytes_per_launch": float(lb[i]),
                                        "GBs": float(lb[i] / (ms[i] * 1e-3) / 1e9)
                                        if ms[i] > 0 else None,
                                        "samples": int(r["phase_samples"][i])}
                     for i in range(3)}
        per_phase["work_totals"] = r["work_totals"]
        per_phase["timing"] = ("kernel durations from a run launched kernel by kernel "
                               f"({r['eager_ms_per_step']:.1f} ms to the fixpoint); the timed "
                               "runs replay captured graphs of 32 iterations")
    elif eng == 1:
        pb = phase_bytes(L.n, r["work"], r["nsplit"])
        mb = method_bytes(L.n, L.m, st.mark_length, r["work"], r["nsplit"])
        kernel, kern_ms = "k_persistent", r["kern_ms"]
        bytes_launch, touched_launch = float(mb.sum()), float(pb.sum())
        per_phase = None
    else:
        pb = phase_bytes(L.n, r["work"], r["nsplit"])
        mb = method_bytes(L.n, L.m, st.mark_length, r["work"], r["nsplit"])
        ms = r["phase_ms"][:2]
        q = int(np.argmax(ms))  # every phase runs once per iteration
        kernel = names[q]
        bytes_launch = float(mb[:-1, q].mean())
        touched_launch = float(pb[:-1, q].mean())
        kern_ms = float(ms[q])
        per_phase = {names[i]: {"avg_us": float(ms[i] * 1e3),
                                "method_bytes_per_launch": float(mb[:-1, i].mean()),
                                "method_GBs": float(mb[:-1, i].mean() / (ms[i] * 1e-3) / 1e9)
                                if ms[i] > 0 else None,
                                "touched_bytes_per_launch": float(pb[:-1, i].mean()),
                                "touched_GBs": float(pb[:-1, i].mean() / (ms[i] * 1e-3) / 1e9)
                                if ms[i] > 0 else None,
                                "samples": int(r["phase_samples"][i])} for i in range(2)}
    # (a run of a few iterations may sample none)
    achieved = touched_launch / (kern_ms * 1e-3) / 1e9 if kern_ms > 0 else None
    method_rate = bytes_launch / (kern_ms * 1e-3) / 1e9 if kern_ms > 0 else None
    fmt = lambda v: "n/a" if v is None else f"{v:.1f}"
    log(f"{r['ms_per_step']:.2f} ms/step, #It={iters}, {kernel}: {kern_ms * 1e3:.2f} us/launch, "
        f"bytes moved {fmt(achieved)} GB/s (method passes completed at {fmt(method_rate)} GB/s); "
        f"copy {copy_gbs:.0f} GB/s")
    cfg = {"workload": args.workload, "description": wl["desc"], "n": L.n, "m": L.m, "K": L.K,
           "iterations": iters, "blocks": st.blocks, "pre_blocks": st.pre_blocks,
           "mark_length": st.mark_length, "form": "plain", "algorithm": args.algorithm,
           "engine": ENGINE_NAMES.get(eng, str(eng)), "workgroups": grid,
           "engine_choice": "automatic (cached tuner)" if args.engine == 0 else "fixed"}
    res = base_record(args, "transitions*iterations/sec (plain refinement to fixpoint)",
                      L.m * iters / (r["ms_per_step"] * 1e-3), r["ms_per_step"], cfg)
    res.update({
        "seconds_to_fixpoint": r["ms_per_step"] / 1000.0,
        "ms_per_step_sem": r["ms_per_step_sem"],
        "t_alg_ms": r["kern_ms"],
        "t_alg_ms_sem": r["t_alg_ms_sem"],
        "t_pre_ms": st.t_pre_ms,
        "us_per_iteration": r["kern_ms"] * 1000.0 / iters,
        "roofline": {
            "bound": "hbm",
            "kernel": kernel,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS if achieved is not None else None,
            "traffic": stored_traffic(kernel.split(" ")[0], args.workload),
            "bytes_per_launch": touched_launch,
            "bytes_definition": "bytes the kernel moves per launch: the byte model of its "
                                "loads and stores (int32 ids, 64-bit mark words and bids, "
                                "1-bit flags) times the work counters of each iteration "
                                "(members and in-transitions of the splitter, touched, split "
                                "states), averaged over the iterations",
            "kernel_ms": kern_ms,
            "measured_copy_GBs": copy_gbs,
            "method_bytes_per_launch": bytes_launch,
            "method_pass_rate_GBs": method_rate,
            "method_pass_rate_definition": "bytes of Algorithm 3's passes over all transitions "
                                           "and states completed per second (these kernels "
                                           "skip most of them, so this rate can exceed the "
                                           "memory bandwidth; it is not a bandwidth)",
            "per_phase": per_phase,
        },
    })
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        res["cpu_baseline"] = cpu_baseline(L, iters, r["block"], args.cpu_seconds)
        if not res["cpu_baseline"].get("partition_equal_to_gpu", True):
            raise SystemExit("the GPU partition differs from the oracle's")
    return res


def form_signature(bisim, gen, args):
    """The multi-way signature refinement baseline on the same workload (the
    splitting style of the paper's section 5 comparison systems): time to the
    fixpoint and rounds, beside the labelled algorithm's figures."""
    wl = workload(args.workload)
    L = wl["make"](gen)
    log(f"workload {args.workload}: n={L.n} m={L.m} K={L.K}")
    src, lab, dst, init = upload(bisim, L)
    h = bisim.LTS(src, lab, dst, L.n, L.K, init)
    h.set_option(bisim.OPT_ALGORITHM,
                 bisim.ALGORITHM_HYBRID if args.hybrid else bisim.ALGORITHM_SIGNATURE)
    out = bisim.DeviceArray(L.n, np.int32)
    for w in range(args.warmup):
        _, st = h.run(out)
        log(f"warmup {w}: rounds={st.iterations} blocks={st.blocks} t_alg={st.t_alg_ms:.1f} ms")
    bisim.synchronize()
    t0 = time.perf_counter()
    alg_ms = []
    for _ in range(args.steps):
        _, st = h.run(out)
        alg_ms.append(st.t_alg_ms)
    bisim.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    h.close()
    log(f"{ms:.2f} ms/step, iterations={st.iterations}, blocks={st.blocks}")
    name = ("signature rounds, then Algorithm 3 (hybrid)" if args.hybrid
            else "multi-way signature refinement (baseline)")
    cfg = {"workload": args.workload, "description": wl["desc"], "n": L.n, "m": L.m, "K": L.K,
           "iterations": st.iterations, "blocks": st.blocks, "pre_blocks": st.pre_blocks,
           "form": "signature", "algorithm": name}
    res = base_record(args, "transitions*iterations/sec (rounds and iterations to fixpoint)",
                      L.m * st.iterations / (ms * 1e-3), ms, cfg)
    res.update({"seconds_to_fixpoint": ms / 1000.0, "t_pre_ms": st.t_pre_ms,
                "t_alg_ms": float(np.mean(alg_ms)), "roofline": None,
                "note": "a comparison baseline, not the paper's method"})
    return res


def form_batched(bisim, gen, args):
    t = time.perf_counter()
    insts = gen.batch(count=args.count, n_lo=100, n_hi=args.n_hi, seed=1)
    N = sum(x.n for x in insts)
    M = sum(x.m for x in insts)
    log(f"batch: {len(insts)} instances, sum n={N} sum m={M} ({time.perf_counter() - t:.1f}s)")
    t = time.perf_counter()
    b = bisim.Batch(insts)
    if args.batch_wg:  # fixed configuration instead of the autotuner
        b.set_option(bisim.BOPT_WG_SIZE, args.batch_wg)
    out = bisim.DeviceArray(b.N, np.int32)
    log(f"batch loaded and preprocessed ({time.perf_counter() - t:.1f}s)")
    st = None
    for w in range(args.warmup):
        _, its, st = b.run(out)
        log(f"warmup {w}: max #It={st['max_iterations']} t_alg={st['t_alg_ms']:.1f} ms "
            f"(wg {st['workgroup_size']}, grid {st['grid']}, lds/global {st['lds_instances']}/"
            f"{st['global_instances']})")
    bisim.synchronize()
    t0 = time.perf_counter()
    alg = []
    for _ in range(args.steps):
        _, its, st = b.run(out)
        alg.append(st["t_alg_ms"])
    bisim.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / args.steps
    work = float(sum(x.m * int(i) for x, i in zip(insts, its)))
    mask_bytes = 8 if max(x.K for x in insts) > 32 else 4
    moved = batch_bytes([x.n for x in insts], st, mask_bytes)
    kern_ms = float(np.mean(alg))
    achieved = moved / (kern_ms * 1e-3) / 1e9
    copy_gbs = bisim.copy_bandwidth(1 << 30)
    log(f"k_batch {kern_ms:.1f} ms per launch, {moved / 1e9:.2f} GB moved (byte model) -> "
        f"{achieved:.1f} GB/s; copy {copy_gbs:.0f} GB/s; work {st['work']}")
    gpu_blocks = b.split(out.numpy())  # the timed runs' partitions, checked with the oracle below
    b.close()
    # the same instances one at a time through the plain single-instance engine
    rng = np.random.default_rng(0)
    sample = rng.choice(len(insts), size=min(args.plain_sample, len(insts)), replace=False)
    t_s, it_s = 0.0, 0
    for k in sample:
        L = insts[int(k)]
        src, lab, dst, init = upload(bisim, L)
        with bisim.LTS(src, lab, dst, L.n, L.K, init) as h:
            h.set_option(bisim.OPT_ENGINE, args.engine)
            o = bisim.DeviceArray(max(L.n, 1), np.int32)
            h.run(o)
            bisim.synchronize()
            t1 = time.perf_counter()
            _, s1 = h.run(o)
            bisim.synchronize()
            t_s += time.perf_counter() - t1
            it_s += s1.iterations
            assert s1.iterations == its[int(k)]
        log(f"plain instance {int(k)}: n={L.n} #It={s1.iterations}")
    scale = float(its.sum()) / max(it_s, 1)
    plain_est_ms = t_s * 1000.0 * scale
    log(f"batched {ms:.1f} ms; plain one-by-one estimate {plain_est_ms:.0f} ms "
        f"({len(sample)} sampled instances, scaled by iterations)")
    cfg = {"workload": f"batch-{args.count}-up-to-{args.n_hi}",
           "description": f"{args.count} LTSs, log-uniform 100..{args.n_hi} states, Poisson(6), "
                          "K~U{1..32}, half planted quotients, seed 1",
           "instances": args.count, "sum_n": N, "sum_m": M,
           "max_iterations": int(its.max()), "sum_iterations": int(its.sum()),
           "form": "batched", "workgroup_size": st["workgroup_size"], "grid": st["grid"],
           "lds_instances": st["lds_instances"], "global_instances": st["global_instances"]}
    res = base_record(args, "transitions*iterations/sec (batched refinement to fixpoint)",
                      work / (ms * 1e-3), ms, cfg)
    res.update({"seconds_to_fixpoint": ms / 1000.0,
                "t_alg_ms": kern_ms,
                "roofline": {
                    "bound": "hbm",
                    "kernel": "k_batch",
                    "achieved": achieved,
                    "peak": HBM_PEAK_GBS,
                    "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS,
                    "traffic": stored_traffic("k_batch", cfg["workload"]),
                    "bytes_per_launch": moved,
                    "bytes_definition": "bytes the batched kernel moves per launch: the byte "
                                        "model of its global loads, stores and atomics "
                                        "(bench.py batch_bytes) times its work totals per "
                                        "tier; LDS-resident state counts nothing",
                    "kernel_ms": kern_ms,
                    "measured_copy_GBs": copy_gbs,
                    "work_totals": {"lds_tier": st["work"][0], "member_list_tier": st["work"][1]},
                    "note": "one launch refines every instance; its time is the critical path "
                            "of the slowest instance (one workgroup, one dependent chain of "
                            "global-memory round trips per phase), so the kernel is latency-"
                            "bound and moves little data per second",
                },
                "plain_one_by_one_estimate_s": plain_est_ms / 1000.0,
                "speedup_vs_plain": plain_est_ms / ms,
                "iteration_count": {"batched_critical_path": int(its.max()),
                                    "plain_sequential_total": int(its.sum())}})
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        res["cpu_baseline"] = cpu_baseline_batch(insts, its, args.count, args.n_hi,
                                                 args.cpu_seconds, gpu_blocks=gpu_blocks)
        log(f"cpu baseline: GPU partitions equal to the oracle's on "
            f"{res['cpu_baseline']['instances_equal_to_gpu']} sampled instances")
    return res


def form_learned(bisim, gen, args):
    from paper_2105_11788_amd import learn
    t = time.perf_counter()
    mlp, losses, rows = learn.train_policy(train_seeds=range(1001, 1001 + args.train_lts),
                                           steps=args.train_steps)
    t_train = time.perf_counter() - t
    log(f"trained on {rows} rows in {t_train:.1f}s, loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    wl = workload(args.workload)
    L = wl["make"](gen)
    log(f"workload {args.workload}: n={L.n} m={L.m} K={L.K}")
    rp = run_single(bisim, L, args, args.engine, trace=False)
    rl = run_single(bisim, L, args, args.engine, mlp=mlp, trace=False)
    assert (rp["block"] == rl["block"]).all(), "learned policy changed the partition"
    ip, il = rp["stats"].iterations, rl["stats"].iterations
    log(f"plain #It={ip} {rp['ms_per_step']:.1f} ms; learned #It={il} {rl['ms_per_step']:.1f} ms")
    # for context: the same policy machinery with an untrained network (random
    # weights), which orders splitters arbitrarily
    untrained = bisim.MLP(bisim.POLICY_FEATURES, seed=12345)
    ru = run_single(bisim, L, argparse.Namespace(**{**vars(args), "steps": 1, "warmup": 0}),
                    args.engine, mlp=untrained, trace=False)
    assert (ru["block"] == rp["block"]).all()
    iu = ru["stats"].iterations
    log(f"untrained network #It={iu}")
    # held-out LTSs of the training shape: plain (per-phase engine) against the
    # learned and the untrained network, iterations and time to the fixpoint
    held = []
    for regime in ("kripke", "zipf64"):
        for seed in range(2001, 2007):
            H = learn.training_lts(regime, seed)
            row = {"regime": regime, "seed": seed}
            for name, net in (("plain", None), ("learned", mlp), ("untrained", untrained)):
                learn.iterations(H, net, engine=2)  # first call: set-up
                it_, blk_, ms_ = learn.iterations(H, net, engine=2)
                row[name] = {"iterations": int(it_), "t_alg_ms": float(ms_)}
            held.append(row)
    ratio = lambda key, f: float(np.mean([r[f][key] / r["plain"][key] for r in held]))
    held_summary = {"lts": len(held),
                    "iteration_ratio_learned_over_plain": ratio("iterations", "learned"),
                    "wall_ratio_learned_over_plain": ratio("t_alg_ms", "learned"),
                    "iteration_ratio_untrained_over_plain": ratio("iterations", "untrained")}
    log(f"held-out LTSs: {held_summary}")
    cfg = {"workload": args.workload, "description": wl["desc"], "n": L.n, "m": L.m, "K": L.K,
           "form": "learned", "iterations": il, "plain_iterations": ip,
           "untrained_network_iterations": iu,
           "rescore_every": args.rescore, "train_rows": rows, "train_seconds": t_train}
    res = base_record(args, "transitions*iterations/sec (learned-splitter refinement)",
                      L.m * il / (rl["ms_per_step"] * 1e-3), rl["ms_per_step"], cfg)
    res.update({"seconds_to_fixpoint": rl["ms_per_step"] / 1000.0,
                "plain_seconds_to_fixpoint": rp["ms_per_step"] / 1000.0,
                "iteration_ratio_learned_over_plain": il / ip,
                "wall_ratio_learned_over_plain": rl["ms_per_step"] / rp["ms_per_step"],
                "partition_equal": True,
                "held_out": {"summary": held_summary, "runs": held}})
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form", default="batched",
                    choices=["plain", "batched", "learned", "signature"])
    ap.add_argument("--workload", default="planted-quotient-1M",
                    help="one of " + ", ".join(sorted(WORKLOADS)) + ", or fan-out-<n>")
    ap.add_argument("--engine", type=int, default=0,
                    help="0 automatic, 1 persistent, 2 per-phase kernels (all states), "
                         "3 per-phase kernels over member lists")
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--hybrid", action="store_true",
                    help="signature form: signature rounds, then Algorithm 3")
    ap.add_argument("--algorithm", type=int, default=3, choices=[2, 3],
                    help="plain form: 3 = labelled algorithm, 2 = one-action RCPP algorithm")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--count", type=int, default=4096)
    ap.add_argument("--n-hi", type=int, default=200_000,
                    help="batched form: largest instance size (log-uniform from 100)")
    ap.add_argument("--plain-sample", type=int, default=64)
    ap.add_argument("--batch-wg", type=int, default=0,
                    help="batched form: fixed workgroup size instead of the autotuner")
    ap.add_argument("--rescore", type=int, default=4096,
                    help="learned form: full re-scoring period R")
    ap.add_argument("--train-lts", type=int, default=12)
    ap.add_argument("--train-steps", type=int, default=300)
    args = ap.parse_args()
    try:
        workload(args.workload)
    except (KeyError, ValueError):
        ap.error(f"unknown workload {args.workload}")

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the refinement of one "
                                   "LTS is a single-device fixpoint; run with --gpus 1"}))
        sys.exit(2)

    from paper_2105_11788_amd import bisim, gen
    bisim.load_library()
    if bisim.device_count() < 1:
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(3)
    res = {"plain": form_plain, "batched": form_batched, "learned": form_learned,
           "signature": form_signature}[args.form](
        bisim, gen, args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
