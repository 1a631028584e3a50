#!/usr/bin/env python3
"""Benchmark: strong-bisimulation refinement on one MI355X.

A step is one full fixpoint of the plain refinement loop (coarsest_partition:
every iteration of select -> mark -> compare/elect -> relabel until no block
is unstable) on an LTS already loaded in HBM.  The metric is
transitions x iterations per second, m * #It / (seconds per step).

Default workload: a planted-quotient LTS with ~1.03M states and ~8.2M
transitions (50,000 quotient nodes, Poisson(8) out-degree, Zipf(1.1) labels
over 16 actions, U{1..40} copies per node, seed 1).

Prints one JSON line.  Extra fields: `roofline` for the persistent
refinement kernel (algorithmic bytes per launch from the per-iteration work
counters / its HIP-event-timed duration, against 8 TB/s), and `cpu_baseline`
(the CPU oracle's lock-step simulation timed on a bounded prefix of the same
workload, single-threaded).
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
    "planted-quotient-10M": dict(
        desc="planted quotient: 487,805 quotient nodes, Poisson(10), Zipf(1.1) over 64 actions, "
             "U{1..40} copies, pi_0={S}, seed 1",
        make=lambda g: g.planted_quotient(q=487_805, deg_mean=10.0, K=64, seed=1)),
}


def algorithmic_bytes(n: int, work: np.ndarray, nsplit: np.ndarray) -> float:
    """Bytes one fixpoint must move with this layout (int32 ids, 64-bit mark
    words, 1-bit unstable/touched/leader-touched flags), summed over
    iterations.  Per iteration:
      select   n/8 (unstable bitmap)
      mark     4n (block[] scan) + 8 per member of C (in_ptr pair)
               + 24 per in-transition (source, rank, mark-word RMW)
               + 8 per touched state (list append, leader test)
      compare  24 per touched state (list, block, own + leader mark words)
               + [a leader was touched] (4n block scan + n/4 touched/leader bits)
               + 12 per split state (bid, list append)
      relabel  20 per split state (list, block r/w, new-leader word)
               + 28 per touched state (list, mark word, touched/leader words)
    The final pass reads the candidate only."""
    members, edges, touched, ltany = (work[:, i].astype(np.float64) for i in range(4))
    s = nsplit.astype(np.float64)
    per = (n / 8 + 4 * n + 8 * members + 24 * edges + 8 * touched + 24 * touched
           + ltany * (4 * n + n / 4) + 12 * s + 20 * s + 28 * touched)
    per[-1] = 0.0  # final pass: no splitter
    return float(per.sum())


def cpu_baseline(L, target_s: float = 12.0):
    """The lock-step oracle (Algorithm 3 simulation) on a bounded prefix of
    the same workload: time(1 + X iterations) - time(1 iteration)."""
    import oracle
    oracle.lib()

    def timed(k):
        t = time.perf_counter()
        r = oracle.alg3_trace(L.n, L.K, L.src, L.lab, L.dst, L.init, max_iters=k)
        return time.perf_counter() - t, r

    t1, _ = timed(1)
    t5, r5 = timed(6)
    per_it = max((t5 - t1) / 5, 1e-6)
    X = int(max(5, min(100000, target_s / per_it)))
    tX, rX = timed(1 + X)
    X_done = rX["iters"] - 1 if not rX["truncated"] else X
    el = max(tX - t1, 1e-9)
    return {
        "value": L.m * X_done / el,
        "unit": "transition*iterations/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"lock-step simulation of the labelled algorithm (CPU oracle), iterations "
                  f"2..{1 + X_done} of the same workload, {el:.1f} s after subtracting the "
                  f"preprocessing + first iteration ({t1:.2f} s); single thread",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="planted-quotient-1M", choices=sorted(WORKLOADS))
    ap.add_argument("--engine", type=int, default=1, help="1 persistent, 2 per-phase kernels")
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the refinement of one "
                                   "LTS is a single-device fixpoint; run with --gpus 1"}))
        sys.exit(2)

    from paper_2105_11788_amd import bisim, gen

    wl = WORKLOADS[args.workload]
    t = time.perf_counter()
    L = wl["make"](gen)
    t_gen = time.perf_counter() - t
    print(f"[bench] workload {args.workload}: n={L.n} m={L.m} K={L.K} (generated in {t_gen:.1f}s)",
          file=sys.stderr, flush=True)

    bisim.load_library()
    if bisim.device_count() < 1:
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(3)
    to = lambda a: bisim.DeviceArray.from_numpy(a, np.int32)
    src, lab, dst = to(L.src), to(L.lab), to(L.dst)
    init = None if L.init is None else to(L.init)
    h = bisim.LTS(src, lab, dst, L.n, L.K, init)
    h.set_option(bisim.OPT_ENGINE, args.engine)
    if args.grid:
        h.set_option(bisim.OPT_GRID, args.grid)
    out = bisim.DeviceArray(L.n, np.int32)

    for w in range(args.warmup):
        _, st = h.run(out)
        print(f"[bench] warmup {w}: #It={st.iterations} blocks={st.blocks} "
              f"t_alg={st.t_alg_ms:.1f} ms", file=sys.stderr, flush=True)

    bisim.synchronize()
    t0 = time.perf_counter()
    alg_ms = []
    for k in range(args.steps):
        _, st = h.run(out)
        alg_ms.append(st.t_alg_ms)
    bisim.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    iters = st.iterations
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.2f} ms/step, #It={iters}",
          file=sys.stderr, flush=True)

    # one traced run outside the timed region for the byte count
    tr = h.set_trace(iters + 1, work=True)
    _, st_tr = h.run(out)
    assert st_tr.iterations == iters
    h.set_trace(0)
    work = tr[2].numpy().reshape(-1, 4)[:iters]
    nsplit = tr[1].numpy()[:iters]
    bytes_launch = algorithmic_bytes(L.n, work, nsplit)
    kern_ms = float(np.mean(alg_ms))
    achieved = bytes_launch / (kern_ms * 1e-3) / 1e9
    h.close()

    value = L.m * iters / (ms_per_step * 1e-3)
    res = {
        "metric": "transitions*iterations/sec (plain refinement to fixpoint)",
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
        "config": {
            "workload": args.workload,
            "description": wl["desc"],
            "n": L.n, "m": L.m, "K": L.K,
            "iterations": iters,
            "blocks": st.blocks,
            "pre_blocks": st.pre_blocks,
            "mark_length": st.mark_length,
            "form": "plain",
            "engine": {1: "persistent", 2: "per-phase"}.get(args.engine, str(args.engine)),
        },
        "seconds_to_fixpoint": ms_per_step / 1000.0,
        "t_pre_ms": st.t_pre_ms,
        "us_per_iteration": kern_ms * 1000.0 / iters,
        "roofline": {
            "bound": "hbm",
            "kernel": "k_persistent" if args.engine == 1 else "k_phase_*",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "bytes_per_launch": bytes_launch,
            "kernel_ms": kern_ms,
        },
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline ...", file=sys.stderr, flush=True)
        res["cpu_baseline"] = cpu_baseline(L, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
