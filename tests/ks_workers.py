"""Process-pool helpers for checking large batches against the oracle.

Workers start as fresh interpreters (spawn), regenerate the instances they
are given from the batch's seed, and run the Kanellakis-Smolka oracle on
them, so that neither the instances nor a GPU context cross a process
boundary; only the partitions come back.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np


def _ks_chunk(job):
    import oracle
    from paper_2105_11788_amd import gen
    ks_idx, count, n_lo, n_hi, seed = job
    out = []
    for k in ks_idx:
        L = gen.batch_instance(k, count=count, n_lo=n_lo, n_hi=n_hi, seed=seed)
        blk, nb = oracle.ks_coarsest(L.n, L.K, L.src, L.lab, L.dst, L.init)
        out.append((k, blk, nb))
    return out


def ks_batch(indices, count, n_lo, n_hi, seed, workers=None):
    """{k: (partition, block count)} for the given instances of
    gen.batch(count, n_lo, n_hi, seed=seed), over a pool of spawned workers
    (at most 16: the GPU host's share of cores)."""
    import oracle
    oracle.lib()  # build once before the workers load it
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    idx = list(indices)
    # interleave so that large and small instances mix across jobs
    jobs = [(idx[j::4 * workers], count, n_lo, n_hi, seed) for j in range(4 * workers)]
    jobs = [j for j in jobs if j[0]]
    res = {}
    with mp.get_context("spawn").Pool(workers) as pool:
        for part in pool.imap_unordered(_ks_chunk, jobs):
            for k, blk, nb in part:
                res[k] = (blk, nb)
    return res


def lifted_quotient(P, qblock):
    """Canonical partition of a planted-quotient expansion P induced by a
    partition qblock of its quotient: each state goes to the smallest state
    whose quotient node lies in the same quotient block."""
    lab = qblock[P.meta["state_to_q"]].astype(np.int64)
    first = np.full(int(lab.max()) + 1 if lab.size else 0, np.iinfo(np.int64).max, np.int64)
    np.minimum.at(first, lab, np.arange(P.n, dtype=np.int64))
    return first[lab].astype(np.int32)
