"""Pins of the oracle's multi-way signature refinement (`signature_rounds`):
its fixpoint against the Kanellakis-Smolka oracle, each round's partition
against k-step bisimilarity computed over state pairs (the transfer
condition of Definition 2 iterated k times from pi_pre), and hand-derived
round counts on Fan_out_n and the chain."""
import numpy as np
import pytest

import oracle
from paper_2105_11788_amd import gen


def k_step_partitions(L, pre, kmax):
    """R_0 = same block of pi_pre; R_{j+1}(s,t) iff R_j(s,t) and every
    s -a-> s' is matched by some t -a-> t' with R_j(s',t'), and vice versa.
    Returns the canonical partitions of R_1 .. R_kmax."""
    n = L.n
    succ = [dict() for _ in range(n)]
    for s, a, t in zip(L.src.tolist(), L.lab.tolist(), L.dst.tolist()):
        succ[s].setdefault(a, set()).add(t)
    R = [[pre[s] == pre[t] for t in range(n)] for s in range(n)]

    def matched(s, t):
        for a, ss in succ[s].items():
            ts = succ[t].get(a)
            if not ts or not all(any(R[s2][t2] for t2 in ts) for s2 in ss):
                return False
        return True

    out = []
    for _ in range(kmax):
        R = [[R[s][t] and matched(s, t) and matched(t, s) for t in range(n)] for s in range(n)]
        out.append(np.array([min(t for t in range(n) if R[s][t]) for s in range(n)], np.int32))
    return out


@pytest.mark.parametrize("seed", range(40))
def test_rounds_are_k_step_bisimilarity(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 13))
    L = gen.random_lts(n, int(rng.integers(0, 3 * n)), int(rng.integers(1, 4)), seed,
                       init_blocks=int(rng.integers(0, 3)))
    r = oracle.signature_rounds(L.n, L.K, L.src, L.lab, L.dst, L.init, keep_blocks=True)
    pre = oracle.preprocess(L.n, L.K, L.src, L.lab, L.dst, L.init)["pre_block"]
    ks = k_step_partitions(L, pre.tolist(), r["rounds"])
    for j in range(r["rounds"]):
        assert (r["blocks"][j] == ks[j]).all(), (seed, j)
    # the last round changed nothing, every earlier one split something
    if r["rounds"] > 1:
        assert (r["blocks"][-1] == r["blocks"][-2]).all()
    for j in range(1, r["rounds"] - 1):
        assert len(set(r["blocks"][j].tolist())) > len(set(r["blocks"][j - 1].tolist()))
    assert (r["block"] == oracle.bruteforce_gfp(L.n, L.src, L.lab, L.dst, L.init)).all()


@pytest.mark.parametrize("seed", range(6))
def test_fixpoint_equals_kanellakis_smolka(seed):
    L = gen.random_lts(400, 1500, 3, seed, init_blocks=seed % 3)
    r = oracle.signature_rounds(L.n, L.K, L.src, L.lab, L.dst, L.init)
    ks, nb = oracle.ks_coarsest(L.n, L.K, L.src, L.lab, L.dst, L.init)
    assert (r["block"] == ks).all()
    pre_blocks = oracle.preprocess(L.n, L.K, L.src, L.lab, L.dst, L.init)["pre_blocks"]
    assert r["rounds"] <= nb - pre_blocks + 1


@pytest.mark.parametrize("n", [4, 5, 9, 64, 300])
def test_fan_out_rounds(n):
    # pi_pre = {0,1}, {2..n-2}, {n-1}; each round peels the top chain state
    # (one whose a-successor left the chain block), and one more round finds
    # nothing: n - 3 rounds
    L = gen.fan_out(n)
    r = oracle.signature_rounds(L.n, L.K, L.src, L.lab, L.dst)
    assert r["rounds"] == n - 3
    exp = np.arange(n)
    exp[1] = 0
    assert (r["block"] == exp).all()


@pytest.mark.parametrize("n", [3, 4, 10, 200])
def test_chain_rounds(n):
    # pi_pre = {s_0..s_{n-3}}, {s_{n-2}}, {s_{n-1}}: n - 3 peeling rounds, one final
    L = gen.chain_tail(n)
    r = oracle.signature_rounds(L.n, L.K, L.src, L.lab, L.dst)
    assert r["rounds"] == max(n - 2, 1)
    assert (r["block"] == np.arange(n)).all()


@pytest.mark.parametrize("seed", range(30))
def test_hybrid_equals_kanellakis_smolka(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 400))
    L = gen.random_lts(n, int(rng.integers(0, 4 * n)), int(rng.integers(1, 4)), seed,
                       init_blocks=seed % 3)
    for stall in (1, 2, 64):
        h = oracle.hybrid_trace(L.n, L.K, L.src, L.lab, L.dst, L.init, stall=stall)
        ks, _ = oracle.ks_coarsest(L.n, L.K, L.src, L.lab, L.dst, L.init)
        assert (h["block"] == ks).all(), (seed, stall)
        assert h["iters"] == h["rounds"] + h["alg3_iters"]


@pytest.mark.parametrize("n", [7, 8, 20, 300])
def test_hybrid_fan_out(n):
    # rounds 1 and 2 each peel one chain state (one new block each), so the
    # switch comes after round 2, from {0,1}, {2..n-4}, {n-3}, {n-2}, {n-1}.
    # Algorithm 3 from there: C = 0 (no split), n - 6 peels of the chain block,
    # the chain block {2} once more, the n - 3 singletons 3..n-1 once each, and
    # the final pass: 2n - 6 iterations; 2n - 4 in all, as for Algorithm 3 alone.
    L = gen.fan_out(n)
    h = oracle.hybrid_trace(L.n, L.K, L.src, L.lab, L.dst)
    assert h["rounds"] == 2 and h["alg3_iters"] == 2 * n - 6 and h["iters"] == 2 * n - 4
    exp = np.arange(n)
    exp[1] = 0
    assert (h["block"] == exp).all()


def test_hybrid_stops_at_a_signature_fixpoint():
    # a planted quotient refines in a few large multi-way rounds: no switch
    L = gen.planted_quotient(q=2000, deg_mean=6.0, K=8, seed=7)
    s = oracle.signature_rounds(L.n, L.K, L.src, L.lab, L.dst)
    h = oracle.hybrid_trace(L.n, L.K, L.src, L.lab, L.dst)
    assert s["fixpoint"] and h["alg3_iters"] == 0 and h["iters"] == s["rounds"]
