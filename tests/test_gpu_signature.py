"""GPU parity of the multi-way signature refinement baseline
(BISIM_ALGORITHM_SIGNATURE) and of the hybrid (BISIM_ALGORITHM_HYBRID:
signature rounds, then Algorithm 3) against the oracle: canonical block ids
equal to Kanellakis-Smolka's, round and iteration counts equal to the
oracle's signature_rounds and hybrid_trace."""
import os

import numpy as np
import pytest

import oracle
from paper_2105_11788_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2105_11788_amd import bisim
    bisim.load_library()
    assert bisim.device_count() > 0, "GPU tests need a GPU"
    return bisim


def run_sig(B, L, trace=0, hybrid=False, engine=0):
    from paper_2105_11788_amd.bisim import DeviceArray
    t = lambda a: DeviceArray.from_numpy(a, np.int32)
    init = None if L.init is None else t(L.init)
    with B.LTS(t(L.src), t(L.lab), t(L.dst), L.n, L.K, init) as h:
        h.set_option(B.OPT_ALGORITHM, B.ALGORITHM_HYBRID if hybrid else B.ALGORITHM_SIGNATURE)
        if engine:
            h.set_option(B.OPT_ENGINE, engine)
        if trace:
            h.set_trace(trace)
        blk, st = h.run()
        return blk.numpy(), st


def assert_parity(B, L, rounds=True):
    ks, nb = oracle.ks_coarsest(L.n, L.K, L.src, L.lab, L.dst, L.init)
    blk, st = run_sig(B, L)
    assert (blk == ks).all(), L.name
    assert st.blocks == nb
    if rounds:
        r = oracle.signature_rounds(L.n, L.K, L.src, L.lab, L.dst, L.init)
        assert st.iterations == r["rounds"], (L.name, st.iterations, r["rounds"])


@pytest.mark.parametrize("n", [4, 5, 64, 300, 2000])
def test_fan_out(B, n):
    assert_parity(B, gen.fan_out(n))


@pytest.mark.parametrize("n", [2, 3, 1000])
def test_chain(B, n):
    assert_parity(B, gen.chain_tail(n))


def test_figures(B):
    assert_parity(B, gen.figure1())
    assert_parity(B, gen.figure2())


@pytest.mark.parametrize("seed", range(8))
def test_random(B, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(50, 3000))
    L = gen.random_lts(n, int(rng.integers(0, 4 * n)), int(rng.integers(1, 6)), seed,
                       init_blocks=seed % 4)
    assert_parity(B, L)


def test_kripke_and_many_actions(B):
    assert_parity(B, gen.kripke_uniform(2000, 9000, seed=3))
    assert_parity(B, gen.uniform_zipf(1500, 8000, K=64, seed=2))


def test_planted_quotient_medium(B):
    assert_parity(B, gen.planted_quotient(q=3000, deg_mean=6.0, K=8, seed=4))


def test_planted_quotient_1m_full(B):
    # round count checked against the C-side oracles only through the result
    L = gen.planted_quotient()
    assert_parity(B, L, rounds=False)


def test_empty_and_errors(B):
    from paper_2105_11788_amd.bisim import BisimError
    e = gen.LTS(0, 1, np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.int64),
                None, name="empty")
    blk, st = run_sig(B, e)
    assert blk.size == 0 and st.iterations == 0
    no_tr = gen.LTS(5, 1, np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.int64),
                    None, name="no transitions")
    assert_parity(B, no_tr)
    with pytest.raises(BisimError):
        run_sig(B, gen.fan_out(10), trace=8)
    # (distinct actions of a state) * n >= 2^32: refused before any kernel
    n = 70_000
    big = gen.LTS(n, n, np.zeros(n, np.int64), np.arange(n, dtype=np.int64),
                  np.arange(n, dtype=np.int64), None, name="one state, 70000 actions")
    with pytest.raises(BisimError):
        run_sig(B, big)


def assert_hybrid(B, L, engines=(1, 2)):
    ks, nb = oracle.ks_coarsest(L.n, L.K, L.src, L.lab, L.dst, L.init)
    ref = oracle.hybrid_trace(L.n, L.K, L.src, L.lab, L.dst, L.init)
    for e in engines:
        blk, st = run_sig(B, L, hybrid=True, engine=e)
        assert (blk == ks).all(), (L.name, e)
        assert st.blocks == nb
        assert st.iterations == ref["iters"], (L.name, e, st.iterations, ref)
    return ref


@pytest.mark.parametrize("n", [7, 64, 300, 3000])
def test_hybrid_fan_out(B, n):
    ref = assert_hybrid(B, gen.fan_out(n))
    assert ref["alg3_iters"] > 0  # switched to Algorithm 3


def test_hybrid_chain_and_figures(B):
    assert_hybrid(B, gen.chain_tail(1000))
    assert_hybrid(B, gen.figure1())
    assert_hybrid(B, gen.figure2())


@pytest.mark.parametrize("seed", range(6))
def test_hybrid_random(B, seed):
    rng = np.random.default_rng(50 + seed)
    n = int(rng.integers(50, 3000))
    assert_hybrid(B, gen.random_lts(n, int(rng.integers(0, 4 * n)), int(rng.integers(1, 6)),
                                    seed, init_blocks=seed % 4))


def test_hybrid_no_switch_and_large(B):
    ref = assert_hybrid(B, gen.planted_quotient(q=3000, deg_mean=6.0, K=8, seed=4))
    assert ref["alg3_iters"] == 0
    L = gen.planted_quotient()
    ks, nb = oracle.ks_coarsest(L.n, L.K, L.src, L.lab, L.dst, L.init)
    blk, st = run_sig(B, L, hybrid=True)
    assert (blk == ks).all() and st.blocks == nb


def test_hybrid_errors(B):
    from paper_2105_11788_amd.bisim import BisimError
    with pytest.raises(BisimError):
        run_sig(B, gen.fan_out(10), trace=8, hybrid=True)


def test_many_actions_per_state(B):
    # states with more than 64 distinct actions (multi-word mark slots for
    # Algorithm 3; ranks up to 90 in the signature keys) and every state of
    # out-degree 90, so the hybrid's Algorithm 3 part marks with combining
    rng = np.random.default_rng(3)
    n, K = 300, 200
    src = np.repeat(np.arange(n), 90)
    L = gen.LTS(n, K, src, rng.integers(0, K, size=src.size), rng.integers(0, n, size=src.size),
                None, name="300 states, 90 transitions each, 200 actions")
    assert oracle.preprocess(L.n, L.K, L.src, L.lab, L.dst)["nr_marks"].max() > 64
    assert_parity(B, L)
    assert_hybrid(B, L)
    Q = gen.LTS(20, 150, np.repeat(np.arange(20), 100), rng.integers(0, 150, 2000),
                rng.integers(0, 20, 2000), None, name="quotient with >64-action sets")
    P, _ = gen.expand_quotient(Q, np.random.default_rng(1), 1, 6)
    assert_parity(B, P)
    assert_hybrid(B, P)
    # a chain whose states also loop on 70 actions of their own: the signature
    # rounds stall, and Algorithm 3 continues on multi-word mark slots
    C = gen.chain_tail(400)
    loops = np.repeat(np.arange(400), 70)
    W = gen.LTS(400, 72, np.concatenate([C.src, loops]),
                np.concatenate([C.lab, np.tile(np.arange(2, 72), 400)]),
                np.concatenate([C.dst, loops]), None, name="chain with 70 self-loop actions")
    ref = assert_hybrid(B, W)
    assert ref["alg3_iters"] > 0
    assert_parity(B, W)


def test_kripke_with_propositions_hybrid(B):
    # one action and a proposition partition: pi_pre is the leader-normalised pi_0
    assert_hybrid(B, gen.kripke_uniform(2000, 9000, seed=5))
    assert_parity(B, gen.kripke_uniform(2000, 9000, seed=5))


@pytest.mark.parametrize("seed", [0, 1])
def test_sources_around_the_wave_size(B, seed):
    # out-degrees 1..70: up to 64 a source's transitions are compared lane
    # against lane (many sources straddle a 64-transition boundary of the
    # by-source layout), beyond that they go through the sort; two actions
    # and targets drawn from a planted quotient make most sources repeat
    # (action, block) pairs in every round
    rng = np.random.default_rng(seed)
    q = 40
    deg = rng.integers(1, 71, size=q)
    src = np.repeat(np.arange(q), deg)
    Q = gen.LTS(q, 2, src, rng.integers(0, 2, src.size), rng.integers(0, q, src.size), None,
                name=f"quotient with out-degrees 1..70, seed {seed}")
    P, _ = gen.expand_quotient(Q, np.random.default_rng(seed + 5), 1, 30)
    assert_parity(B, P)
    assert_hybrid(B, P)
    # beside a chain that takes ~100 rounds, so the later rounds run on the
    # by-source layout
    C = gen.chain_tail(100)
    U = gen.LTS(P.n + C.n, 2, np.concatenate([P.src, C.src + P.n]),
                np.concatenate([P.lab, C.lab]), np.concatenate([P.dst, C.dst + P.n]), None,
                name=P.name + " beside a 100-state chain")
    assert_parity(B, U)
    n = 1200
    deg = rng.integers(1, 71, size=n)
    src = np.repeat(np.arange(n), deg)
    R = gen.LTS(n, 2, src, rng.integers(0, 2, src.size), rng.integers(0, n, src.size),
                rng.integers(0, 3, n).astype(np.int64), name=f"random, out-degrees 1..70, seed {seed}")
    assert_parity(B, R)


def test_repeated_runs_on_one_handle(B):
    # the handle keeps the run's buffers: runs after the first reuse them,
    # also when a later run needs more of them (the by-source layout that a
    # hybrid run stopping after two rounds never reaches)
    from paper_2105_11788_amd.bisim import DeviceArray
    L = gen.fan_out(300)
    ks, nb = oracle.ks_coarsest(L.n, L.K, L.src, L.lab, L.dst, L.init)
    rounds = oracle.signature_rounds(L.n, L.K, L.src, L.lab, L.dst, L.init)["rounds"]
    hyb = oracle.hybrid_trace(L.n, L.K, L.src, L.lab, L.dst, L.init)["iters"]
    t = lambda a: DeviceArray.from_numpy(a, np.int32)
    with B.LTS(t(L.src), t(L.lab), t(L.dst), L.n, L.K, None) as h:
        for alg, its in [(B.ALGORITHM_HYBRID, hyb), (B.ALGORITHM_SIGNATURE, rounds),
                         (B.ALGORITHM_SIGNATURE, rounds), (B.ALGORITHM_HYBRID, hyb)]:
            h.set_option(B.OPT_ALGORITHM, alg)
            blk, st = h.run()
            assert (blk.numpy() == ks).all() and st.blocks == nb
            assert st.iterations == its, (alg, st.iterations, its)


def test_sorted_paths(B):
    # the radix-sort paths that large inputs take (states grouped by a stable
    # sort of their hashes, large sources' pairs sorted), forced on small LTSs
    os.environ["BISIM_SIGNATURE_SORT_ONLY"] = "1"
    try:
        for L in [gen.fan_out(300), gen.chain_tail(200), gen.figure2(),
                  gen.random_lts(2000, 9000, 4, 7, init_blocks=2)]:
            assert_parity(B, L)
            assert_hybrid(B, L)
    finally:
        os.environ.pop("BISIM_SIGNATURE_SORT_ONLY", None)
