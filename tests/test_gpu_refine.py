"""GPU parity: the HIP refinement (through the C ABI) against the CPU oracle.

Bar: bit-exact block ids (canonical, smallest member), identical iteration
counts, and identical splitter / split-count traces, on every engine (1: one
persistent launch, 2: a kernel per phase scanning all states, 3: a kernel per
phase over member lists)."""
import ctypes
import json
import os

import numpy as np
import pytest

import oracle
from ks_workers import lifted_quotient
from paper_2105_11788_amd import gen

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")
ENGINES = [1, 2, 3]
ALG2_ENGINES = [1, 2]  # the member-list engine runs Algorithm 3 only


@pytest.fixture(scope="module")
def B():
    from paper_2105_11788_amd import bisim
    bisim.load_library()
    assert bisim.device_count() > 0, "GPU tests need a GPU"
    return bisim


def dev(L):
    from paper_2105_11788_amd.bisim import DeviceArray
    t = lambda a: DeviceArray.from_numpy(a, np.int32)
    return t(L.src), t(L.lab), t(L.dst), (None if L.init is None else t(L.init))


def run_gpu(B, L, engine=1, trace=0, first=-1, grid=0, algorithm=3):
    src, lab, dst, init = dev(L)
    with B.LTS(src, lab, dst, L.n, L.K, init) as h:
        h.set_option(B.OPT_ENGINE, engine)
        if algorithm != 3:
            h.set_option(B.OPT_ALGORITHM, algorithm)
        if first >= 0:
            h.set_option(B.OPT_FIRST_SPLITTER, first)
        if grid:
            h.set_option(B.OPT_GRID, grid)
        tr = h.set_trace(trace) if trace else None
        blk, st = h.run()
        out = {"block": blk.numpy(), "stats": st}
        if tr is not None:
            k = min(st.iterations, trace)
            out["C"] = tr[0].numpy()[:k]
            out["nsplit"] = tr[1].numpy()[:k]
        return out


def assert_parity(B, L, engines=ENGINES, trace=True):
    cap = 3 * L.n + 2 if trace else 0
    ref = oracle.alg3_trace(L.n, L.K, L.src, L.lab, L.dst, L.init, trace_cap=cap)
    ks, nb = oracle.ks_coarsest(L.n, L.K, L.src, L.lab, L.dst, L.init)
    assert (ref["block"] == ks).all()
    for e in engines:
        g = run_gpu(B, L, engine=e, trace=cap)
        assert (g["block"] == ks).all(), (L.name, e)
        st = g["stats"]
        assert st.iterations == ref["iters"], (L.name, e, st.iterations, ref["iters"])
        assert st.blocks == nb and st.pre_blocks == ref["pre_blocks"]
        if trace:
            assert (g["C"] == ref["C"]).all(), (L.name, e)
            assert (g["nsplit"] == ref["nsplit"]).all(), (L.name, e)


def test_library_loads(B):
    assert B.load_library() is not None


def test_figure2(B):
    g = json.load(open(os.path.join(GOLD, "figure2.json")))
    L = gen.figure2()
    src, lab, dst, _ = dev(L)
    with B.LTS(src, lab, dst, L.n, L.K) as h:
        pb, nm = h.preprocessed()
        assert pb.tolist() == g["final_partition"]
        assert nm.tolist() == g["nr_marks"]
        blk, st = h.run()
    assert blk.numpy().tolist() == g["final_partition"]
    assert st.iterations == g["iterations_alg3"] and st.mark_length == g["mark_length"]
    assert_parity(B, L)


@pytest.mark.parametrize("engine", ENGINES)
def test_figure1(B, engine):
    g = json.load(open(os.path.join(GOLD, "figure1.json")))
    L = gen.figure1()
    r = run_gpu(B, L, engine=engine, trace=16)
    assert r["block"].tolist() == g["final_partition"]
    assert r["stats"].iterations == g["alg3_iterations"]
    assert r["C"].tolist() == g["alg3_splitters"]
    # the iteration drawn in the figure: splitter B_s4 forced first
    ref = oracle.alg3_trace(L.n, 1, L.src, L.lab, L.dst, L.init, trace_cap=16, keep_blocks=True,
                            force_first_C=g["forced_first_splitter"])
    assert ref["blocks"][0].tolist() == g["after_one_iteration"]
    r2 = run_gpu(B, L, engine=engine, trace=16, first=g["forced_first_splitter"])
    assert r2["C"].tolist() == ref["C"].tolist()
    assert r2["stats"].iterations == ref["iters"]
    assert r2["block"].tolist() == g["final_partition"]


@pytest.mark.parametrize("n", [4, 5, 9, 64, 65, 700, 5000])
def test_fan_out(B, n):
    L = gen.fan_out(n)
    for e in ENGINES:
        r = run_gpu(B, L, engine=e)
        assert r["stats"].iterations == 2 * n - 4
        exp = np.arange(n)
        exp[1] = 0
        assert (r["block"] == exp).all()


def hubs_lts(n: int, m: int, K: int, hubs: int, seed: int):
    """A sparse random LTS plus `hubs` states with transitions into long runs
    of consecutive states: waves of the mark step then hold the same source
    many times, with more such sources than a workgroup combines."""
    rng = np.random.default_rng(seed)
    base = gen.random_lts(n, m, K, seed)
    src, lab, dst = [base.src], [base.lab], [base.dst]
    for h in range(hubs):
        w = int(rng.integers(600, 2000))
        lo = int(rng.integers(0, n - w))
        src.append(np.full(w, h, np.int64))
        dst.append(np.arange(lo, lo + w, dtype=np.int64))
        lab.append(rng.integers(0, 3, w))
    cat = lambda xs: np.concatenate(xs).astype(np.int64)
    return gen.LTS(n, K, cat(src), cat(lab), cat(dst), None,
                   name=f"hubs(n={n},m={m},K={K},hubs={hubs},seed={seed})")


@pytest.mark.parametrize("seed", [5, 6])
def test_high_out_degree_sources(B, seed):
    L = hubs_lts(6000, 24000, 4, 12, seed)
    assert np.bincount(L.src, minlength=L.n).max() >= 64  # takes the combining marking
    assert_parity(B, L)


@pytest.mark.parametrize("n", [3, 1000, 20000])
def test_chain(B, n):
    L = gen.chain_tail(n)
    for e in ENGINES:
        r = run_gpu(B, L, engine=e)
        assert r["stats"].iterations == 2 * n - 2
        assert (r["block"] == np.arange(n)).all()


def test_kripke_uniform_1000(B):
    """The n=1000, m=5000 Kripke structure: full trace parity."""
    assert_parity(B, gen.kripke_uniform(1000, 5000, seed=1))


@pytest.mark.parametrize("seed", range(6))
def test_random_medium_trace(B, seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(50, 3000))
    m = int(rng.integers(0, 6 * n))
    K = int(rng.integers(1, 20))
    L = gen.random_lts(n, m, K, seed=seed, init_blocks=int(rng.integers(0, 5)))
    assert_parity(B, L)


def test_many_tiny(B):
    rng = np.random.default_rng(7)
    for k in range(150):
        n = int(rng.integers(1, 9))
        L = gen.random_lts(n, int(rng.integers(0, 16)), int(rng.integers(1, 4)), seed=500 + k,
                           init_blocks=int(rng.integers(0, 3)))
        assert_parity(B, L, engines=[1 + (k % 3)])


def test_more_than_64_actions_per_state(B):
    """States with > 64 distinct outgoing actions use multi-word mark slots."""
    rng = np.random.default_rng(3)
    n, K = 300, 200
    src = np.repeat(np.arange(n), 90)
    lab = rng.integers(0, K, size=src.size)
    dst = rng.integers(0, n, size=src.size)
    L = gen.LTS(n, K, src, lab, dst)
    pp = oracle.preprocess(L.n, L.K, L.src, L.lab, L.dst)
    assert pp["nr_marks"].max() > 64
    assert_parity(B, L)
    # a planted quotient whose copies share >64-action sets
    Q = gen.LTS(20, 150, np.repeat(np.arange(20), 100), rng.integers(0, 150, 2000),
                rng.integers(0, 20, 2000))
    P, s2q = gen.expand_quotient(Q, np.random.default_rng(1), 1, 6)
    assert_parity(B, P)


def test_planted_quotient_medium(B):
    P = gen.planted_quotient(q=2000, deg_mean=8.0, K=16, seed=2)
    assert_parity(B, P, trace=False)
    r = run_gpu(B, P, engine=1, trace=200)
    ref = oracle.alg3_trace(P.n, P.K, P.src, P.lab, P.dst, trace_cap=200)
    assert (r["C"] == ref["C"]).all() and (r["nsplit"] == ref["nsplit"]).all()


def test_empty_and_degenerate(B):
    c = lambda v: B.DeviceArray.from_numpy(np.array(v, np.int32))
    z = c([])
    with B.LTS(z, z, z, 0, 1) as h:
        blk, st = h.run()
        assert blk.count == 0 and st.iterations == 1 and st.blocks == 0
    # no transitions, an initial partition: already stable
    with B.LTS(z, z, z, 5, 3, c([0, 0, 2, 2, 0])) as h:
        blk, st = h.run()
        assert blk.numpy().tolist() == [0, 0, 2, 2, 0] and st.iterations == 3
    # one state with a self-loop
    o = c([0])
    with B.LTS(o, o, o, 1, 1) as h:
        blk, st = h.run()
        assert blk.numpy().tolist() == [0] and st.iterations == 2


def test_errors(B):
    c = lambda v: B.DeviceArray.from_numpy(np.array(v, np.int32))
    with pytest.raises(B.BisimError) as e:
        B.LTS(c([0]), c([0]), c([3]), 3, 1)
    assert e.value.status == B.E_RANGE
    with pytest.raises(B.BisimError) as e:
        B.LTS(c([0]), c([1]), c([2]), 3, 1)
    assert e.value.status == B.E_RANGE
    with pytest.raises(B.BisimError) as e:
        B.LTS(c([0]), c([0]), c([1]), 3, 1, init=c([0, 0, 7]))
    assert e.value.status == B.E_RANGE
    with pytest.raises(B.BisimError) as e:
        B.LTS(c([0]), c([0]), c([1]), 3, 0)
    assert e.value.status == B.E_INVALID
    # iteration cap hook: the chain needs 2n-2 passes
    L = gen.chain_tail(50)
    src, lab, dst, _ = dev(L)
    for eng in ENGINES:
        with B.LTS(src, lab, dst, L.n, L.K) as h:
            h.set_option(B.OPT_ENGINE, eng)
            h.set_option(B.OPT_ITER_LIMIT, 10)
            with pytest.raises(B.BisimError) as e:
                h.run()
            assert e.value.status == B.E_ITERCAP
            h.set_option(B.OPT_ITER_LIMIT, 0)  # handle stays usable
            blk, st = h.run()
            assert st.iterations == 98
        with pytest.raises(B.BisimError):
            B.LTS(src, lab, dst, L.n, L.K).set_option(B.OPT_FIRST_SPLITTER, 10**6)


def test_repeat_runs_and_grids_deterministic(B):
    L = gen.planted_quotient(q=1500, deg_mean=6.0, K=8, seed=9)
    src, lab, dst, _ = dev(L)
    res = []
    with B.LTS(src, lab, dst, L.n, L.K) as h:
        for eng, grid in [(1, 0), (1, 7), (2, 0), (2, 3), (3, 0), (3, 5), (1, 0)]:
            h.set_option(B.OPT_ENGINE, eng)
            h.set_option(B.OPT_GRID, grid)
            tr = h.set_trace(4096)
            blk, st = h.run()
            res.append((blk.numpy(), st.iterations, tr[0].numpy()))
    for b, it, t in res[1:]:
        assert (b == res[0][0]).all() and it == res[0][1] and (t == res[0][2]).all()


# --------------------------------------------------------------------------
# full-size workloads (both engines; the per-phase engine is the one the
# benchmark times).  The coarsest partition is unique (Theorem 1 with the
# uniqueness argument of section 4.2), so element-wise equality with the
# Kanellakis-Smolka oracle is the complete check.
# --------------------------------------------------------------------------
@pytest.fixture(scope="module")
def pq1m():
    P = gen.planted_quotient(q=50_000, deg_mean=8.0, K=16, seed=1)
    ks, nb = oracle.ks_coarsest(P.n, P.K, P.src, P.lab, P.dst)
    Q = P.meta["Q"]
    qb, qn = oracle.ks_coarsest(Q.n, Q.K, Q.src, Q.lab, Q.dst)
    assert nb == qn and (ks == lifted_quotient(P, qb)).all()
    return P, ks, nb


@pytest.mark.parametrize("engine", ENGINES)
def test_planted_quotient_1m_full(B, pq1m, engine):
    """~1M states, ~8.2M transitions, 16 actions (Zipf 1.1), copies U{1..40}:
    whole partition vs the Kanellakis-Smolka oracle and the lifted quotient;
    the first 64 iterations' trace vs the lock-step oracle; Theorem 3 bounds."""
    P, ks, nb = pq1m
    r = run_gpu(B, P, engine=engine, trace=64)
    assert (r["block"] == ks).all()
    st = r["stats"]
    assert st.blocks == nb
    assert nb + 1 <= st.iterations <= 3 * P.n - st.pre_blocks + 1
    ref = oracle.alg3_trace(P.n, P.K, P.src, P.lab, P.dst, trace_cap=64, max_iters=64)
    assert (r["C"] == ref["C"]).all() and (r["nsplit"] == ref["nsplit"]).all()


@pytest.mark.parametrize("engine", ENGINES)
def test_chain_100k_full(B, engine):
    L = gen.chain_tail(100_000)
    r = run_gpu(B, L, engine=engine)
    assert r["stats"].iterations == 199_998
    assert (r["block"] == np.arange(100_000)).all()


def _preprocessed(B, L, collide=False):
    """(method, pi_pre, nr_marks) of lts_load on L; collide sets the test
    hook that gives every state the same one-pass key."""
    src, lab, dst, init = dev(L)
    if collide:
        os.environ["BISIM_ONEPASS_COLLIDE"] = "1"
    try:
        h = B.LTS(src, lab, dst, L.n, L.K, init)
    finally:
        os.environ.pop("BISIM_ONEPASS_COLLIDE", None)
    with h:
        pb = B.DeviceArray(max(L.n, 1), np.int32)
        nm = B.DeviceArray(max(L.n, 1), np.int32)
        L_ = B.load_library()
        L_.bisim_get_preprocessed.argtypes = [ctypes.c_void_p] * 3
        L_.bisim_get_preprocessed.restype = ctypes.c_int32
        assert L_.bisim_get_preprocessed(h._h, pb.ptr, nm.ptr) == 0
        return h.preprocess_method(), pb.numpy()[:L.n], nm.numpy()[:L.n]


@pytest.mark.parametrize("case", ["zipf100", "zipf200", "distinct", "init_partition"])
def test_one_pass_preprocessing_matches_the_rounds(B, case):
    """Many actions and at most 64 outgoing transitions per state: pi_pre and
    the action counts come from the one-pass kernels and equal the oracle's
    Algorithm 4 (section 4.1); with every key made to collide the exact check
    fails and the rounds give the same arrays.  The whole refinement then
    matches the oracle (partition, iterations, splitter trace), which also
    checks the action ranks the marks are laid out by."""
    L = {"zipf100": lambda: gen.uniform_zipf(800, 4000, 100, seed=31),
         "zipf200": lambda: gen.uniform_zipf(3000, 12000, 200, seed=32),
         "distinct": lambda: gen.chain_distinct(2000),
         "init_partition": lambda: gen.random_lts(600, 2400, 80, seed=33, init_blocks=5)}[case]()
    pre = oracle.preprocess(L.n, L.K, L.src, L.lab, L.dst, L.init)
    method, pb, nm = _preprocessed(B, L)
    assert method == 1
    assert (pb == pre["pre_block"]).all() and (nm == pre["nr_marks"]).all()
    method_c, pb_c, nm_c = _preprocessed(B, L, collide=True)
    assert method_c == 0
    assert (pb_c == pb).all() and (nm_c == nm).all()
    assert_parity(B, L)


def test_one_pass_preprocessing_not_taken(B):
    # few actions, or a state with more than 64 outgoing transitions: rounds
    assert _preprocessed(B, gen.uniform_zipf(500, 2000, 64, seed=34))[0] == 0
    L = gen.uniform_zipf(100, 8000, 90, seed=35)  # about 80 outgoing transitions per state
    method, pb, nm = _preprocessed(B, L)
    pre = oracle.preprocess(L.n, L.K, L.src, L.lab, L.dst, L.init)
    assert method == 0 and (pb == pre["pre_block"]).all() and (nm == pre["nr_marks"]).all()


@pytest.mark.parametrize("engine", ENGINES)
def test_distinct_actions_chain_full(B, engine):
    """25,217 states, 25,216 transitions, each with an action of its own (the
    shape of Table 1's row with as many actions as transitions): one round of
    the action-by-action preprocessing per action, which alone separates all
    states; then one iteration per block and a final pass."""
    L = gen.chain_distinct(25_217)
    pre = oracle.preprocess(L.n, L.K, L.src, L.lab, L.dst, L.init)
    r = run_gpu(B, L, engine=engine)
    assert r["stats"].pre_blocks == L.n and r["stats"].iterations == L.n + 1
    assert (r["block"] == np.arange(L.n)).all()
    assert (r["block"] == pre["pre_block"]).all()


@pytest.mark.parametrize("engine", ENGINES)
def test_sync_product_full(B, engine):
    P = gen.sync_product(seed=1)
    ks, nb = oracle.ks_coarsest(P.n, P.K, P.src, P.lab, P.dst)
    r = run_gpu(B, P, engine=engine, trace=64)
    assert (r["block"] == ks).all() and r["stats"].blocks == nb
    assert nb + 1 <= r["stats"].iterations <= 3 * P.n - r["stats"].pre_blocks + 1
    ref = oracle.alg3_trace(P.n, P.K, P.src, P.lab, P.dst, trace_cap=64, max_iters=64)
    assert (r["C"] == ref["C"]).all() and (r["nsplit"] == ref["nsplit"]).all()


@pytest.fixture(scope="module")
def pq10m():
    """The 10M-state workload: 487,805 quotient nodes, Poisson(10), Zipf(1.1)
    over 64 actions, copies U{1..40} (~10M states, ~100M transitions)."""
    P = gen.planted_quotient(q=487_805, deg_mean=10.0, K=64, seed=1)
    print(f"[pq10m] n={P.n} m={P.m}", flush=True)
    ks, nb = oracle.ks_coarsest(P.n, P.K, P.src, P.lab, P.dst)
    Q = P.meta["Q"]
    qb, qn = oracle.ks_coarsest(Q.n, Q.K, Q.src, Q.lab, Q.dst)
    assert nb == qn and (ks == lifted_quotient(P, qb)).all()
    print(f"[pq10m] oracle: {nb} blocks", flush=True)
    return P, ks, nb


@pytest.mark.parametrize("engine", [2, 3])
def test_planted_quotient_10m_full(B, pq10m, engine):
    """The 10M-state workload on the per-phase engines: partition bit-exact
    against the oracle, block count, Theorem 3 bounds, and the first 64
    iterations' splitters against the lock-step oracle."""
    P, ks, nb = pq10m
    r = run_gpu(B, P, engine=engine, trace=64)
    st = r["stats"]
    print(f"[pq10m] GPU: #It={st.iterations} in {st.t_alg_ms:.0f} ms", flush=True)
    assert (r["block"] == ks).all()
    assert st.blocks == nb
    assert nb + 1 <= st.iterations <= 3 * P.n - st.pre_blocks + 1
    ref = oracle.alg3_trace(P.n, P.K, P.src, P.lab, P.dst, trace_cap=64, max_iters=64)
    assert (r["C"] == ref["C"]).all() and (r["nsplit"] == ref["nsplit"]).all()


# --------------------------------------------------------------------------
# Algorithm 2 (relational coarsest partition, one action)
# --------------------------------------------------------------------------
def assert_parity_alg2(B, L):
    cap = 3 * L.n + 2
    ref = oracle.alg3_trace(L.n, 1, L.src, L.lab, L.dst, L.init, trace_cap=cap, variant=2)
    ks, nb = oracle.ks_coarsest(L.n, 1, L.src, L.lab, L.dst, L.init)
    for e in ALG2_ENGINES:
        g = run_gpu(B, L, engine=e, trace=cap, algorithm=2)
        assert (g["block"] == ks).all(), (L.name, e)
        st = g["stats"]
        assert st.iterations == ref["iters"], (L.name, e, st.iterations, ref["iters"])
        assert st.blocks == nb and st.pre_blocks == ref["pre_blocks"]
        assert (g["C"] == ref["C"]).all(), (L.name, e)
        assert (g["nsplit"] == ref["nsplit"]).all(), (L.name, e)
    return ref["iters"]


@pytest.mark.parametrize("engine", ALG2_ENGINES)
def test_algorithm2_figure1(B, engine):
    g = json.load(open(os.path.join(GOLD, "figure1.json")))
    L = gen.figure1()
    r = run_gpu(B, L, engine=engine, trace=16, algorithm=2)
    assert r["block"].tolist() == g["final_partition"]
    assert r["stats"].iterations == g["alg2_iterations"]
    assert_parity_alg2(B, L)


def test_algorithm2_kripke_and_random(B):
    cases = [gen.kripke_uniform(1000, 5000, seed=s) for s in (1, 2, 3)]
    cases += [gen.random_lts(n, 4 * n, 1, seed=300 + n, init_blocks=3) for n in (3, 17, 300)]
    cases += [gen.random_lts(n, 2 * n, 1, seed=400 + n) for n in (1, 2)]
    cases += [gen.LTS(5, 1, [], [], [], np.array([0, 1, 0, 1, 4]))]
    for L in cases:
        assert_parity_alg2(B, L)


def test_member_list_engine_runs_algorithm3_only(B):
    L = gen.figure1()
    src, lab, dst, init = dev(L)
    with B.LTS(src, lab, dst, L.n, L.K, init) as h:
        h.set_option(B.OPT_ENGINE, 3)
        h.set_option(B.OPT_ALGORITHM, 2)
        with pytest.raises(B.BisimError) as e:
            h.run()
        assert e.value.status == B.E_UNSUPPORTED
        h.set_option(B.OPT_ALGORITHM, 3)  # the handle stays usable
        blk, st = h.run()
        assert st.iterations == 8


def test_automatic_engine_tunes_once_and_caches(B, tmp_path, monkeypatch):
    """Engine 0 on an LTS of >= 200k states times engines 2 and 3 at a few
    grid sizes on its first iterations, caches the winner, and reuses it;
    the result is the oracle's either way."""
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("BISIM_TUNE_CACHE", str(cache))
    P = gen.planted_quotient(q=12000, deg_mean=8.0, K=16, seed=4)
    assert P.n >= 200_000
    ks, nb = oracle.ks_coarsest(P.n, P.K, P.src, P.lab, P.dst)
    src, lab, dst, _ = dev(P)
    for rep in range(2):
        with B.LTS(src, lab, dst, P.n, P.K) as h:
            blk, st = h.run()
            eng, grid = h.run_config()
        assert (blk.numpy() == ks).all() and st.blocks == nb
        assert eng in (2, 3) and grid > 0
        lines = [l for l in cache.read_text().splitlines() if l.startswith("lts_")]
        assert len(lines) == 1  # tuned on the first handle, cached for the second
        assert lines[0].split()[1] == str(eng)


def test_member_list_engine_graph_replays_match_eager_launches(B):
    """Engine 3 replays captured graphs of 32 iterations unless kernel timing
    is on, which launches kernel by kernel: both give the same partition,
    iteration count and splitter trace, over repeated runs on one handle
    (each graph replayed many times, with eager runs in between)."""
    L = gen.planted_quotient(q=3000, deg_mean=6.0, K=8, seed=21)
    ks, nb = oracle.ks_coarsest(L.n, L.K, L.src, L.lab, L.dst)
    src, lab, dst, _ = dev(L)
    res = []
    with B.LTS(src, lab, dst, L.n, L.K) as h:
        h.set_option(B.OPT_ENGINE, 3)
        tr = h.set_trace(1 << 16)
        for prof in (0, 1, 0, 7, 0):
            h.set_option(B.OPT_PROFILE_EVERY, prof)
            blk, st = h.run()
            res.append((blk.numpy(), st.iterations, tr[0].numpy()[:st.iterations].copy()))
    assert st.iterations > 64  # more than one replay of the graph
    for b, it, c in res:
        assert (b == ks).all() and it == res[0][1] and (c == res[0][2]).all()


def test_algorithm2_needs_one_action(B):
    L = gen.figure2()  # two actions
    src, lab, dst, _ = dev(L)
    with B.LTS(src, lab, dst, L.n, L.K) as h:
        with pytest.raises(B.BisimError) as e:
            h.set_option(B.OPT_ALGORITHM, 2)
        assert e.value.status == B.E_UNSUPPORTED
        with pytest.raises(B.BisimError):
            h.set_option(B.OPT_ALGORITHM, 4)
