"""GPU parity for the batched engine: every instance of a batch equals the
oracle (partition bit-exact, #It equal to the lock-step oracle's), in both
storage tiers (LDS-resident and global), for several workgroup sizes."""
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


def mixed_instances():
    out = [gen.figure1(), gen.figure2(), gen.fan_out(40), gen.chain_tail(300),
           gen.LTS(0, 1, [], [], []),                                   # empty
           gen.LTS(7, 2, [], [], [], np.array([0, 0, 2, 2, 0, 5, 5])),   # no transitions
           gen.kripke_uniform(1000, 5000, seed=3),
           gen.planted_quotient(q=120, deg_mean=4.0, K=8, seed=4)]
    rng = np.random.default_rng(11)
    for k in range(40):
        n = int(rng.integers(1, 400))
        out.append(gen.random_lts(n, int(rng.integers(0, 5 * n)), int(rng.integers(1, 30)),
                                  seed=900 + k, init_blocks=int(rng.integers(0, 4))))
    return out


def check(B, insts, blocks, its, trace_every=1):
    for k, L in enumerate(insts):
        ks, nb = oracle.ks_coarsest(L.n, L.K, L.src, L.lab, L.dst, L.init)
        assert (blocks[k] == ks).all(), (k, L.name)
        if k % trace_every == 0:
            r = oracle.alg3_trace(L.n, L.K, L.src, L.lab, L.dst, L.init)
            assert its[k] == r["iters"], (k, L.name, its[k], r["iters"])


SPILL_SKIP = pytest.mark.skip(
    reason="512- and 1024-thread builds of the batched kernel are switched off: builds that "
           "spilled 212-332 bytes per lane made illegal memory accesses and the cause is "
           "not found; the kernel is built for 256 threads only")


@pytest.mark.parametrize("wg,lds", [
    (256, 0), (256, 1024), (256, 1 << 14), (256, 40000),
    pytest.param(1024, 0, marks=SPILL_SKIP), pytest.param(1024, 1 << 14, marks=SPILL_SKIP),
    pytest.param(512, 1024, marks=SPILL_SKIP)])
def test_mixed_batch_tiers(B, wg, lds):
    insts = mixed_instances()
    with B.Batch(insts) as b:
        b.set_option(B.BOPT_WG_SIZE, wg)
        if lds:
            b.set_option(B.BOPT_LDS_LIMIT, lds)
        out, its, st = b.run()
        blocks = b.split(out.numpy())
    check(B, insts, blocks, its)
    if lds:
        # LDS bytes an instance needs: 3 bitmaps, 64-bit bids, mark words
        # (32-bit when every K <= 32), block ids
        mask = 8 if max(x.K for x in insts) > 32 else 4
        need = lambda n: 24 * ((n + 63) // 64) + 8 * n + ((mask * n + 7) // 8) * 8 + 4 * n
        assert st["lds_instances"] == sum(need(x.n) <= lds for x in insts)
        assert st["global_instances"] == len(insts) - st["lds_instances"] > 0
    assert st["max_iterations"] == its.max() and st["sum_iterations"] == its.sum()


def test_batch_autotuned_and_repeatable(B, tmp_path, monkeypatch):
    monkeypatch.setenv("BISIM_TUNE_CACHE", str(tmp_path / "tune.txt"))
    insts = mixed_instances()
    with B.Batch(insts) as b:
        out1, its1, st1 = b.run()
        r1 = out1.numpy()
        out2, its2, st2 = b.run()
        assert (out2.numpy() == r1).all() and (its1 == its2).all()
        blocks = b.split(r1)
    check(B, insts, blocks, its1)
    assert (tmp_path / "tune.txt").exists()
    # a second handle reads the cached choice
    with B.Batch(insts) as b2:
        out3, its3, st3 = b2.run()
        assert (out3.numpy() == r1).all()
        assert (st3["workgroup_size"], st3["grid"]) == (st1["workgroup_size"], st1["grid"])


def test_batch_matches_single_instance_runs(B):
    insts = [gen.planted_quotient(q=300, deg_mean=6.0, K=12, seed=s) for s in range(4)]
    with B.Batch(insts) as b:
        out, its, _ = b.run()
        blocks = b.split(out.numpy())
    for k, L in enumerate(insts):
        t = lambda a: B.DeviceArray.from_numpy(a, np.int32)
        with B.LTS(t(L.src), t(L.lab), t(L.dst), L.n, L.K) as h:
            blk, st = h.run()
        assert (blk.numpy() == blocks[k]).all() and st.iterations == its[k]


def test_batch_many_small(B):
    insts = gen.batch(count=1024, n_lo=10, n_hi=2000, seed=5)
    with B.Batch(insts) as b:
        out, its, st = b.run()
        blocks = b.split(out.numpy())
    check(B, insts, blocks, its, trace_every=16)


def test_batch_errors(B):
    bad = gen.LTS(3, 2, [0], [1], [3])  # target outside the instance
    with pytest.raises(B.BisimError) as e:
        B.Batch([gen.figure2(), bad])
    assert e.value.status == B.E_RANGE
    lab_bad = gen.LTS(3, 1, [0], [1], [2])  # label >= K of its instance
    with pytest.raises(B.BisimError) as e:
        B.Batch([lab_bad])
    assert e.value.status == B.E_RANGE
    wide = gen.LTS(2, 100, np.zeros(70, np.int32), np.arange(70), np.ones(70, np.int32))
    with pytest.raises(B.BisimError) as e:
        B.Batch([wide])
    assert e.value.status == B.E_UNSUPPORTED


def test_batch_4096_up_to_200k_full(B):
    """The full batch shape (4096 instances, log-uniform 100..200k states,
    ~0.65G transitions): every instance's partition against the oracle
    (computed over a pool of host processes), in two launch configurations
    at the ends of the autotuner's range (the whole LDS, so most instances
    are LDS-resident and the large ones keep their bitmaps and lists in LDS;
    a 16 KiB LDS budget, so most take the global-memory tier), with
    identical per-instance iteration counts; #It vs the lock-step oracle on
    a sample of small instances."""
    import ks_workers
    count, n_lo, n_hi = 4096, 100, 200_000
    insts = gen.batch(count=count, n_lo=n_lo, n_hi=n_hi, seed=1)
    print(f"[batch-200k] generated {len(insts)} instances", flush=True)
    runs = []
    with B.Batch(insts) as b:
        for wg, lds in [(256, 0), (256, 16384)]:
            b.set_option(B.BOPT_WG_SIZE, wg)
            b.set_option(B.BOPT_LDS_LIMIT, lds)
            out, its, st = b.run()
            runs.append((b.split(out.numpy()), its.copy(), dict(st)))
            print(f"[batch-200k] wg {wg} lds {lds}: max #It {its.max()}, lds/global instances "
                  f"{st['lds_instances']}/{st['global_instances']}, {st['t_alg_ms']:.0f} ms",
                  flush=True)
    assert runs[0][2]["global_instances"] > 0 and runs[1][2]["global_instances"] > \
        runs[0][2]["global_instances"]
    assert (runs[0][1] == runs[1][1]).all()
    ref = ks_workers.ks_batch(range(count), count, n_lo, n_hi, seed=1)
    print("[batch-200k] oracle done", flush=True)
    for k in range(count):
        ks, nb = ref[k]
        for blocks, its, _ in runs:
            assert (blocks[k] == ks).all(), (k, insts[k].n)
        assert runs[0][1][k] >= nb + 1, k
    rng = np.random.default_rng(7)
    small = [k for k in range(count) if insts[k].n <= 3000]
    for k in rng.choice(small, 24, replace=False):
        L = insts[int(k)]
        r = oracle.alg3_trace(L.n, L.K, L.src, L.lab, L.dst, L.init)
        assert runs[0][1][int(k)] == r["iters"], (int(k), r["iters"])


def test_batch_4096_up_to_10k_full(B):
    """4096 instances, log-uniform 100..10k states, Poisson(6), K ~ U{1..32},
    half planted: every instance's partition vs the oracle, #It on a sample."""
    insts = gen.batch(count=4096, n_lo=100, n_hi=10_000, seed=1)
    with B.Batch(insts) as b:
        out, its, st = b.run()
        blocks = b.split(out.numpy())
    check(B, insts, blocks, its, trace_every=64)
