"""Host-side logic of bench.py: workload names, the byte models behind the
roofline figures, the standard error and the stored-traffic lookup (no GPU)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_workload_names():
    assert bench.workload("planted-quotient-1M")["make"]
    L = bench.workload("fan-out-12")["make"](__import__("paper_2105_11788_amd.gen").gen)
    assert L.n == 12 and L.m == 3 * 12 - 3  # section 5: n states, 3n - 3 transitions
    with pytest.raises(KeyError):
        bench.workload("no-such-workload")


def test_sem():
    assert bench.sem([1.0]) is None
    xs = [1.0, 2.0, 3.0, 4.0]
    assert bench.sem(xs) == pytest.approx(np.std(xs, ddof=1) / 2.0)


def test_phase_bytes_model():
    # two iterations and the final pass; work columns: members, in-transitions, touched
    n = 1000
    work = np.array([[10, 50, 30, 0], [5, 20, 12, 0], [0, 0, 0, 0]])
    nsplit = np.array([4, 2, 0])
    pb = bench.phase_bytes(n, work, nsplit)
    assert pb.shape == (3, 2) and (pb[-1] == 0).all()
    assert pb[0, 0] == 4 * n + n / 4 + 0 * 20 + 8 * 10 + 40 * 50
    assert pb[1, 0] == 4 * n + n / 4 + 20 * 4 + 8 * 5 + 40 * 20
    assert pb[1, 1] == 4 * n + n / 4 + n / 8 + 16 * 12 + 20 * 2 + 24 * 30


def test_method_bytes_positive_and_final_pass_zero():
    work = np.array([[10, 50, 30, 0], [0, 0, 0, 0]])
    mb = bench.method_bytes(1000, 8000, 5000, work, np.array([3, 0]))
    assert mb.shape == (2, 2) and (mb[0] > 0).all() and (mb[-1] == 0).all()


def test_stored_traffic_unknown_kernel_is_null():
    assert bench.stored_traffic("k_no_such_kernel", "planted-quotient-1M") is None


def test_cpu_baseline_batch_small():
    from paper_2105_11788_amd import gen
    insts = gen.batch(count=8, n_lo=50, n_hi=300, seed=3)
    its = np.arange(8) + 10
    r = bench.cpu_baseline_batch(insts, its, 8, 300, target_s=0.2, workers=2)
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["value"] > 0
    assert r["all_cores"]["cores"] == 2 and r["all_cores"]["value"] > 0


def test_cpu_baseline_batch_checks_partitions():
    import oracle
    from paper_2105_11788_amd import gen
    insts = gen.batch(count=6, n_lo=50, n_hi=200, seed=4)
    its = np.arange(6) + 10
    good = [oracle.ks_coarsest(L.n, L.K, L.src, L.lab, L.dst, L.init)[0] for L in insts]
    r = bench.cpu_baseline_batch(insts, its, 6, 200, target_s=10.0, workers=1, gpu_blocks=good)
    assert r["partition_equal_to_gpu"] and r["instances_equal_to_gpu"] == "6 of 6"
    bad = [b.copy() for b in good]
    k = int(np.argmax([L.n for L in insts]))
    bad[k][-1] = bad[k][-1] + 1  # a planted mistake in one instance
    r = bench.cpu_baseline_batch(insts, its, 6, 200, target_s=10.0, workers=1, gpu_blocks=bad)
    assert not r["partition_equal_to_gpu"] and r["instances_equal_to_gpu"] == "5 of 6"


def test_cpu_baseline_single_checks_partition():
    import oracle
    from paper_2105_11788_amd import gen
    L = gen.kripke_uniform(300, 1500, seed=2)
    ks, nb = oracle.ks_coarsest(L.n, L.K, L.src, L.lab, L.dst, L.init)
    r = bench.cpu_baseline(L, 500, ks, target_s=0.05)
    assert r["partition_equal_to_gpu"] and r["blocks"] == nb and r["cores"] == 1
    assert r["value"] == pytest.approx(L.m * 500 / r["seconds_to_fixpoint"])
    wrong = ks.copy()
    wrong[-1] = wrong[-1] + 1 if wrong[-1] + 1 < L.n else 0
    assert not bench.cpu_baseline(L, 500, wrong, target_s=0.0)["partition_equal_to_gpu"]


def test_lists_bytes_model():
    w = {"members": 100, "in_transitions": 600, "touched": 300, "segments": 4,
         "member_visits": 2000, "split_states": 50, "split_blocks": 5, "split_iterations": 3}
    n, iters = 6400, 11  # ten working iterations and the final pass
    lb = bench.lists_bytes(n, iters, w)
    assert len(lb) == 3
    assert lb[0] == pytest.approx((8 * 10 + 8 * 100 + 52 * 600 + 16 * 300 + 12 * 4) / 10)
    # ten splitters of ten members each: ten prefetches of 28 + 16 x 10 bytes
    assert lb[1] == pytest.approx((24 * 300 + 56 * 50 + 24 * 4 + 12 * 2000 + 10 * (28 + 160)) / 10)
    assert lb[2] == pytest.approx((32 * 300 + 96 * 50 + 8 * 3 + 76 * 50 + 64 * 5) / 10)


def test_batch_bytes_model():
    sizes = [10, 5000, 300, 20000]
    st = {"global_instances": 2,
          "work": [[7, 40, 90, 0, 0, 0, 0, 2], [100, 30, 200, 80, 10, 500, 20, 4]]}
    got = bench.batch_bytes(sizes, st, 4)
    n_list = 20000 + 5000  # the two largest instances take the member-list tier
    exp = 8 * sum(sizes) + 8 * 40 + 8 * 90 + 76 * n_list + 8 * 100 + 8 * 30 + 16 * 200 \
        + 24 * 80 + 4 * 500 + 132 * 20 + 24 * 4
    assert got == pytest.approx(exp)
