"""GPU test of coarsest_partition_noalloc (the allocation-free entry point):
its partitions, iteration and block counts equal those of lts_load +
coarsest_partition on the same inputs, over consecutive calls that reuse the
static region (a larger LTS, then a smaller one, then the larger one again);
inputs beyond the region are rejected; the calls take no device memory."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_2105_11788_amd import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    from paper_2105_11788_amd import bisim
    bisim.load_library()
    if bisim.device_count() < 1:
        pytest.skip("no GPU")
    return bisim


def dev(B, a):
    return B.DeviceArray.from_numpy(np.ascontiguousarray(a, dtype=np.int32))


def free_bytes(B):
    H = B.hip()
    f, t = ctypes.c_size_t(0), ctypes.c_size_t(0)
    H.hipMemGetInfo.argtypes = [ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    H.hipMemGetInfo.restype = ctypes.c_int
    assert H.hipMemGetInfo(ctypes.byref(f), ctypes.byref(t)) == 0
    return f.value


def reference(B, L, d):
    with B.LTS(d["src"], d["lab"], d["dst"], L.n, L.K, d["init"]) as h:
        out, st = h.run()
        return out.numpy(), st


def test_noalloc_matches_handle_calls(B):
    big = gen.planted_quotient(q=4000, deg_mean=8.0, K=16, seed=3)   # ~82k states, ~650k tr.
    small = gen.kripke_uniform(1000, 5000, seed=2)                   # 1000 states, pi_0 given
    wide = gen.uniform_lts(3000, 100.0, 200, seed=4)                 # > 64 actions per state
    cases = []
    for L in (big, small, wide):
        d = {"src": dev(B, L.src), "lab": dev(B, L.lab), "dst": dev(B, L.dst),
             "init": None if L.init is None else dev(B, L.init)}
        ref, rst = reference(B, L, d)
        ks, nb = oracle.ks_coarsest(L.n, L.K, L.src, L.lab, L.dst, L.init)
        assert (ref == ks).all() and rst.blocks == nb
        cases.append((L, d, ref, rst, B.DeviceArray(L.n, np.int32)))
    print(f"[noalloc] sizes {[(c[0].n, c[0].m, c[0].K) for c in cases]}", flush=True)
    # warm-up call: the first call on a device loads the region
    L, d, ref, rst, out = cases[1]
    B.coarsest_partition_noalloc(d["src"], d["lab"], d["dst"], L.n, L.K, d["init"], out)
    free0 = free_bytes(B)
    for idx in (0, 1, 2, 0, 1):  # larger, then smaller inputs, reusing the region
        L, d, ref, rst, out = cases[idx]
        out.fill(0xFF)
        st = B.coarsest_partition_noalloc(d["src"], d["lab"], d["dst"], L.n, L.K, d["init"], out)
        got = out.numpy()
        print(f"[noalloc] case {idx}: n={L.n} #It={st.iterations} blocks={st.blocks}", flush=True)
        assert (got == ref).all(), idx
        assert st.iterations == rst.iterations and st.blocks == rst.blocks, idx
        assert st.pre_blocks == rst.pre_blocks and st.mark_length == rst.mark_length, idx
    assert free_bytes(B) >= free0  # nothing was allocated on the device


def test_noalloc_rejects_beyond_region(B):
    n = B.NOALLOC_SCRATCH_BYTES // 64
    src = B.DeviceArray(1, np.int32).fill(0)
    out = B.DeviceArray(16, np.int32).fill(0x11)
    with pytest.raises(B.BisimError) as e:
        B.coarsest_partition_noalloc(B.DeviceArray(0, np.int32), src, src, n, 1, None,
                                     type("O", (), {"ptr": out.ptr, "count": n})())
    assert e.value.status == B.E_UNSUPPORTED
    assert (out.numpy() == 0x11111111).all()  # nothing was written


def test_noalloc_range_error_and_empty(B):
    L = gen.kripke_uniform(50, 200, seed=5)
    bad = L.dst.copy()
    bad[7] = L.n  # a target outside [0, n)
    out = B.DeviceArray(L.n, np.int32)
    with pytest.raises(B.BisimError) as e:
        B.coarsest_partition_noalloc(dev(B, L.src), dev(B, L.lab), dev(B, bad), L.n, L.K, None,
                                     out)
    assert e.value.status == B.E_RANGE
    # the region stays usable after an error, and empty inputs work
    st = B.coarsest_partition_noalloc(dev(B, L.src), dev(B, L.lab), dev(B, L.dst), L.n, L.K,
                                      dev(B, L.init), out)
    ks, nb = oracle.ks_coarsest(L.n, L.K, L.src, L.lab, L.dst, L.init)
    assert (out.numpy() == ks).all() and st.blocks == nb
    e0 = B.DeviceArray(0, np.int32)
    st = B.coarsest_partition_noalloc(e0, e0, e0, 0, 1, None, None)
    assert st.blocks == 0
