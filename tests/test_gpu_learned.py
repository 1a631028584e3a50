"""GPU parity for the learned splitter: the network kernels against the fp64
reference (forward within a derived fp32 error bound, gradients, Adam),
the training-data collector against features and counterfactual targets
recomputed from their definitions on the oracle's trace, the learned policy's
partition against the oracle (bit-exact), and what a trained network gains."""
import math
from collections import defaultdict

import numpy as np
import pytest

import oracle
from oracle import mlp as ref
from paper_2105_11788_amd import gen

pytestmark = pytest.mark.gpu
U = 2.0 ** -24  # fp32 unit roundoff


@pytest.fixture(scope="module")
def B():
    from paper_2105_11788_amd import bisim
    bisim.load_library()
    assert bisim.device_count() > 0, "GPU tests need a GPU"
    return bisim


def forward_error_bound(w, x, F):
    """Worst-case fp32 accumulation error of the network (inputs and parameters
    already bf16): each dot product of L terms errs by at most L*u times the
    sum of its absolute terms, plus the propagated error of its inputs (ReLU is
    1-Lipschitz)."""
    _, c = ref.forward(w, x, F)
    p = c["p"]
    A1 = np.abs(c["x"]) @ np.abs(p["W1"]).T + np.abs(p["b1"])
    e1 = (F + 1) * U * A1
    A2 = np.abs(c["h1"]) @ np.abs(p["W2"]).T + np.abs(p["b2"])
    e2 = (ref.H + 1) * U * A2 + e1 @ np.abs(p["W2"]).T
    A3 = np.abs(c["h2"]) @ np.abs(p["w3"]) + abs(p["b3"][0])
    e3 = (ref.H + 1) * U * A3 + e2 @ np.abs(p["w3"])
    return e3


@pytest.mark.parametrize("F", [19, 5])
def test_mlp_forward_matches_reference(B, F):
    rng = np.random.default_rng(F)
    w = ref.he_init(F, seed=F)
    w[-1] = 0.37  # non-zero output bias
    x = (rng.random((2000, F)) * 8.0).astype(np.float32)
    net = B.MLP(F, init=w)
    y = net.forward(x)
    yr, _ = ref.forward(w, x, F)
    bound = forward_error_bound(w, x, F)
    assert (np.abs(y - yr) <= 2 * bound + 1e-30).all(), np.max(np.abs(y - yr) / (bound + 1e-30))


def test_mlp_gradient_and_adam_match_reference(B):
    F = 19
    rng = np.random.default_rng(3)
    w = ref.he_init(F, seed=11)
    x = (rng.random((512, F)) * 6.0).astype(np.float32)
    t = rng.normal(size=512).astype(np.float32)
    net = B.MLP(F, init=w)
    loss, g = net.train_step(x, t, lr=0.0, want_grad=True)
    lr_, gr = ref.loss_and_grad(w, x, t, F)
    assert abs(loss - lr_) <= 1e-4 * (1 + lr_)
    # fp32 sums over 512 rows and 64 units: relative error ~ 600 * 2^-24 ~ 4e-5 of
    # the summed magnitudes; compare against the gradient's max-norm
    scale = np.max(np.abs(gr))
    assert np.max(np.abs(g - gr)) <= 1e-3 * scale
    # Adam's first step moves each parameter by lr * sign(g) (bias-corrected)
    lr = 1e-3
    net2 = B.MLP(F, init=w)
    net2.train_step(x, t, lr=lr)
    w1 = net2.params()
    wr, _, _ = ref.adam_step(w, gr, np.zeros_like(gr), np.zeros_like(gr), 1, lr)
    clear = np.abs(gr) > 1e-3 * scale  # sign unambiguous
    assert np.allclose(w1[clear], wr[clear], atol=1e-6, rtol=0)
    assert np.all(np.abs(w1 - w) <= lr * (1 + 1e-3) + 1e-7)


def test_mlp_forward_bf16_inputs(B):
    """bf16 inputs give exactly what fp32 inputs of the same values give (the
    forward pass rounds its inputs to bf16 either way)."""
    F = 19
    rng = np.random.default_rng(4)
    x = (rng.random((1000, F)) * 8.0).astype(np.float32)
    bits = (x.view(np.uint32) >> 16).astype(np.uint16)  # truncation: exact bf16 values
    xb = (bits.astype(np.uint32) << 16).view(np.float32)
    net = B.MLP(F, seed=3)
    y32 = net.forward(np.ascontiguousarray(xb))
    y16 = net.forward_bf16(bits)
    assert np.array_equal(y32, y16)


def test_mlp_training_is_reproducible(B):
    """The gradient is summed without floating-point atomics (workgroup
    partials added in a fixed order), so identical steps give identical
    gradients and identical parameters, bit for bit."""
    F = 19
    rng = np.random.default_rng(8)
    w = ref.he_init(F, seed=12)
    x = (rng.random((20000, F)) * 5.0).astype(np.float32)
    t = rng.normal(size=20000).astype(np.float32)
    xd, td = B.DeviceArray.from_numpy(x), B.DeviceArray.from_numpy(t)
    runs = []
    for _ in range(2):
        net = B.MLP(F, init=w)
        loss, g = net.train_step(xd, td, lr=0.0, want_grad=True)
        for _ in range(5):
            net.train_step(xd, td, lr=1e-3)
        runs.append((loss, g, net.params()))
    assert runs[0][0] == runs[1][0]
    assert np.array_equal(runs[0][1], runs[1][1])
    assert np.array_equal(runs[0][2], runs[1][2])


def test_mlp_training_reduces_loss(B):
    F = 19
    rng = np.random.default_rng(5)
    x = (rng.random((4096, F)) * 4).astype(np.float32)
    t = (np.sin(x[:, 0]) + 0.3 * x[:, 3]).astype(np.float32)
    net = B.MLP(F, seed=1)
    xd, td = B.DeviceArray.from_numpy(x), B.DeviceArray.from_numpy(t)
    losses = [net.train_step(xd, td, lr=3e-3) for _ in range(300)]
    assert losses[-1] < 0.2 * losses[0]


def _dev(B, L):
    t = lambda a: B.DeviceArray.from_numpy(a, np.int32)
    return t(L.src), t(L.lab), t(L.dst), (None if L.init is None else t(L.init))


def test_learned_policy_partition_exact(B):
    net = B.MLP(B.POLICY_FEATURES, seed=3)
    cases = [gen.figure1(), gen.figure2(), gen.fan_out(50), gen.chain_tail(200),
             gen.kripke_uniform(1000, 5000, seed=2), gen.uniform_zipf(800, 4000, 64, seed=3),
             gen.planted_quotient(q=300, deg_mean=6.0, K=16, seed=4)]
    for L in cases:
        ks, nb = oracle.ks_coarsest(L.n, L.K, L.src, L.lab, L.dst, L.init)
        its = {}
        for engine in (1, 2):
            for R in (1, 7, 64):
                src, lab, dst, init = _dev(B, L)
                with B.LTS(src, lab, dst, L.n, L.K, init) as h:
                    h.set_option(B.OPT_ENGINE, engine)
                    B.set_splitter_policy(h, B.POLICY_LEARNED, net, R)
                    blk, st = h.run()
                    b1 = blk.numpy()
                    blk2, st2 = h.run()  # deterministic repeat
                assert (b1 == ks).all(), (L.name, engine, R)
                assert (blk2.numpy() == b1).all() and st2.iterations == st.iterations
                assert nb + 1 <= st.iterations <= 3 * L.n - st.pre_blocks + 1
                its.setdefault(R, set()).add(st.iterations)
        # both engines follow the same splitter order
        assert all(len(v) == 1 for v in its.values()), (L.name, its)


def _trace_state(L, k):
    """Partition at the start of iteration k, and for each label the number
    of iterations completed when its block was created or last split ('born')
    and when it was last the splitter ('used'), from the lock-step oracle."""
    pp = oracle.preprocess(L.n, L.K, L.src, L.lab, L.dst, L.init)
    r = oracle.alg3_trace(L.n, L.K, L.src, L.lab, L.dst, L.init, trace_cap=k + 1,
                          keep_blocks=True)
    parts = [pp["pre_block"]] + [r["blocks"][i] for i in range(min(k, r["iters"]))]
    born = np.zeros(L.n, np.int64)
    used = np.zeros(L.n, np.int64)
    for i in range(1, len(parts)):
        before, after = parts[i - 1], parts[i]
        changed = np.nonzero(before != after)[0]
        for s in changed:
            born[before[s]] = i
            born[after[s]] = i
        used[r["C"][i - 1]] = i
    return parts[min(k, len(parts) - 1)], born, used


def test_collector_matches_definitions(B):
    L = gen.uniform_zipf(300, 1500, 12, seed=21)
    src, lab, dst, init = _dev(B, L)
    with B.LTS(src, lab, dst, L.n, L.K, init) as h:
        f, t, meta = B.collect_training(h, sample_every=5, max_cands=6, cap=5000)
    assert f.shape[0] > 20
    assert set(np.unique(f[:, 18]).tolist()) == {0.0, 1.0}  # both values of the flag occur
    S, A, D = L.src, L.lab, L.dst
    cache = {}
    for row in range(f.shape[0]):
        k, X = int(meta[row, 0]), int(meta[row, 1])
        if k not in cache:
            cache[k] = _trace_state(L, k)
        block, born, used = cache[k]
        assert block[X] == X
        mem = block == X
        size = mem.sum()
        out8 = [np.sum(mem[S] & (A % 8 == q)) for q in range(8)]
        in8 = [np.sum(mem[D] & (A % 8 == q)) for q in range(8)]
        exp = np.log1p(np.array([size, *out8, *in8, k - born[X]], np.float64))
        exp = np.append(exp, 1.0 if used[X] > born[X] else 0.0).astype(np.float32)
        assert np.allclose(f[row], exp, rtol=2e-6, atol=0), (row, k, X, f[row], exp)
        marked = defaultdict(set)
        for s, a, d in zip(S, A, D):
            if block[d] == X:
                marked[s].add(a)
        split_blocks = {block[s] for s in range(L.n) if marked[s] != marked[block[s]]}
        assert math.isclose(t[row], math.log1p(len(split_blocks)), rel_tol=2e-6), (row, k, X)


def test_trained_network_gain(B, capsys):
    from paper_2105_11788_amd import learn
    mlp, losses, rows = learn.train_policy(train_seeds=range(1001, 1013), steps=300)
    assert losses[-1] < 0.7 * losses[0]
    res = []
    for regime in ("kripke", "zipf64"):
        for s in range(2001, 2007):
            L = learn.training_lts(regime, s)
            ks, _ = oracle.ks_coarsest(L.n, L.K, L.src, L.lab, L.dst, L.init)
            ip, bp, _ = learn.iterations(L)
            il, bl, _ = learn.iterations(L, mlp)
            assert (bp == ks).all() and (bl == ks).all()
            res.append((regime, ip, il))
    with capsys.disabled():
        for regime, ip, il in res:
            print(f"[learned] {regime}: plain #It {ip}  learned #It {il}  ratio {il / ip:.3f}")
    ratio = np.mean([il / ip for _, ip, il in res])
    kripke = np.mean([il / ip for r, ip, il in res if r == "kripke"])
    print(f"[learned] mean #It ratio learned/plain = {ratio:.3f} over {len(res)} held-out LTSs "
          f"(one-action Kripke structures {kripke:.3f})")
    # the network must cut the iteration count on held-out LTSs of the
    # training shape: by at least 2 % on average, and on the one-action
    # Kripke structures (where a re-chosen unchanged splitter is useless) by
    # at least 3 %
    assert ratio < 0.98, ratio
    assert kripke < 0.97, kripke
