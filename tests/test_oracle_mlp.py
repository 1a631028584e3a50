"""Pins for the fp64 network reference: the bf16 rounding definition,
central finite differences of the loss, a hand-computed tiny forward pass,
and Adam's first step."""
import numpy as np

from oracle import mlp


def test_bf16_rounding_definition():
    f = np.float32
    vals = np.array([1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-9, 1.0 + 2**-7 + 2**-8, -2.5, 0.0,
                     65504.0, 1e-40], np.float32)
    got = mlp.bf16_round(vals)
    # 1+2^-8 is a tie between 1 and 1+2^-7 -> even (1.0); 1+3*2^-9 rounds up;
    # 1+2^-7+2^-8 is a tie between 1+2^-7 (odd) and 1+2^-6 -> 1+2^-6
    exp = np.array([1.0, 1.0, 1.0 + 2**-7, 1.0 + 2**-6, -2.5, 0.0, 65536.0, 0.0], np.float32)
    assert got[:7].tolist() == exp[:7].tolist()
    # a subnormal keeps its top 16 bits: 1e-40 is 0x000116C2, the dropped half
    # 0x16C2 is below 0x8000, so it rounds down to 0x00010000
    assert got[7:8].view(np.uint32)[0] == 0x00010000
    # idempotent, and exact for values with <= 8 significant bits
    assert (mlp.bf16_round(got) == got).all()
    assert mlp.bf16_round(f(0.15625))[()] == f(0.15625)


def test_tiny_forward_by_hand():
    F = 2
    p = {k: np.zeros(s, np.float32) for k, s in mlp.shapes(F).items()}
    p["W1"][0] = [1.0, -1.0]
    p["W1"][1] = [0.5, 0.5]
    p["b1"][0] = 0.25
    p["W2"][0, 0] = 2.0
    p["W2"][1, 1] = -1.0
    p["W2"][2, 1] = 3.0
    p["w3"][0] = 1.0
    p["w3"][2] = 0.5
    p["b3"][0] = -1.0
    flat = mlp.flatten(p)
    x = np.array([[3.0, 1.0], [0.0, 2.0]], np.float32)
    # row 0: h1 = [relu(3-1+0.25)=2.25, relu(2)=2]; z2 = [4.5, -2, 6]; h2 = [4.5, 0, 6]
    #        y = 4.5 + 0.5*6 - 1 = 6.5
    # row 1: h1 = [relu(-2+0.25)=0, relu(1)=1]; z2 = [0, -1, 3]; y = 0 + 1.5 - 1 = 0.5
    y, _ = mlp.forward(flat, x, F)
    assert y.tolist() == [6.5, 0.5]


def test_gradient_matches_central_differences():
    F = 5
    rng = np.random.default_rng(0)
    w = mlp.he_init(F, seed=3)
    x = rng.normal(size=(7, F)).astype(np.float32)
    t = rng.normal(size=7)
    # differentiate the fp64 function of the (already rounded) parameters
    wr = mlp.bf16_round(w).astype(np.float64)
    xr = mlp.bf16_round(x).astype(np.float64)
    loss, g = mlp.loss_and_grad(wr, xr, t, F, round_bf16=False)
    eps = 1e-6
    idx = rng.choice(wr.size, 60, replace=False)
    for i in idx:
        wp, wm = wr.copy(), wr.copy()
        wp[i] += eps
        wm[i] -= eps
        lp, _ = mlp.loss_and_grad(wp, xr, t, F, round_bf16=False)
        lm, _ = mlp.loss_and_grad(wm, xr, t, F, round_bf16=False)
        num = (lp - lm) / (2 * eps)
        assert abs(num - g[i]) <= 1e-6 + 1e-5 * abs(num), (i, num, g[i])


def test_adam_first_step_moves_by_lr():
    # with bias correction the first step is lr * g / (|g| + eps) = lr * sign(g)
    w = np.array([1.0, -2.0, 0.5], np.float32)
    g = np.array([0.3, -4.0, 0.0])
    w1, m, v = mlp.adam_step(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(w1, [0.99, -1.99, 0.5], atol=1e-6)


def test_param_count():
    assert mlp.n_params(18) == 64 * 18 + 64 + 64 * 64 + 64 + 64 + 1
