"""fp64 reference of the splitter-scoring network (test infrastructure only).

Network (a reading: the paper has no learning; the sizes come from the
build's brief): y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 with W1 [H, F],
W2 [H, H], w3 [H], H = 64.  Parameters are held as fp32 master values; the
forward pass uses bf16 copies of every parameter and of the input (rounded
to nearest, ties to even) and accumulates in floating point; activations are
not rounded.  Loss: mean squared error.  Optimiser: Adam on the fp32 masters,
gradients taken with respect to the bf16 copies.

This module computes all of that in fp64 from the definitions, for
comparison with the GPU kernels.
"""
from __future__ import annotations

import numpy as np

H = 64
PARAM_ORDER = ("W1", "b1", "W2", "b2", "w3", "b3")


def bf16_round(x) -> np.ndarray:
    """Round fp32 values to the nearest bf16 (ties to even), returned as fp32.
    bf16 keeps the fp32 sign, exponent and top 7 fraction bits."""
    a = np.ascontiguousarray(np.asarray(x, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a)
    out = r.astype(np.uint32).view(np.float32).copy()
    out[nan] = np.nan
    return out


def shapes(F: int):
    return {"W1": (H, F), "b1": (H,), "W2": (H, H), "b2": (H,), "w3": (H,), "b3": (1,)}


def n_params(F: int) -> int:
    return int(sum(np.prod(s) for s in shapes(F).values()))


def unflatten(flat, F: int):
    flat = np.asarray(flat)
    out, o = {}, 0
    for k in PARAM_ORDER:
        s = shapes(F)[k]
        c = int(np.prod(s))
        out[k] = flat[o:o + c].reshape(s)
        o += c
    assert o == flat.size
    return out


def flatten(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[k]).reshape(-1) for k in PARAM_ORDER])


def forward(flat_fp32, x, F: int, round_bf16: bool = True):
    """Returns (y [B], cache).  flat_fp32: master parameters; x [B, F]."""
    if round_bf16:
        p = unflatten(np.asarray(flat_fp32, np.float32), F)
        p = {k: bf16_round(v).astype(np.float64) for k, v in p.items()}
        x = bf16_round(np.asarray(x, np.float32)).astype(np.float64)
    else:  # plain fp64 function of the given values
        p = unflatten(np.asarray(flat_fp32, np.float64), F)
        x = np.asarray(x, np.float64)
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["w3"] + p["b3"][0]
    return y, {"p": p, "x": x, "z1": z1, "h1": h1, "z2": z2, "h2": h2}


def loss_and_grad(flat_fp32, x, t, F: int, round_bf16: bool = True):
    """MSE loss (1/B) sum (y - t)^2 and its gradient w.r.t. the parameters
    used by the forward pass (flattened in PARAM_ORDER)."""
    y, c = forward(flat_fp32, x, F, round_bf16)
    t = np.asarray(t, np.float64)
    B = y.shape[0]
    loss = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / B
    p = c["p"]
    g = {}
    g["w3"] = c["h2"].T @ dy
    g["b3"] = np.array([dy.sum()])
    dh2 = np.outer(dy, p["w3"])
    dz2 = dh2 * (c["z2"] > 0)
    g["W2"] = dz2.T @ c["h1"]
    g["b2"] = dz2.sum(0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (c["z1"] > 0)
    g["W1"] = dz1.T @ c["x"]
    g["b1"] = dz1.sum(0)
    return loss, flatten(g)


def adam_step(flat_fp32, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (bias-corrected) of the fp32 master parameters, in fp64;
    returns (new master fp32, m, v)."""
    w = np.asarray(flat_fp32, np.float64)
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    w = w - lr * mh / (np.sqrt(vh) + eps)
    return w.astype(np.float32), m, v


def he_init(F: int, seed: int) -> np.ndarray:
    """He-normal weights, zero biases (fp32), from a numpy PCG64 stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = {"W1": rng.normal(0, np.sqrt(2.0 / F), (H, F)), "b1": np.zeros(H),
         "W2": rng.normal(0, np.sqrt(2.0 / H), (H, H)), "b2": np.zeros(H),
         "w3": rng.normal(0, np.sqrt(1.0 / H), (H,)), "b3": np.zeros(1)}
    return flatten(p).astype(np.float32)
