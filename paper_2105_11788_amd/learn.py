"""Training the splitter-priority network on the plain method's own traces.

Pipeline (all arithmetic on the GPU, through the C ABI):
  1. plain refinement runs on training LTSs with sampled candidates:
     per sampled unstable block, its 19 features and the counterfactual
     target log(1 + blocks that would split if it were the splitter now)
     (bisim_collect_training);
  2. full-batch Adam on the mean squared error (mlp_train_step);
  3. the trained network drives the learned splitter policy
     (bisim_set_splitter_policy); the result is the same partition, only the
     splitter order and hence the iteration count change.

Training LTSs: n = 1000, m = 5000, uniform sources and targets, in two
regimes: one action with the initial partition from a Bernoulli(0.5)
proposition, and 64 actions with Zipf(1.1) labels and pi_0 = {S}.
"""
from __future__ import annotations

from typing import Iterable, List, Tuple

import numpy as np

from . import bisim, gen


def training_lts(regime: str, seed: int) -> gen.LTS:
    if regime == "kripke":
        return gen.kripke_uniform(1000, 5000, seed=seed)
    if regime == "zipf64":
        return gen.uniform_zipf(1000, 5000, 64, seed=seed)
    raise ValueError(regime)


def _upload(L):
    t = lambda a: bisim.DeviceArray.from_numpy(a, np.int32)
    return t(L.src), t(L.lab), t(L.dst), (None if L.init is None else t(L.init))


def collect(ltss: Iterable[gen.LTS], sample_every: int = 4, max_cands: int = 32,
            cap_per_lts: int = 4000) -> Tuple[np.ndarray, np.ndarray]:
    feats: List[np.ndarray] = []
    tgts: List[np.ndarray] = []
    for L in ltss:
        src, lab, dst, init = _upload(L)
        with bisim.LTS(src, lab, dst, L.n, L.K, init) as h:
            f, t, _ = bisim.collect_training(h, sample_every, max_cands, cap_per_lts)
        feats.append(f)
        tgts.append(t)
    return np.concatenate(feats), np.concatenate(tgts)


def train(mlp: bisim.MLP, X: np.ndarray, T: np.ndarray, steps: int = 400,
          lr: float = 3e-3) -> List[float]:
    xd = bisim.DeviceArray.from_numpy(np.ascontiguousarray(X, np.float32))
    td = bisim.DeviceArray.from_numpy(np.ascontiguousarray(T, np.float32))
    return [mlp.train_step(xd, td, lr) for _ in range(steps)]


def iterations(L: gen.LTS, mlp=None, rescore_every: int = 64, engine: int = 1):
    """(#It, block ids) of one run, plain (mlp None) or learned."""
    src, lab, dst, init = _upload(L)
    with bisim.LTS(src, lab, dst, L.n, L.K, init) as h:
        h.set_option(bisim.OPT_ENGINE, engine)
        if mlp is not None:
            bisim.set_splitter_policy(h, bisim.POLICY_LEARNED, mlp, rescore_every)
        blk, st = h.run()
        return st.iterations, blk.numpy(), st.t_alg_ms


def train_policy(train_seeds=range(1001, 1025), steps: int = 400, lr: float = 3e-3,
                 init_seed: int = 7, sample_every: int = 4, max_cands: int = 32):
    """Collect from both regimes, train a fresh network; returns (mlp, losses, rows)."""
    ltss = [training_lts(r, s) for r in ("kripke", "zipf64") for s in train_seeds]
    X, T = collect(ltss, sample_every, max_cands)
    mlp = bisim.MLP(bisim.POLICY_FEATURES, seed=init_seed)
    losses = train(mlp, X, T, steps, lr)
    return mlp, losses, X.shape[0]
