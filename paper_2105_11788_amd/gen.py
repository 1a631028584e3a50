"""Seeded synthetic labelled transition systems (LTSs).

This module only draws inputs: it contains none of the refinement method's
arithmetic, and both the HIP path and the CPU oracle consume what it returns.
Every generator is a pure function of its arguments and a seed (numpy PCG64).

An LTS here is (S, Act, ->) as in the paper's Definition 1, with
S = {0..n-1}, Act = {0..K-1}, and the transition relation given as three
int32 arrays src, lab, dst of length m (order arbitrary, duplicates allowed).
An optional init int32[n] encodes the initial partition pi_0 of the relational
coarsest partition problem (section 2): states with equal init value share a
block.  init=None means pi_0 = {S}.

The paper measures on the VLTS suite, which is not available here; the
families below are synthetic stand-ins with the shapes the workloads name
(uniform Kripke structures, planted-quotient LTSs with Zipf labels, deep
chains, synchronised products, a batch of uneven instances) plus the paper's
own Fan_out_n family (section 5, Figure 3) and its two worked examples
(Figures 1 and 2).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class LTS:
    n: int
    K: int
    src: np.ndarray
    lab: np.ndarray
    dst: np.ndarray
    init: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.src.shape[0])

    def __post_init__(self):
        self.src = np.ascontiguousarray(self.src, dtype=np.int32)
        self.lab = np.ascontiguousarray(self.lab, dtype=np.int32)
        self.dst = np.ascontiguousarray(self.dst, dtype=np.int32)
        if self.init is not None:
            self.init = np.ascontiguousarray(self.init, dtype=np.int32)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.uint64(seed)))


def zipf_labels(rng: np.random.Generator, size: int, K: int, s: float = 1.1) -> np.ndarray:
    """Labels 0..K-1 with P(label = r-1) proportional to r**-s (truncated Zipf)."""
    if K == 1:
        return np.zeros(size, dtype=np.int32)
    p = np.arange(1, K + 1, dtype=np.float64) ** (-s)
    p /= p.sum()
    return rng.choice(K, size=size, p=p).astype(np.int32)


# ---------------------------------------------------------------------------
# Kripke structure with uniform random transitions (one action label)
# ---------------------------------------------------------------------------
def kripke_uniform(n: int = 1000, m: int = 5000, seed: int = 1) -> LTS:
    """src, dst iid uniform over states, |Act| = 1, pi_0 from one Bernoulli(0.5)
    atomic proposition: init[s] = smallest state with the same proposition value
    (so init labels already lie in S, as the paper's block labels must)."""
    rng = _rng(seed)
    src = rng.integers(0, n, size=m, dtype=np.int64).astype(np.int32)
    dst = rng.integers(0, n, size=m, dtype=np.int64).astype(np.int32)
    ap = rng.integers(0, 2, size=n)
    init = np.empty(n, dtype=np.int32)
    for v in (0, 1):
        idx = np.nonzero(ap == v)[0]
        if idx.size:
            init[idx] = idx[0]
    return LTS(n, 1, src, np.zeros(m, np.int32), dst, init,
               name=f"kripke_uniform(n={n},m={m},seed={seed})")


# ---------------------------------------------------------------------------
# Planted quotient: a random quotient graph Q expanded into bisimilar copies
# ---------------------------------------------------------------------------
def random_quotient(q: int, deg_mean: float, K: int, rng: np.random.Generator,
                    zipf_s: float = 1.1) -> LTS:
    """Quotient graph Q: q nodes, Poisson(deg_mean) out-degree, Zipf labels,
    uniform targets, duplicate (B, a, B') edges removed."""
    deg = rng.poisson(deg_mean, size=q)
    src = np.repeat(np.arange(q, dtype=np.int64), deg)
    mq = src.size
    lab = zipf_labels(rng, mq, K, zipf_s).astype(np.int64)
    dst = rng.integers(0, q, size=mq, dtype=np.int64)
    key = (src * K + lab) * q + dst
    key = np.unique(key)
    dst = key % q
    lab = (key // q) % K
    src = key // (q * K)
    return LTS(q, K, src, lab, dst, None, name=f"quotient(q={q})")


def expand_quotient(Q: LTS, rng: np.random.Generator, copies_lo: int = 1,
                    copies_hi: int = 40):
    """Expand every quotient node B into c_B ~ U{lo..hi} copy states.  For each
    copy u of B and each Q-edge (B, a, B') add u -a-> v with v a uniformly drawn
    copy of B'.  The map copy -> B is then a functional bisimulation, so the
    coarsest partition of the expansion is the lift of Q's.  State ids are a
    seeded permutation, and transitions are shuffled."""
    q = Q.n
    c = rng.integers(copies_lo, copies_hi + 1, size=q, dtype=np.int64)
    cstart = np.zeros(q + 1, dtype=np.int64)
    np.cumsum(c, out=cstart[1:])
    n = int(cstart[-1])
    perm = rng.permutation(n).astype(np.int64)        # position -> state id
    owner = np.repeat(np.arange(q, dtype=np.int64), c)  # position -> quotient node
    # per Q edge: one transition per copy of its source node
    qsrc = Q.src.astype(np.int64)
    qdst = Q.dst.astype(np.int64)
    qlab = Q.lab.astype(np.int64)
    reps = c[qsrc]
    e_idx = np.repeat(np.arange(qsrc.size, dtype=np.int64), reps)
    # copy index within the source node for each emitted transition
    first = np.zeros(qsrc.size + 1, dtype=np.int64)
    np.cumsum(reps, out=first[1:])
    within = np.arange(e_idx.size, dtype=np.int64) - first[e_idx]
    u_pos = cstart[qsrc[e_idx]] + within
    tgt_node = qdst[e_idx]
    v_pos = cstart[tgt_node] + (rng.random(e_idx.size) * c[tgt_node]).astype(np.int64)
    src = perm[u_pos]
    dst = perm[v_pos]
    lab = qlab[e_idx]
    order = rng.permutation(src.size)
    state_to_q = np.empty(n, dtype=np.int64)
    state_to_q[perm] = owner
    return (LTS(n, Q.K, src[order], lab[order], dst[order], None),
            state_to_q.astype(np.int32))


def planted_quotient(q: int = 50_000, deg_mean: float = 8.0, K: int = 16,
                     seed: int = 1, zipf_s: float = 1.1, copies_hi: int = 40) -> LTS:
    """Labelled LTS with a planted quotient (meta['Q'], meta['state_to_q'])."""
    rng = _rng(seed)
    Q = random_quotient(q, deg_mean, K, rng, zipf_s)
    lts, s2q = expand_quotient(Q, rng, 1, copies_hi)
    lts.name = f"planted_quotient(q={q},deg={deg_mean},K={K},seed={seed})"
    lts.meta = {"Q": Q, "state_to_q": s2q}
    return lts


# ---------------------------------------------------------------------------
# Worst-case depth structures
# ---------------------------------------------------------------------------
def chain_tail(n: int = 100_000, permute_seed: Optional[int] = None) -> LTS:
    """s_i -0-> s_{i+1} for 0 <= i <= n-3 and s_{n-2} -1-> s_{n-1}: every state
    is alone in its bisimulation class, and refinement peels the chain one
    state per iteration.  With permute_seed the state ids are permuted."""
    assert n >= 2
    src = np.arange(n - 1, dtype=np.int64)
    dst = src + 1
    lab = np.zeros(n - 1, dtype=np.int64)
    lab[-1] = 1
    name = f"chain_tail(n={n})"
    if permute_seed is not None:
        p = _rng(permute_seed).permutation(n)
        src, dst = p[src], p[dst]
        name += f"[perm {permute_seed}]"
    return LTS(n, 2, src, lab, dst, None, name=name)


def chain_distinct(n: int = 25_217) -> LTS:
    """s_i -i-> s_{i+1} for 0 <= i <= n-2: a chain whose every transition has
    an action of its own (K = n - 1), the shape of the Table 1 row with as
    many actions as transitions.  Every state's outgoing action set is its
    own, so the preprocessing alone separates all states."""
    assert n >= 2
    src = np.arange(n - 1, dtype=np.int64)
    return LTS(n, n - 1, src, src.copy(), src + 1, None, name=f"chain_distinct(n={n})")


def sync_product(procs: int = 4, length: int = 30, K: int = 8,
                 shared=(6, 7), p_shared: float = 1.0 / 30.0, seed: int = 1) -> LTS:
    """Synchronised product of `procs` cyclic processes j -> j+1 mod `length`.
    Position j of process p carries label lambda_p(j): a shared label (drawn
    from `shared`) with probability p_shared, else a local label drawn from
    the remaining ones.  A local label moves its process alone; a shared label
    a fires one joint step, iff every process currently offers a.  All
    length**procs tuples are states (state = sum_p j_p * length**p)."""
    rng = _rng(seed)
    local = np.array([a for a in range(K) if a not in shared], dtype=np.int64)
    shared = np.array(shared, dtype=np.int64)
    lam = np.empty((procs, length), dtype=np.int64)
    for p in range(procs):
        is_sh = rng.random(length) < p_shared
        lam[p] = np.where(is_sh, shared[rng.integers(0, shared.size, length)],
                          local[rng.integers(0, local.size, length)])
    n = length ** procs
    states = np.arange(n, dtype=np.int64)
    digits = [(states // length ** p) % length for p in range(procs)]
    srcs, labs, dsts = [], [], []
    for p in range(procs):
        lp = lam[p][digits[p]]
        ok = np.isin(lp, local)
        nxt = states + np.where(digits[p] == length - 1, -(length - 1), 1) * length ** p
        srcs.append(states[ok]); labs.append(lp[ok]); dsts.append(nxt[ok])
    # joint steps
    l0 = lam[0][digits[0]]
    joint = np.isin(l0, shared)
    for p in range(1, procs):
        joint &= lam[p][digits[p]] == l0
    s = states[joint]
    t = np.zeros_like(s)
    for p in range(procs):
        d = (s // length ** p) % length
        t += ((d + 1) % length) * length ** p
    srcs.append(s); labs.append(l0[joint]); dsts.append(t)
    src = np.concatenate(srcs); lab = np.concatenate(labs); dst = np.concatenate(dsts)
    order = rng.permutation(src.size)
    return LTS(n, K, src[order], lab[order], dst[order], None,
               name=f"sync_product(procs={procs},len={length},K={K},seed={seed})",
               meta={"lam": lam})


# ---------------------------------------------------------------------------
# The paper's own examples
# ---------------------------------------------------------------------------
def fan_out(n: int) -> LTS:
    """Fan_out_n (section 5, Figure 3): i -a-> i+1 for 1 < i < n-1, and
    0 -b-> i, 1 -b-> i for every state i.  Labels: a = 0, b = 1."""
    assert n >= 2
    a_src = np.arange(2, n - 1, dtype=np.int64)
    a_dst = a_src + 1
    allst = np.arange(n, dtype=np.int64)
    src = np.concatenate([a_src, np.zeros(n, np.int64), np.ones(n, np.int64)])
    dst = np.concatenate([a_dst, allst, allst])
    lab = np.concatenate([np.zeros(a_src.size, np.int64), np.ones(2 * n, np.int64)])
    return LTS(n, 2, src, lab, dst, None, name=f"fan_out({n})")


def figure1() -> LTS:
    """Figure 1's Kripke structure with 0-based ids (s1..s5 -> 0..4):
    s1->s4, s2->s5, s2->s3, s3->s2; pi_0 = {{s1,s2,s3},{s4,s5}}."""
    src = [0, 1, 1, 2]
    dst = [3, 4, 2, 1]
    return LTS(5, 1, src, [0, 0, 0, 0], dst, np.array([0, 0, 0, 3, 3]), name="figure1")


def figure2() -> LTS:
    """Figure 2's LTS (labels a=0, b=1, c=2): s0-a->s1, s1-a->s0, s1-b->s2,
    s0-a->s2, s0-c->s2, s1-c->s1, s2-c->s0, s2-c->s2, listed unsorted."""
    t = [(2, 2, 0), (0, 0, 1), (1, 1, 2), (1, 0, 0), (0, 2, 2), (2, 2, 2),
         (1, 2, 1), (0, 0, 2)]
    src, lab, dst = zip(*t)
    return LTS(3, 3, src, lab, dst, None, name="figure2")


# ---------------------------------------------------------------------------
# Random small/medium LTSs for parity sweeps
# ---------------------------------------------------------------------------
def random_lts(n: int, m: int, K: int, seed: int, init_blocks: int = 0) -> LTS:
    """Uniform src/dst/label; optional random init partition with
    `init_blocks` classes (init values are arbitrary state indices)."""
    rng = _rng(seed)
    src = rng.integers(0, max(n, 1), size=m, dtype=np.int64)
    dst = rng.integers(0, max(n, 1), size=m, dtype=np.int64)
    lab = rng.integers(0, K, size=m, dtype=np.int64)
    init = None
    if init_blocks and n:
        cls = rng.integers(0, init_blocks, size=n)
        reps = rng.integers(0, n, size=init_blocks)
        init = reps[cls]
    return LTS(n, K, src, lab, dst, init, name=f"random(n={n},m={m},K={K},seed={seed})")


def uniform_zipf(n: int = 1000, m: int = 5000, K: int = 64, seed: int = 1) -> LTS:
    """Uniform src/dst, Zipf(1.1) labels over K actions, pi_0 = {S}."""
    rng = _rng(seed)
    src = rng.integers(0, n, size=m, dtype=np.int64)
    dst = rng.integers(0, n, size=m, dtype=np.int64)
    lab = zipf_labels(rng, m, K)
    return LTS(n, K, src, lab, dst, None, name=f"uniform_zipf(n={n},m={m},K={K},seed={seed})")


def uniform_lts(n: int, deg_mean: float, K: int, seed: int) -> LTS:
    """Poisson(deg_mean) out-degree per state, uniform targets and labels."""
    rng = _rng(seed)
    deg = rng.poisson(deg_mean, size=n)
    src = np.repeat(np.arange(n, dtype=np.int64), deg)
    dst = rng.integers(0, n, size=src.size, dtype=np.int64)
    lab = rng.integers(0, K, size=src.size, dtype=np.int64)
    order = rng.permutation(src.size)
    return LTS(n, K, src[order], lab[order], dst[order], None,
               name=f"uniform(n={n},deg={deg_mean},K={K},seed={seed})")


# ---------------------------------------------------------------------------
# Batch of uneven instances
# ---------------------------------------------------------------------------
def _batch_plan(count: int, n_lo: int, n_hi: int, K_hi: int, seed: int):
    """Sizes, action counts and per-instance seeds of a batch (the master
    generator's first three draws)."""
    rng = _rng(seed)
    sizes = np.floor(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=count))).astype(np.int64)
    Ks = rng.integers(1, K_hi + 1, size=count)
    seeds = rng.integers(0, 2**62, size=count)
    return sizes, Ks, seeds


def _batch_member(k: int, nk: int, Kk: int, sk: int, deg_mean: float) -> LTS:
    sub = _rng(sk)
    if k % 2 == 0:
        q = max(1, int(np.ceil(nk / 20.5)))
        Q = random_quotient(q, deg_mean, Kk, sub)
        lts, s2q = expand_quotient(Q, sub)
        lts.meta = {"Q": Q, "state_to_q": s2q}
    else:
        lts = uniform_lts(nk, deg_mean, Kk, sk ^ 0x5bd1e995)
    lts.name = f"batch[{k}]"
    return lts


def batch(count: int = 4096, n_lo: int = 100, n_hi: int = 200_000,
          deg_mean: float = 6.0, K_hi: int = 32, seed: int = 1) -> List[LTS]:
    """`count` independent LTSs with log-uniform sizes in [n_lo, n_hi],
    Poisson(deg_mean) out-degree and K ~ U{1..K_hi}.  Even-indexed instances
    have planted quotients (ceil(n/20.5) quotient nodes, copies U{1..40},
    Zipf(1.1) labels); odd-indexed ones are uniform."""
    sizes, Ks, seeds = _batch_plan(count, n_lo, n_hi, K_hi, seed)
    return [_batch_member(k, int(sizes[k]), int(Ks[k]), int(seeds[k]), deg_mean)
            for k in range(count)]


def batch_instance(k: int, count: int = 4096, n_lo: int = 100, n_hi: int = 200_000,
                   deg_mean: float = 6.0, K_hi: int = 32, seed: int = 1) -> LTS:
    """Instance k of batch(count, n_lo, n_hi, deg_mean, K_hi, seed), drawn
    alone (identical to the list's element k)."""
    sizes, Ks, seeds = _batch_plan(count, n_lo, n_hi, K_hi, seed)
    return _batch_member(k, int(sizes[k]), int(Ks[k]), int(seeds[k]), deg_mean)
