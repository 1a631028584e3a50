"""CPU oracle for strong-bisimulation partition refinement.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product library.  It shares no code
with the HIP implementation and imports nothing from it.

Contents
  ks_coarsest      Kanellakis-Smolka splitter refinement (section 3.1,
                   Algorithm 1, generalised to labels); C, timed baseline.
  preprocess       section 4.1 preprocessing arrays and pi_pre; C.
  alg3_trace       lock-step simulation of Algorithm 3 (or Algorithm 2);
                   C.  Iteration count, splitter sequence, per-iteration
                   partitions.
  check_stable / check_refines / check_canonical      C checkers.
  bruteforce_gfp   greatest-fixpoint bisimulation over state pairs
                   (Definition 2), pure Python, tiny inputs.
  enumerate_coarsest   exhaustive search over all partitions refining pi_0
                   for the one with fewest blocks that is a bisimulation
                   (the problem statement of section 2), tiny inputs.
  signature_rounds multi-way signature refinement from pi_pre (the
                   signature-based approach the paper compares against in
                   section 5), pure Python: rounds to the fixpoint.
  hybrid_trace     signature rounds while each splits many blocks, then
                   Algorithm 3 from the partition reached (the combination of
                   multi-way splitting with the linear bound that section 6
                   leaves as future work).
  mlp_*            fp64 reference of the splitter-scoring network (separate
                   module, oracle.mlp).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-Wno-unused-result", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_native = None


def native_ks():
    """ks_coarsest from the same source compiled with -O3 -march=native for
    the host that runs it (the timed CPU baseline), built once per process in
    a temporary directory.  Returns a callable with ks_coarsest's signature."""
    global _native
    if _native is None:
        import tempfile
        d = tempfile.mkdtemp(prefix="oracle_native_")
        so = os.path.join(d, "liboracle_native.so")
        subprocess.check_call(["gcc", "-O3", "-march=native", "-std=c11", "-fPIC", "-shared",
                               "-Wall", "-Wno-unused-result", _SRC, "-o", so])
        L = ctypes.CDLL(so)
        P = ctypes.c_void_p
        L.orc_ks_coarsest.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, P, P, P, P, P]
        L.orc_ks_coarsest.restype = ctypes.c_int64
        _native = L

    def run(n, K, src, lab, dst, init=None):
        src, lab, dst, init = _i32(src), _i32(lab), _i32(dst), _i32(init)
        out = np.empty(max(n, 0), dtype=np.int32)
        r = _native.orc_ks_coarsest(n, src.size, K, _p(src), _p(lab), _p(dst), _p(init), _p(out))
        if r < 0:
            raise OracleError(f"orc_ks_coarsest: {r}")
        return out, int(r)
    return run


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        L.orc_ks_coarsest.argtypes = [i32, i64, i32, P, P, P, P, P]
        L.orc_ks_coarsest.restype = i64
        L.orc_preprocess.argtypes = [i32, i64, i32, P, P, P, P, P, P, P, P, P, P, P, P, P]
        L.orc_preprocess.restype = i64
        L.orc_alg3.argtypes = [i32, i64, i32, P, P, P, P, P, P, i64, P, P, P, i32, i64, i32]
        L.orc_alg3.restype = i64
        L.orc_check_stable.argtypes = [i32, i64, P, P, P, P]
        L.orc_check_stable.restype = ctypes.c_int
        L.orc_check_refines.argtypes = [i32, P, P]
        L.orc_check_refines.restype = ctypes.c_int
        L.orc_check_canonical.argtypes = [i32, P]
        L.orc_check_canonical.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.int32)


class OracleError(RuntimeError):
    pass


def ks_coarsest(n, K, src, lab, dst, init=None):
    """Canonical coarsest partition (block id = smallest member) and its
    block count, by Kanellakis-Smolka refinement."""
    src, lab, dst, init = _i32(src), _i32(lab), _i32(dst), _i32(init)
    out = np.empty(max(n, 0), dtype=np.int32)
    r = lib().orc_ks_coarsest(n, src.size, K, _p(src), _p(lab), _p(dst), _p(init), _p(out))
    if r < 0:
        raise OracleError(f"orc_ks_coarsest: {r}")
    return out, int(r)


def preprocess(n, K, src, lab, dst, init=None):
    """Section 4.1 arrays: dict with s_src, s_lab, s_dst, action_switch, order,
    nr_marks, off, mark_length, pre_block, pre_blocks."""
    src, lab, dst, init = _i32(src), _i32(lab), _i32(dst), _i32(init)
    m = src.size
    o = {k: np.empty(m, np.int32) for k in ("s_src", "s_lab", "s_dst", "action_switch", "order")}
    o["nr_marks"] = np.empty(n, np.int32)
    o["off"] = np.empty(n, np.int64)
    ml = np.zeros(1, np.int64)
    o["pre_block"] = np.empty(n, np.int32)
    r = lib().orc_preprocess(n, m, K, _p(src), _p(lab), _p(dst), _p(init), _p(o["s_src"]),
                             _p(o["s_lab"]), _p(o["s_dst"]), _p(o["action_switch"]),
                             _p(o["order"]), _p(o["nr_marks"]), _p(o["off"]), _p(ml),
                             _p(o["pre_block"]))
    if r < 0:
        raise OracleError(f"orc_preprocess: {r}")
    o["mark_length"] = int(ml[0])
    o["pre_blocks"] = int(r)
    return o


def alg3_trace(n, K, src, lab, dst, init=None, trace_cap=0, keep_blocks=False,
               force_first_C=-1, max_iters=0, variant=3):
    """Lock-step Algorithm 3 (variant=3) or Algorithm 2 (variant=2).
    Returns dict: block, iters, pre_blocks, C (splitter per iteration, -1 for
    the final pass), nsplit, blocks (iteration x n, if keep_blocks)."""
    src, lab, dst, init = _i32(src), _i32(lab), _i32(dst), _i32(init)
    out = np.empty(n, np.int32)
    pre = np.zeros(1, np.int64)
    tC = np.empty(trace_cap, np.int32) if trace_cap else None
    tS = np.empty(trace_cap, np.int64) if trace_cap else None
    tB = np.empty((trace_cap, n), np.int32) if (trace_cap and keep_blocks) else None
    r = lib().orc_alg3(n, src.size, K, _p(src), _p(lab), _p(dst), _p(init), _p(out), _p(pre),
                       trace_cap, _p(tC), _p(tS), _p(tB), force_first_C, max_iters, variant)
    truncated = (r == -4)
    if truncated:
        r = max_iters
    elif r < 0:
        raise OracleError(f"orc_alg3: {r}")
    res = {"block": out, "iters": int(r), "pre_blocks": int(pre[0]), "truncated": truncated}
    if trace_cap:
        k = min(int(r), trace_cap)
        res["C"] = tC[:k].copy()
        res["nsplit"] = tS[:k].copy()
        if keep_blocks:
            res["blocks"] = tB[:k].copy()
    return res


def check_stable(n, src, lab, dst, block) -> bool:
    src, lab, dst, block = _i32(src), _i32(lab), _i32(dst), _i32(block)
    r = lib().orc_check_stable(n, src.size, _p(src), _p(lab), _p(dst), _p(block))
    if r < 0:
        raise OracleError(f"orc_check_stable: {r}")
    return bool(r)


def check_refines(n, block, init) -> bool:
    block, init = _i32(block), _i32(init)
    r = lib().orc_check_refines(n, _p(block), _p(init))
    if r < 0:
        raise OracleError(f"orc_check_refines: {r}")
    return bool(r)


def check_canonical(n, block) -> bool:
    block = _i32(block)
    return bool(lib().orc_check_canonical(n, _p(block)))


# ---------------------------------------------------------------------------
# Definition-level references for tiny inputs (pure Python)
# ---------------------------------------------------------------------------
def _succ(n, src, lab, dst):
    succ = [dict() for _ in range(n)]
    for s, a, t in zip(np.asarray(src).tolist(), np.asarray(lab).tolist(), np.asarray(dst).tolist()):
        succ[s].setdefault(a, set()).add(t)
    return succ


def canonical_from_classes(n, cls):
    """Relabel a class assignment so that each id is the smallest member."""
    first = {}
    out = np.empty(n, np.int32)
    for s in range(n):
        c = cls[s]
        if c not in first:
            first[c] = s
        out[s] = first[c]
    return out


def bruteforce_gfp(n, src, lab, dst, init=None):
    """Greatest bisimulation contained in the equivalence of pi_0, as the
    greatest fixpoint of R -> {(s,t) in R : every s-a->s' is matched by some
    t-a->t' with (s',t') in R, and vice versa} (Definition 2).  O(n^2) pairs
    per round; meant for n <= ~12."""
    succ = _succ(n, src, lab, dst)
    iv = [0] * n if init is None else list(np.asarray(init).tolist())
    R = [[iv[s] == iv[t] for t in range(n)] for s in range(n)]

    def matched(s, t):
        for a, ss in succ[s].items():
            ts = succ[t].get(a)
            if not ts:
                return False
            for s2 in ss:
                if not any(R[s2][t2] for t2 in ts):
                    return False
        return True

    changed = True
    while changed:
        changed = False
        for s in range(n):
            for t in range(n):
                if R[s][t] and not (matched(s, t) and matched(t, s)):
                    R[s][t] = False
                    changed = True
    cls = [min(t for t in range(n) if R[s][t]) for s in range(n)]
    return canonical_from_classes(n, cls)


def _set_partitions(items):
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for p in _set_partitions(rest):
        for i in range(len(p)):
            yield p[:i] + [[first] + p[i]] + p[i + 1:]
        yield [[first]] + p


def is_bisimulation_partition(n, succ, cls):
    """Definition 2 for the relation induced by the class assignment `cls`."""
    for s in range(n):
        for t in range(n):
            if cls[s] != cls[t]:
                continue
            for a, ss in succ[s].items():
                ts = succ[t].get(a, ())
                for s2 in ss:
                    if not any(cls[t2] == cls[s2] for t2 in ts):
                        return False
    return True


def enumerate_coarsest(n, src, lab, dst, init=None):
    """Among all partitions refining pi_0 whose induced relation is a
    bisimulation, the one with the fewest blocks (the problem statement).
    Also asserts that it is unique and that every other bisimulation partition
    refines it.  Bell-number cost: n <= 8."""
    succ = _succ(n, src, lab, dst)
    iv = [0] * n if init is None else list(np.asarray(init).tolist())
    groups = {}
    for s in range(n):
        groups.setdefault(iv[s], []).append(s)
    glist = list(groups.values())

    def product(i):
        if i == len(glist):
            yield []
            return
        for p in _set_partitions(glist[i]):
            for rest in product(i + 1):
                yield p + rest

    best = None
    found = []
    for part in product(0):
        cls = [0] * n
        for bi, b in enumerate(part):
            for s in b:
                cls[s] = bi
        if is_bisimulation_partition(n, succ, cls):
            found.append(cls)
            if best is None or len(part) < best[0]:
                best = (len(part), cls)
    assert best is not None
    winners = [c for c in found if len(set(c)) == best[0]]
    canon = {tuple(canonical_from_classes(n, c)) for c in winners}
    assert len(canon) == 1, "coarsest bisimulation partition not unique"
    top = best[1]
    for c in found:  # every bisimulation partition refines the coarsest one
        for s in range(n):
            for t in range(n):
                if c[s] == c[t]:
                    assert top[s] == top[t]
    return canonical_from_classes(n, best[1])


def signature_rounds(n, K, src, lab, dst, init=None, keep_blocks=False, stall=0):
    """Multi-way signature refinement (the signature-based splitting of the
    comparison systems in section 5): starting from pi_pre (section 4.1),
    every round gives each state the signature {(a, block(t)) : s -a-> t},
    and states stay together iff they were together and their signatures are
    equal; every new block is named by its smallest state.  Stops after the
    first round that changes nothing, or, with stall > 0, after the second
    of two consecutive rounds that each add fewer than `stall` blocks.
    Returns dict: block (canonical), rounds (including that last
    round), fixpoint (whether the last round changed nothing), blocks
    (per-round partitions, if keep_blocks).  Pure Python: meant for m up to
    about 10^5."""
    pre = preprocess(n, K, src, lab, dst, init)["pre_block"]
    part = [int(x) for x in pre]
    out = {(int(a), int(b), int(c)) for a, b, c in zip(src, lab, dst)}
    succ = [[] for _ in range(n)]
    for s_, a, t in out:
        succ[s_].append((a, t))
    nblocks = len(set(part))
    rounds = 0
    hist = []
    prev_few = False
    while True:
        rounds += 1
        leader = {}
        new = [0] * n
        for s_ in range(n):
            key = (part[s_], frozenset((a, part[t]) for a, t in succ[s_]))
            new[s_] = leader.setdefault(key, s_)  # states are visited in increasing order
        part = new
        if keep_blocks:
            hist.append(np.array(part, np.int32))
        nb = len(leader)
        if nb == nblocks:
            fixpoint = True
            break
        few = nb - nblocks < stall
        if stall and few and prev_few:
            fixpoint = False
            break
        prev_few = few
        nblocks = nb
    res = {"block": np.array(part, np.int32), "rounds": rounds, "fixpoint": fixpoint}
    if keep_blocks:
        res["blocks"] = hist
    return res


def hybrid_trace(n, K, src, lab, dst, init=None, stall=64):
    """Multi-way signature rounds (signature_rounds with `stall`) followed,
    unless they reached the fixpoint, by Algorithm 3 started from the
    partition they reached with every block unstable.  That partition refines
    pi_pre and is coarser than the coarsest stable one, so Algorithm 3 ends in
    the same result; section 4.1's preprocessing leaves it unchanged.  Returns
    dict: block, rounds, alg3_iters, iters (= rounds + alg3_iters)."""
    r = signature_rounds(n, K, src, lab, dst, init, stall=stall)
    if r["fixpoint"]:
        return {"block": r["block"], "rounds": r["rounds"], "alg3_iters": 0,
                "iters": r["rounds"]}
    a = alg3_trace(n, K, src, lab, dst, r["block"])
    return {"block": a["block"], "rounds": r["rounds"], "alg3_iters": a["iters"],
            "iters": r["rounds"] + a["iters"]}
