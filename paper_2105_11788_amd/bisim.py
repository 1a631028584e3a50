"""Python binding of libbisim.so (include/bisim.h): argument marshalling only.

Every step of the computation runs in the HIP library; this module moves
arrays between host and device and turns status codes into exceptions.
There is no CPU fallback: if the library is not built or no GPU is present,
calls fail.

Device buffers are plain HIP allocations made through the same HIP runtime
that libbisim.so links (ROCm's libamdhip64.so.7), so the library never shares
a process with a second, differently versioned HIP runtime.  Any object with
an integer `ptr` attribute (a device address) can be passed where a
DeviceArray is expected.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbisim.so")

OK = 0
E_INVALID = -1
E_RANGE = -2
E_NOMEM = -3
E_DEVICE = -4
E_ITERCAP = -5
E_UNSUPPORTED = -6

OPT_ENGINE = 1
OPT_FIRST_SPLITTER = 2
OPT_ITER_LIMIT = 3
OPT_GRID = 4
OPT_PROFILE_EVERY = 5
OPT_ALGORITHM = 6  # 3: labelled (Algorithm 3, default); 2: one-action RCPP (Algorithm 2)
OPT_COUNT_WORK = 7  # engine 3: accumulate work totals (LTS.work())
ALGORITHM_RCPP, ALGORITHM_LABELLED, ALGORITHM_SIGNATURE, ALGORITHM_HYBRID = 2, 3, 100, 101  # OPT_ALGORITHM values

ENGINE_AUTO = 0
ENGINE_PERSISTENT = 1
ENGINE_PHASES = 2
ENGINE_LISTS = 3

EXPORTS = ["lts_load", "coarsest_partition", "lts_free", "bisim_last_error",
           "bisim_set_option", "bisim_set_trace", "bisim_get_preprocessed",
           "lts_batch_load", "coarsest_partition_batch", "lts_batch_free",
           "bisim_batch_set_option", "mlp_num_params", "mlp_create", "mlp_free",
           "mlp_get_params", "mlp_forward", "mlp_train_step", "bisim_set_splitter_policy",
           "bisim_collect_training", "bisim_get_phase_times", "bisim_device_copy",
           "coarsest_partition_noalloc", "bisim_get_work", "mlp_forward_bf16",
           "bisim_get_run_config", "bisim_get_preprocess_method"]

# size of the static device region of coarsest_partition_noalloc (bisim.h)
NOALLOC_SCRATCH_BYTES = 64 << 20


class BisimError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"bisim status {status}: {msg}")
        self.status = status


class bisim_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int64), ("blocks", ctypes.c_int64),
                ("pre_blocks", ctypes.c_int64), ("mark_length", ctypes.c_int64),
                ("t_pre_ms", ctypes.c_double), ("t_alg_ms", ctypes.c_double)]


_lib = None
_hip = None


def load_library(path: str = LIB_PATH):
    """Load libbisim.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2105_11788_amd.build` "
                          "(or __graft_entry__.build()) first")
    L = ctypes.CDLL(path)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.lts_load.argtypes = [P, P, P, i32, i64, i32, P, P, ctypes.POINTER(P)]
    L.lts_load.restype = i32
    L.coarsest_partition.argtypes = [P, P, ctypes.POINTER(bisim_stats)]
    L.coarsest_partition.restype = i32
    L.lts_free.argtypes = [P]
    L.lts_free.restype = None
    L.bisim_last_error.argtypes = []
    L.bisim_last_error.restype = ctypes.c_char_p
    L.bisim_set_option.argtypes = [P, i32, i64]
    L.bisim_set_option.restype = i32
    L.bisim_set_trace.argtypes = [P, P, P, P, i64]
    L.bisim_set_trace.restype = i32
    L.bisim_get_preprocessed.argtypes = [P, P, P]
    L.bisim_get_preprocessed.restype = i32
    L.coarsest_partition_noalloc.argtypes = [P, P, P, i32, i64, i32, P, P,
                                             ctypes.POINTER(bisim_stats), P]
    L.coarsest_partition_noalloc.restype = i32
    _lib = L
    return L


def hip():
    """The HIP runtime libbisim.so is linked against (already loaded by it)."""
    global _hip
    if _hip is None:
        load_library()
        H = ctypes.CDLL("libamdhip64.so.7")
        P, sz = ctypes.c_void_p, ctypes.c_size_t
        H.hipMalloc.argtypes = [ctypes.POINTER(P), sz]
        H.hipFree.argtypes = [P]
        H.hipMemcpy.argtypes = [P, P, sz, ctypes.c_int]
        H.hipMemset.argtypes = [P, ctypes.c_int, sz]
        H.hipGetDeviceCount.argtypes = [ctypes.POINTER(ctypes.c_int)]
        H.hipDeviceSynchronize.argtypes = []
        H.hipGetErrorString.argtypes = [ctypes.c_int]
        H.hipGetErrorString.restype = ctypes.c_char_p
        for f in ("hipMalloc", "hipFree", "hipMemcpy", "hipMemset", "hipGetDeviceCount",
                  "hipDeviceSynchronize"):
            getattr(H, f).restype = ctypes.c_int
        _hip = H
    return _hip


def _hip_check(rc: int, what: str):
    if rc != 0:
        raise BisimError(E_DEVICE, f"{what}: {hip().hipGetErrorString(rc).decode()}")


def device_count() -> int:
    c = ctypes.c_int(0)
    rc = hip().hipGetDeviceCount(ctypes.byref(c))
    return c.value if rc == 0 else 0


def synchronize():
    _hip_check(hip().hipDeviceSynchronize(), "hipDeviceSynchronize")


_H2D, _D2H, _D2D = 1, 2, 3


class DeviceArray:
    """A 1-D device buffer of a numpy dtype."""

    def __init__(self, count: int, dtype=np.int32):
        self.dtype = np.dtype(dtype)
        self.count = int(count)
        self.nbytes = self.count * self.dtype.itemsize
        p = ctypes.c_void_p()
        _hip_check(hip().hipMalloc(ctypes.byref(p), max(self.nbytes, 1)), "hipMalloc")
        self.ptr = p.value

    @classmethod
    def from_numpy(cls, a: np.ndarray, dtype=None) -> "DeviceArray":
        a = np.ascontiguousarray(a, dtype=dtype if dtype is not None else a.dtype)
        d = cls(a.size, a.dtype)
        if d.nbytes:
            _hip_check(hip().hipMemcpy(ctypes.c_void_p(d.ptr), a.ctypes.data_as(ctypes.c_void_p),
                                       d.nbytes, _H2D), "hipMemcpy H2D")
        return d

    def numpy(self) -> np.ndarray:
        out = np.empty(self.count, self.dtype)
        if self.nbytes:
            _hip_check(hip().hipMemcpy(out.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(self.ptr),
                                       self.nbytes, _D2H), "hipMemcpy D2H")
        return out

    def fill(self, byte: int):
        _hip_check(hip().hipMemset(ctypes.c_void_p(self.ptr), byte, self.nbytes), "hipMemset")
        return self

    def free(self):
        if getattr(self, "ptr", None):
            hip().hipFree(ctypes.c_void_p(self.ptr))
            self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _check(status: int):
    if status != OK:
        raise BisimError(status, _lib.bisim_last_error().decode(errors="replace"))


def _dptr(a, name, count=None):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        raise TypeError(f"{name}: pass a DeviceArray (device memory), not a host array")
    p = getattr(a, "ptr", None)
    if not isinstance(p, int):
        raise TypeError(f"{name} must be a DeviceArray or expose an integer device `ptr`")
    if count is not None and getattr(a, "count", count) != count:
        raise ValueError(f"{name} must have {count} entries")
    return ctypes.c_void_p(p)


@dataclass
class Stats:
    iterations: int
    blocks: int
    pre_blocks: int
    mark_length: int
    t_pre_ms: float
    t_alg_ms: float


class LTS:
    """A loaded LTS (lts_load).  src/lab/dst (m entries) and init (n entries
    or None) are int32 DeviceArrays; numpy arrays are uploaded first."""

    def __init__(self, src, lab, dst, n: int, num_actions: int, init=None,
                 stream: Optional[int] = None):
        L = load_library()
        self._L = L
        self.n = int(n)
        self.K = int(num_actions)
        up = lambda a: DeviceArray.from_numpy(a, np.int32) if isinstance(a, np.ndarray) else a
        src, lab, dst, init = up(src), up(lab), up(dst), (None if init is None else up(init))
        self.m = int(getattr(src, "count"))
        ps, pl, pd = (_dptr(x, nm, self.m) if self.m else None
                      for x, nm in ((src, "src"), (lab, "label"), (dst, "dst")))
        pi = _dptr(init, "init_partition", self.n) if (init is not None and self.n) else None
        self.stream = stream
        h = ctypes.c_void_p()
        _check(L.lts_load(ps, pl, pd, self.n, self.m, self.K, pi,
                          ctypes.c_void_p(stream) if stream else None, ctypes.byref(h)))
        self._h = h
        self._trace = None

    def set_option(self, option: int, value: int):
        _check(self._L.bisim_set_option(self._h, option, int(value)))

    def set_trace(self, cap: int, work: bool = False):
        """Record splitter and split count (and, with work=True, the per-iteration
        work counters) of the first `cap` iterations of later runs; returns
        DeviceArrays (trace_C, trace_nsplit[, trace_work of cap*4])."""
        if cap <= 0:
            _check(self._L.bisim_set_trace(self._h, None, None, None, 0))
            self._trace = None
            return None
        tc = DeviceArray(cap, np.int32).fill(0xFF)
        ts = DeviceArray(cap, np.int64).fill(0xFF)
        tw = DeviceArray(cap * 4, np.int64).fill(0) if work else None
        _check(self._L.bisim_set_trace(self._h, ctypes.c_void_p(tc.ptr), ctypes.c_void_p(ts.ptr),
                                       ctypes.c_void_p(tw.ptr) if work else None, cap))
        self._trace = (tc, ts, tw) if work else (tc, ts)
        return self._trace

    def run(self, out: Optional[DeviceArray] = None):
        """coarsest_partition: returns (block_id DeviceArray, Stats)."""
        if out is None:
            out = DeviceArray(self.n, np.int32)
        st = bisim_stats()
        po = _dptr(out, "block_id", self.n) if self.n else None
        _check(self._L.coarsest_partition(self._h, po, ctypes.byref(st)))
        return out, Stats(st.iterations, st.blocks, st.pre_blocks, st.mark_length,
                          st.t_pre_ms, st.t_alg_ms)

    def phase_times(self):
        """(avg kernel ms per phase [select+mark, compare+elect, relabel, re-score],
        samples per phase) of the last run with OPT_PROFILE_EVERY set."""
        L = self._L
        if not getattr(L, "_phase_declared", False):
            L.bisim_get_phase_times.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
            L.bisim_get_phase_times.restype = ctypes.c_int32
            L._phase_declared = True
        ms = np.zeros(4, np.float64)
        cnt = np.zeros(4, np.int64)
        _check(L.bisim_get_phase_times(self._h, ms.ctypes.data_as(ctypes.c_void_p),
                                       cnt.ctypes.data_as(ctypes.c_void_p)))
        return ms, cnt

    def run_config(self):
        """(engine, grid) of the last run: what ENGINE_AUTO resolved to."""
        L = self._L
        e, g = ctypes.c_int32(0), ctypes.c_int32(0)
        L.bisim_get_run_config.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.bisim_get_run_config.restype = ctypes.c_int32
        _check(L.bisim_get_run_config(self._h, ctypes.byref(e), ctypes.byref(g)))
        return e.value, g.value

    def preprocess_method(self):
        """0: pi_pre from Algorithm 4's action rounds; 1: from the one-pass
        kernels (checked exactly, the rounds run if the check fails)."""
        L = self._L
        v = ctypes.c_int32(0)
        L.bisim_get_preprocess_method.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.bisim_get_preprocess_method.restype = ctypes.c_int32
        _check(L.bisim_get_preprocess_method(self._h, ctypes.byref(v)))
        return v.value

    def work(self):
        """Work totals of the last run with OPT_COUNT_WORK (engine 3): dict of
        members, in_transitions, touched, segments, member_visits, split_states,
        split_blocks, split_iterations."""
        L = self._L
        if not getattr(L, "_work_declared", False):
            L.bisim_get_work.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
            L.bisim_get_work.restype = ctypes.c_int32
            L._work_declared = True
        w = np.zeros(8, np.int64)
        _check(L.bisim_get_work(self._h, w.ctypes.data_as(ctypes.c_void_p)))
        keys = ("members", "in_transitions", "touched", "segments", "member_visits",
                "split_states", "split_blocks", "split_iterations")
        return dict(zip(keys, (int(x) for x in w)))

    def preprocessed(self):
        """(pi_pre block ids, nr_marks) as numpy arrays."""
        b = DeviceArray(self.n, np.int32)
        nm = DeviceArray(self.n, np.int32)
        if self.n:
            _check(self._L.bisim_get_preprocessed(self._h, ctypes.c_void_p(b.ptr),
                                                  ctypes.c_void_p(nm.ptr)))
        return b.numpy(), nm.numpy()

    def close(self):
        if getattr(self, "_h", None):
            self._L.lts_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class bisim_batch_stats(ctypes.Structure):
    _fields_ = [("max_iterations", ctypes.c_int64), ("sum_iterations", ctypes.c_int64),
                ("lds_instances", ctypes.c_int64), ("global_instances", ctypes.c_int64),
                ("workgroup_size", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("t_pre_ms", ctypes.c_double), ("t_alg_ms", ctypes.c_double),
                ("work", (ctypes.c_int64 * 8) * 2)]


BOPT_WG_SIZE = 1
BOPT_GRID = 2
BOPT_LDS_LIMIT = 3
BOPT_TUNE = 4


def _declare_batch(L):
    if getattr(L, "_batch_declared", False):
        return
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.lts_batch_load.argtypes = [i32, P, P, P, P, P, P, P, P, ctypes.POINTER(P)]
    L.lts_batch_load.restype = i32
    L.coarsest_partition_batch.argtypes = [P, P, P, ctypes.POINTER(bisim_batch_stats)]
    L.coarsest_partition_batch.restype = i32
    L.lts_batch_free.argtypes = [P]
    L.lts_batch_free.restype = None
    L.bisim_batch_set_option.argtypes = [P, i32, i64]
    L.bisim_batch_set_option.restype = i32
    L._batch_declared = True


class Batch:
    """Many LTSs refined in one launch (lts_batch_load / coarsest_partition_batch).
    `instances` is a sequence of objects with n, K, src, lab, dst, init
    (numpy, instance-local ids); they are concatenated and uploaded."""

    def __init__(self, instances, stream: Optional[int] = None):
        L = load_library()
        _declare_batch(L)
        self._L = L
        self.count = len(instances)
        n_off = np.zeros(self.count + 1, np.int64)
        m_off = np.zeros(self.count + 1, np.int64)
        for k, x in enumerate(instances):
            n_off[k + 1] = n_off[k] + int(x.n)
            m_off[k + 1] = m_off[k] + int(np.asarray(x.src).size)
        self.n_off, self.m_off = n_off, m_off
        self.N = int(n_off[-1])
        K = np.array([int(x.K) for x in instances], np.int32)
        cat = lambda f: np.concatenate([np.asarray(f(x), np.int32) for x in instances]) \
            if self.count else np.zeros(0, np.int32)
        src = DeviceArray.from_numpy(cat(lambda x: x.src), np.int32)
        lab = DeviceArray.from_numpy(cat(lambda x: x.lab), np.int32)
        dst = DeviceArray.from_numpy(cat(lambda x: x.dst), np.int32)
        has_init = any(x.init is not None for x in instances)
        init = None
        if has_init:
            init = DeviceArray.from_numpy(np.concatenate(
                [np.asarray(x.init if x.init is not None else np.zeros(x.n), np.int32)
                 for x in instances]), np.int32)
        h = ctypes.c_void_p()
        p = lambda a: ctypes.c_void_p(a.ptr) if (a is not None and a.count) else None
        _check(L.lts_batch_load(self.count, n_off.ctypes.data_as(ctypes.c_void_p),
                                m_off.ctypes.data_as(ctypes.c_void_p), p(src), p(lab), p(dst),
                                K.ctypes.data_as(ctypes.c_void_p), p(init),
                                ctypes.c_void_p(stream) if stream else None, ctypes.byref(h)))
        self._h = h

    def set_option(self, option: int, value: int):
        _check(self._L.bisim_batch_set_option(self._h, option, int(value)))

    def run(self, out: Optional[DeviceArray] = None):
        """Returns (block ids DeviceArray, per-instance #It int64 array, stats dict)."""
        if out is None:
            out = DeviceArray(self.N, np.int32)
        its = np.zeros(self.count, np.int64)
        st = bisim_batch_stats()
        _check(self._L.coarsest_partition_batch(self._h, ctypes.c_void_p(out.ptr),
                                                its.ctypes.data_as(ctypes.c_void_p),
                                                ctypes.byref(st)))
        d = {f: getattr(st, f) for f, _ in bisim_batch_stats._fields_ if f != "work"}
        d["work"] = [[int(x) for x in row] for row in st.work]
        return out, its, d

    def split(self, flat: np.ndarray):
        """Per-instance views of a concatenated result."""
        return [flat[self.n_off[k]:self.n_off[k + 1]] for k in range(self.count)]

    def close(self):
        if getattr(self, "_h", None):
            self._L.lts_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


POLICY_PLAIN = 0
POLICY_LEARNED = 1
POLICY_FEATURES = 19


def _declare_learned(L):
    if getattr(L, "_learned_declared", False):
        return
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.mlp_num_params.argtypes = [i32]
    L.mlp_num_params.restype = i64
    L.mlp_create.argtypes = [i32, P, ctypes.c_uint64, ctypes.POINTER(P)]
    L.mlp_create.restype = i32
    L.mlp_free.argtypes = [P]
    L.mlp_free.restype = None
    L.mlp_get_params.argtypes = [P, P]
    L.mlp_get_params.restype = i32
    L.mlp_forward.argtypes = [P, P, i64, P, P]
    L.mlp_forward.restype = i32
    L.mlp_forward_bf16.argtypes = [P, P, i64, P, P]
    L.mlp_forward_bf16.restype = i32
    L.mlp_train_step.argtypes = [P, P, P, i64, ctypes.c_float, ctypes.POINTER(ctypes.c_float), P, P]
    L.mlp_train_step.restype = i32
    L.bisim_set_splitter_policy.argtypes = [P, i32, P, i32]
    L.bisim_set_splitter_policy.restype = i32
    L.bisim_collect_training.argtypes = [P, i64, i32, P, P, P, i64, ctypes.POINTER(i64)]
    L.bisim_collect_training.restype = i32
    L._learned_declared = True


class _View:
    """A device pointer range inside another DeviceArray (no ownership)."""

    def __init__(self, base: "DeviceArray", start: int, count: int):
        self.ptr = base.ptr + start * base.dtype.itemsize
        self.count = count
        self.dtype = base.dtype
        self._base = base


class MLP:
    """The splitter-scoring network (mlp_create / mlp_forward / mlp_train_step)."""

    def __init__(self, in_features: int = POLICY_FEATURES, init: Optional[np.ndarray] = None,
                 seed: int = 0):
        L = load_library()
        _declare_learned(L)
        self._L = L
        self.F = int(in_features)
        self.P = int(L.mlp_num_params(self.F))
        if self.P < 0:
            raise ValueError("in_features must be 1..32")
        h = ctypes.c_void_p()
        pinit = None
        if init is not None:
            init = np.ascontiguousarray(init, np.float32)
            if init.size != self.P:
                raise ValueError(f"init must have {self.P} values")
            pinit = init.ctypes.data_as(ctypes.c_void_p)
        _check(L.mlp_create(self.F, pinit, int(seed), ctypes.byref(h)))
        self._h = h

    def params(self) -> np.ndarray:
        out = np.empty(self.P, np.float32)
        _check(self._L.mlp_get_params(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def forward(self, x) -> np.ndarray:
        xd = x if not isinstance(x, np.ndarray) else DeviceArray.from_numpy(x, np.float32)
        rows = xd.count // self.F
        y = DeviceArray(rows, np.float32)
        _check(self._L.mlp_forward(self._h, ctypes.c_void_p(xd.ptr), rows, ctypes.c_void_p(y.ptr),
                                   None))
        return y.numpy()

    def forward_bf16(self, x_bits) -> np.ndarray:
        """mlp_forward_bf16: x_bits holds bf16 bit patterns (uint16, rows x F)."""
        xd = x_bits if not isinstance(x_bits, np.ndarray) else \
            DeviceArray.from_numpy(np.ascontiguousarray(x_bits, np.uint16), np.uint16)
        rows = xd.count // self.F
        y = DeviceArray(rows, np.float32)
        _check(self._L.mlp_forward_bf16(self._h, ctypes.c_void_p(xd.ptr), rows,
                                        ctypes.c_void_p(y.ptr), None))
        return y.numpy()

    def train_step(self, x, t, lr: float, want_grad: bool = False):
        """One Adam step on (x, t); returns the loss before the step (and the
        gradient when want_grad)."""
        xd = x if not isinstance(x, np.ndarray) else DeviceArray.from_numpy(x, np.float32)
        td = t if not isinstance(t, np.ndarray) else DeviceArray.from_numpy(t, np.float32)
        rows = td.count
        g = DeviceArray(self.P, np.float32) if want_grad else None
        loss = ctypes.c_float(0)
        _check(self._L.mlp_train_step(self._h, ctypes.c_void_p(xd.ptr), ctypes.c_void_p(td.ptr),
                                      rows, float(lr), ctypes.byref(loss),
                                      ctypes.c_void_p(g.ptr) if g else None, None))
        return (loss.value, g.numpy()) if want_grad else loss.value

    def close(self):
        if getattr(self, "_h", None):
            self._L.mlp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_splitter_policy(lts: "LTS", policy: int, mlp: Optional[MLP] = None,
                        rescore_every: int = 64):
    L = load_library()
    _declare_learned(L)
    _check(L.bisim_set_splitter_policy(lts._h, int(policy), mlp._h if mlp is not None else None,
                                       int(rescore_every)))
    lts._policy_mlp = mlp  # keep the network alive while the handle uses it


def collect_training(lts: "LTS", sample_every: int = 1, max_cands: int = 64, cap: int = 100_000):
    """Plain run with sampled (features, counterfactual target) rows.
    Returns (feat [rows, 19], target [rows], meta [rows, 2] = (iteration, block))."""
    L = load_library()
    _declare_learned(L)
    f = DeviceArray(cap * POLICY_FEATURES, np.float32)
    t = DeviceArray(cap, np.float32)
    m = DeviceArray(cap * 2, np.int32)
    rows = ctypes.c_int64(0)
    _check(L.bisim_collect_training(lts._h, int(sample_every), int(max_cands), ctypes.c_void_p(f.ptr),
                                    ctypes.c_void_p(t.ptr), ctypes.c_void_p(m.ptr), cap,
                                    ctypes.byref(rows)))
    r = rows.value
    return (f.numpy()[:r * POLICY_FEATURES].reshape(r, POLICY_FEATURES), t.numpy()[:r],
            m.numpy()[:2 * r].reshape(r, 2))


def copy_bandwidth(nbytes: int = 1 << 30, repeats: int = 5) -> float:
    """GB/s of a plain device copy of nbytes (read + write counted), best of
    `repeats` (bisim_device_copy)."""
    L = load_library()
    if not getattr(L, "_copy_declared", False):
        L.bisim_device_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
        L.bisim_device_copy.restype = ctypes.c_int32
        L._copy_declared = True
    nbytes -= nbytes % 16
    a = DeviceArray(nbytes // 4, np.int32).fill(1)
    b = DeviceArray(nbytes // 4, np.int32)
    best = float("inf")
    for _ in range(repeats):
        ms = ctypes.c_double(0)
        _check(L.bisim_device_copy(ctypes.c_void_p(b.ptr), ctypes.c_void_p(a.ptr), nbytes, None,
                                   ctypes.byref(ms)))
        best = min(best, ms.value)
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def coarsest_partition(src, lab, dst, n: int, num_actions: int, init=None,
                       engine: int = ENGINE_AUTO):
    """One-shot: load, refine, free.  Returns (block ids as numpy, Stats)."""
    with LTS(src, lab, dst, n, num_actions, init) as h:
        if engine:
            h.set_option(OPT_ENGINE, engine)
        out, st = h.run()
        return out.numpy(), st


def coarsest_partition_noalloc(src, lab, dst, n: int, num_actions: int, init=None, out=None,
                               stream: Optional[int] = None):
    """coarsest_partition_noalloc: load + refine in the library's static
    device region, allocating nothing.  src/lab/dst/init/out are device
    buffers (DeviceArray or anything with an integer `ptr`), allocated by the
    caller; `out` (n int32 entries) receives the result.  Returns Stats."""
    L = load_library()
    m = int(getattr(src, "count"))
    n = int(n)
    ps, pl, pd = (_dptr(x, nm, m) if m else None
                  for x, nm in ((src, "src"), (lab, "label"), (dst, "dst")))
    pi = _dptr(init, "init_partition", n) if (init is not None and n) else None
    po = _dptr(out, "block_id", n) if n else None
    st = bisim_stats()
    _check(L.coarsest_partition_noalloc(ps, pl, pd, n, m, int(num_actions), pi, po,
                                        ctypes.byref(st),
                                        ctypes.c_void_p(stream) if stream else None))
    return Stats(st.iterations, st.blocks, st.pre_blocks, st.mark_length, st.t_pre_ms,
                 st.t_alg_ms)
