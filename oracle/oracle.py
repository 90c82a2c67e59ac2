"""ctypes front end of the CPU oracle (liboracle.so, built from pcf_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` are the only callers.  Nothing in the
product library imports this module, and this module imports nothing from it.

What the oracle computes is documented in ``pcf_oracle.h``: Algorithm 1 of the
paper (Sec. 3.2) with the PCF model of Sec. 3.3 and the parameter rule
alpha = beta = gamma = delta = floor(n^{3/4}), tau = 100 (Sec. 4.1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = ["pcf_oracle.c"]
DEPS = ["pcf_oracle.c", "pcf_oracle_impl.h", "pcf_oracle.h"]

KEY_F64 = 0
KEY_U64 = 1

MODELS = {"pcf": 0, "spline": 1}

OK = 0
ERR_ARG = 1
ERR_INVALID_KEY = 2
ERR_NOMEM = 3

CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(out_path: str = LIB_PATH, extra_flags: list[str] | None = None) -> str:
    """Compile the oracle with gcc (always recompiles)."""
    cmd = ["gcc", *CFLAGS, *(extra_flags or []), "-o", out_path]
    cmd += [os.path.join(HERE, s) for s in SOURCES]
    cmd += ["-lm"]
    subprocess.run(cmd, check=True)
    return out_path


STDSORT_PATH = os.path.join(HERE, "libstdsort.so")


def build_stdsort(out_path: str = STDSORT_PATH) -> str:
    """Compile the std::sort timing helper (a CPU baseline, not part of the oracle)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", out_path,
           os.path.join(HERE, "std_sort_baseline.cpp")]
    subprocess.run(cmd, check=True)
    return out_path


def stdsort_seconds(x: np.ndarray) -> float:
    """Sorts a copy of fp64 `x` with std::sort on one thread; returns the seconds."""
    if not os.path.exists(STDSORT_PATH):
        build_stdsort()
    lib = ctypes.CDLL(STDSORT_PATH)
    lib.stdsort_f64_seconds.restype = ctypes.c_double
    lib.stdsort_f64_seconds.argtypes = [ctypes.c_void_p, ctypes.c_size_t]
    y = np.ascontiguousarray(x, dtype=np.float64).copy()
    return float(lib.stdsort_f64_seconds(y.ctypes.data, y.size))


class Stats(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_uint64),
        ("max_depth", ctypes.c_uint64),
        ("small_sorts", ctypes.c_uint64),
        ("fail_sorts", ctypes.c_uint64),
        ("fail_keys", ctypes.c_uint64),
        ("single_valued", ctypes.c_uint64),
        ("nonfinite_scale", ctypes.c_uint64),
        ("max_quant_lhs", ctypes.c_double),
    ]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_P64 = ctypes.POINTER(ctypes.c_uint64)
_P32 = ctypes.POINTER(ctypes.c_uint32)


class LevelIO(ctypes.Structure):
    _fields_ = [
        ("alpha", ctypes.c_uint64),
        ("beta", ctypes.c_uint64),
        ("gamma", ctypes.c_uint64),
        ("sample_idx", _P64),
        ("b", _P64),
        ("T", _P64),
        ("sizes", _P64),
        ("part_keys", ctypes.c_void_p),
        ("part_vals", _P32),
        ("sample_pos", _P64),
        ("min_bits", ctypes.c_uint64),
        ("max_bits", ctypes.c_uint64),
        ("scale", ctypes.c_double),
        ("halves", ctypes.c_int),
        ("status", ctypes.c_int),
        ("model", ctypes.c_int),
    ]


_lib = None


def load(path: str = LIB_PATH, rebuild_if_missing: bool = True):
    """Load liboracle.so, compiling it first if it is not there."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        if not rebuild_if_missing:
            raise FileNotFoundError(path)
        build(path)
    lib = ctypes.CDLL(path)
    lib.pcfo_splitmix64.restype = ctypes.c_uint64
    lib.pcfo_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.pcfo_node_seed.restype = ctypes.c_uint64
    lib.pcfo_node_seed.argtypes = [ctypes.c_uint64] * 4
    lib.pcfo_sample_index.restype = ctypes.c_uint64
    lib.pcfo_sample_index.argtypes = [ctypes.c_uint64] * 3
    lib.pcfo_root34.restype = ctypes.c_uint64
    lib.pcfo_root34.argtypes = [ctypes.c_uint64]
    lib.pcfo_quant_lhs_f64.restype = ctypes.c_double
    lib.pcfo_quant_lhs_f64.argtypes = [ctypes.c_uint64, ctypes.c_double, ctypes.c_double]
    lib.pcfo_eta_f64.restype = ctypes.c_double
    lib.pcfo_eta_f64.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.pcfo_level.restype = ctypes.c_int
    lib.pcfo_level.argtypes = [ctypes.c_int, ctypes.c_void_p, _P32, ctypes.c_uint64,
                               ctypes.c_uint64, ctypes.POINTER(LevelIO)]
    lib.pcfo_sort.restype = ctypes.c_int
    lib.pcfo_sort.argtypes = [ctypes.c_int, ctypes.c_void_p, _P32, ctypes.c_void_p, _P32,
                              ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                              ctypes.c_uint64, ctypes.POINTER(Stats)]
    lib.pcfo_sort_model.restype = ctypes.c_int
    lib.pcfo_sort_model.argtypes = [ctypes.c_int, ctypes.c_void_p, _P32, ctypes.c_void_p, _P32,
                                    ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(Stats)]
    if path == LIB_PATH:
        _lib = lib
    return lib


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle returned status {code}")
        self.code = code


def _key_type(keys: np.ndarray) -> int:
    if keys.dtype == np.float64:
        return KEY_F64
    if keys.dtype == np.uint64:
        return KEY_U64
    raise TypeError(f"unsupported key dtype {keys.dtype}")


def _p32(a):
    return None if a is None else a.ctypes.data_as(_P32)


def _p64(a):
    return None if a is None else a.ctypes.data_as(_P64)


def splitmix64(state: int, k: int, lib=None) -> int:
    return int((lib or load()).pcfo_splitmix64(state, k))


def node_seed(seed: int, segment: int, depth: int, offset: int, lib=None) -> int:
    return int((lib or load()).pcfo_node_seed(seed, segment, depth, offset))


def sample_index(nseed: int, j: int, n: int, lib=None) -> int:
    return int((lib or load()).pcfo_sample_index(nseed, j, n))


def root34(n: int, lib=None) -> int:
    return int((lib or load()).pcfo_root34(n))


def quant_lhs_f64(beta: int, lo: float, hi: float, lib=None) -> float:
    return float((lib or load()).pcfo_quant_lhs_f64(beta, lo, hi))


def eta_f64(lo: float, hi: float, lib=None) -> float:
    return float((lib or load()).pcfo_eta_f64(lo, hi))


def sort(keys: np.ndarray, vals: np.ndarray | None = None, seed: int = 0, segment: int = 0,
         tau: int = 100, lib=None, want_vals: bool | None = None, model: str = "pcf"):
    """Learned-Sort (Algorithm 1) of `keys`, carrying `vals` (uint32) stably,
    with the PCF model (Sec. 3.3) or the spline model (App. A.5).

    Returns (sorted_keys, sorted_vals or None, stats dict)."""
    lib = lib or load()
    keys = np.ascontiguousarray(keys)
    kt = _key_type(keys)
    n = keys.shape[0]
    out = np.empty_like(keys)
    if vals is not None:
        vals = np.ascontiguousarray(vals, dtype=np.uint32)
    if want_vals is None:
        want_vals = vals is not None
    vout = np.empty(n, dtype=np.uint32) if want_vals else None
    st = Stats()
    rc = lib.pcfo_sort_model(kt, keys.ctypes.data, _p32(vals), out.ctypes.data, _p32(vout), n,
                             seed, segment, tau, MODELS[model], ctypes.byref(st))
    if rc != OK:
        raise OracleError(rc)
    return out, vout, st.as_dict()


def argsort(keys: np.ndarray, seed: int = 0, segment: int = 0, tau: int = 100, lib=None,
            model: str = "pcf"):
    """Stable argsort: (sorted keys, input positions as uint32, stats)."""
    n = keys.shape[0]
    idx = np.arange(n, dtype=np.uint32)
    return sort(keys, idx, seed=seed, segment=segment, tau=tau, lib=lib, model=model)


def sort_segmented(keys: np.ndarray, offsets: np.ndarray, vals: np.ndarray | None = None,
                   seed: int = 0, tau: int = 100, lib=None, model: str = "pcf"):
    """Every CSR segment sorted on its own, the segment index naming its nodes."""
    out = np.empty_like(keys)
    vout = np.empty(keys.shape[0], dtype=np.uint32) if vals is not None else None
    for s in range(len(offsets) - 1):
        a, b = int(offsets[s]), int(offsets[s + 1])
        if b == a:
            continue
        k, v, _ = sort(keys[a:b], None if vals is None else vals[a:b], seed=seed, segment=s,
                       tau=tau, lib=lib, model=model)
        out[a:b] = k
        if vout is not None:
            vout[a:b] = v
    return out, vout


@dataclass
class Level:
    status: int
    min_bits: int
    max_bits: int
    scale: float
    halves: int
    b: np.ndarray
    T: np.ndarray
    sizes: np.ndarray
    part_keys: np.ndarray
    part_vals: np.ndarray | None
    sample_pos: np.ndarray


def level(keys: np.ndarray, alpha: int, beta: int, gamma: int, nseed: int,
          vals: np.ndarray | None = None, sample_idx: np.ndarray | None = None,
          lib=None, model: str = "pcf") -> Level:
    """One model-based bucketing with explicit parameters (trace for parity)."""
    lib = lib or load()
    keys = np.ascontiguousarray(keys)
    kt = _key_type(keys)
    n = keys.shape[0]
    b = np.zeros(beta + 1, dtype=np.uint64)
    T = np.zeros(beta + 1, dtype=np.uint64)
    sizes = np.zeros(gamma + 1, dtype=np.uint64)
    part = np.empty_like(keys)
    pv = np.empty(n, dtype=np.uint32) if vals is not None else None
    if vals is not None:
        vals = np.ascontiguousarray(vals, dtype=np.uint32)
    spos = np.zeros(alpha, dtype=np.uint64)
    if sample_idx is not None:
        sample_idx = np.ascontiguousarray(sample_idx, dtype=np.uint64)
    io = LevelIO()
    io.alpha, io.beta, io.gamma = alpha, beta, gamma
    io.sample_idx = _p64(sample_idx)
    io.b, io.T, io.sizes = _p64(b), _p64(T), _p64(sizes)
    io.part_keys = part.ctypes.data
    io.part_vals = _p32(pv)
    io.sample_pos = _p64(spos)
    io.model = MODELS[model]
    rc = lib.pcfo_level(kt, keys.ctypes.data, _p32(vals), n, nseed, ctypes.byref(io))
    if rc != OK:
        raise OracleError(rc)
    return Level(io.status, io.min_bits, io.max_bits, io.scale, io.halves, b, T, sizes, part,
                 pv, spos)
