"""Python binding of libpcfsort.so (ctypes; argument marshalling only).

Every function here forwards to the C ABI declared in include/pcfsort.h with
the same name.  Device buffers are torch tensors on a ROCm device (torch is
used only for memory and streams); every step of the sort runs in the
library's HIP kernels.  There is no CPU fallback: if the library or a GPU is
missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpcfsort.so")

OK = 0
ERR_INVALID_ARGUMENT = 1
ERR_INVALID_KEY = 2
ERR_OUT_OF_MEMORY = 3
ERR_HIP = 4
ERR_UNSUPPORTED = 5
PENDING = 6
ERR_UNKNOWN_TICKET = 7
ERR_SHUTDOWN = 8

KEY_F64 = 0
KEY_U64 = 1

EXPORTS = [
    "pcf_status_string", "pcf_last_hip_error", "pcf_version", "pcf_workspace_bytes",
    "pcf_sort_f64", "pcf_sort_u64", "pcf_sort_f64_static", "pcf_sort_inplace",
    "pcf_inplace_workspace_bytes", "pcf_argsort", "pcf_sort_segmented", "pcf_level_trace",
    "pcf_get_policy", "pcf_set_policy", "pcf_autotune", "pcf_load_tuning",
    "pcf_serve_create", "pcf_serve_submit", "pcf_serve_submit_after", "pcf_serve_poll", "pcf_serve_wait",
    "pcf_serve_release", "pcf_serve_get_stats", "pcf_serve_destroy",
    "pcf_profile_enable", "pcf_profile_select", "pcf_profile_read", "pcf_kernel_name", "pcf_graph_stats",
    "pcf_graph_clear", "pcf_policy_for", "pcf_lfail_grid",
]

KERNEL_KINDS = ["setup", "range", "fit", "count", "colscan", "classify", "scatter", "lds_small",
                "lds_big", "radix_keys", "bitonic_keys", "single_keys"]


class PcfError(RuntimeError):
    def __init__(self, code: int, where: str):
        lib = _lib
        msg = lib.pcf_status_string(code).decode() if lib is not None else str(code)
        if code == ERR_HIP and lib is not None:
            msg += f" (hipError {lib.pcf_last_hip_error()})"
        super().__init__(f"{where}: {msg}")
        self.code = code


class Policy(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint32) for name in (
        "max_buckets", "target_child", "bins_per_bucket", "max_bins", "samples_per_bucket",
        "max_samples", "chunk_keys", "lds_cap", "tau", "seed", "model", "scatter_tile")]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


class KernelStat(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("ms", ctypes.c_double), ("keys", ctypes.c_double),
                ("fallback_ms", ctypes.c_double)]


class ServeConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_streams", ctypes.c_uint32),
                ("max_batch_requests", ctypes.c_uint32), ("max_batch_keys", ctypes.c_uint64),
                ("device", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class ServeResult(ctypes.Structure):
    _fields_ = [("d_keys_sorted", ctypes.c_void_p), ("d_idx", ctypes.c_void_p),
                ("n", ctypes.c_uint64), ("latency_ns", ctypes.c_uint64),
                ("queue_ns", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("batch_requests", ctypes.c_uint32)]


class ServeStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "submitted", "completed", "released", "batches", "budget_bytes", "budget_in_use",
        "budget_high_water", "queued")]

    def as_dict(self) -> dict:
        return {n: getattr(self, n) for n, _ in self._fields_}


_lib = None

_VP = ctypes.c_void_p
_SZ = ctypes.c_size_t
_U32 = ctypes.c_uint32
_U64 = ctypes.c_uint64
_I32 = ctypes.c_int32
_INT = ctypes.c_int


def load(path: str = LIB_PATH):
    """Loads libpcfsort.so; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run paper_2405_07122_amd/build.py "
                          f"(or __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    sig = {
        "pcf_status_string": (ctypes.c_char_p, [_INT]),
        "pcf_last_hip_error": (_INT, []),
        "pcf_version": (ctypes.c_char_p, []),
        "pcf_workspace_bytes": (_SZ, [_INT, _SZ, _INT, _U32]),
        "pcf_sort_f64": (_INT, [_VP, _VP, _SZ, _VP, _SZ, _VP, _VP]),
        "pcf_sort_u64": (_INT, [_VP, _VP, _SZ, _VP, _SZ, _VP, _VP]),
        "pcf_sort_f64_static": (_INT, [_VP, _VP, _SZ, _VP, _VP]),
        "pcf_sort_inplace": (_INT, [_INT, _VP, _SZ, _VP, _SZ, _VP]),
        "pcf_inplace_workspace_bytes": (_SZ, [_INT, _SZ]),
        "pcf_argsort": (_INT, [_INT, _VP, _VP, _VP, _SZ, _VP, _SZ, _VP, _VP]),
        "pcf_sort_segmented": (_INT, [_INT, _VP, _VP, _VP, _VP, _VP, _U32, _SZ, _VP, _SZ, _VP,
                                      _VP]),
        "pcf_level_trace": (_INT, [_INT, _VP, _VP, _SZ, _U64, _U32, _U32, _U32, _VP, _VP, _VP,
                                   _VP, _VP, _VP, _VP]),
        "pcf_get_policy": (_INT, [ctypes.POINTER(Policy)]),
        "pcf_set_policy": (_INT, [ctypes.POINTER(Policy)]),
        "pcf_autotune": (_INT, [_INT, _INT, ctypes.c_char_p]),
        "pcf_load_tuning": (_INT, [ctypes.c_char_p]),
        "pcf_serve_create": (_INT, [ctypes.POINTER(ServeConfig), ctypes.POINTER(_VP)]),
        "pcf_serve_submit": (_INT, [_VP, _INT, _VP, _SZ, _INT, ctypes.POINTER(_U64)]),
        "pcf_serve_submit_after": (_INT, [_VP, _INT, _VP, _SZ, _INT, _VP, ctypes.POINTER(_U64)]),
        "pcf_serve_poll": (_INT, [_VP, _U64, ctypes.POINTER(ServeResult)]),
        "pcf_serve_wait": (_INT, [_VP, _U64, _U32, ctypes.POINTER(ServeResult)]),
        "pcf_serve_release": (_INT, [_VP, _U64]),
        "pcf_serve_get_stats": (_INT, [_VP, ctypes.POINTER(ServeStats)]),
        "pcf_serve_destroy": (_INT, [_VP]),
        "pcf_profile_enable": (_INT, [_INT]),
        "pcf_profile_read": (_INT, [ctypes.POINTER(KernelStat), _INT]),
        "pcf_profile_select": (_INT, [ctypes.c_uint32]),
        "pcf_kernel_name": (ctypes.c_char_p, [_INT]),
        "pcf_graph_stats": (_INT, [ctypes.POINTER(_U64)] * 3),
        "pcf_graph_clear": (_INT, []),
        "pcf_policy_for": (_INT, [_INT, _SZ, _INT, ctypes.POINTER(Policy)]),
        "pcf_lfail_grid": (_INT, [_VP, _SZ, _U32, _VP, _U32, _U64, _VP, _VP]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int, where: str):
    if rc != OK:
        raise PcfError(rc, where)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _key_type(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return KEY_F64
    if t.dtype in (torch.int64, torch.uint64):
        return KEY_U64  # 64-bit unsigned keys may travel in an int64 tensor
    raise TypeError(f"keys must be float64 or (u)int64, got {t.dtype}")


def _need_cuda(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("tensors must be contiguous and on a ROCm device")


def version() -> str:
    return load().pcf_version().decode()


def workspace_bytes(key_type: int, n: int, with_payload: bool = False, num_segments: int = 1) -> int:
    return int(load().pcf_workspace_bytes(key_type, n, int(with_payload), num_segments))


def workspace(key_type: int, n: int, with_payload: bool = False, num_segments: int = 1,
              device=None) -> torch.Tensor:
    """A device workspace tensor large enough for the given sort."""
    nb = workspace_bytes(key_type, n, with_payload, num_segments)
    return torch.empty(max(nb, 1), dtype=torch.uint8, device=device or "cuda")


def _ws_args(ws):
    if ws is None:
        return None, 0
    return _ptr(ws), ws.numel() * ws.element_size()


def pcf_sort_f64(keys: torch.Tensor, out: torch.Tensor | None = None, ws=None, d_status=None,
                 stream=None) -> torch.Tensor:
    lib = load()
    if keys.dtype != torch.float64:
        raise TypeError("pcf_sort_f64 needs float64 keys")
    out = torch.empty_like(keys) if out is None else out
    _need_cuda(keys, out)
    wp, wb = _ws_args(ws)
    _check(lib.pcf_sort_f64(_ptr(keys), _ptr(out), keys.numel(), wp, wb, _ptr(d_status),
                            _stream(stream)), "pcf_sort_f64")
    return out


def pcf_sort_u64(keys: torch.Tensor, out: torch.Tensor | None = None, ws=None, d_status=None,
                 stream=None) -> torch.Tensor:
    lib = load()
    if keys.dtype not in (torch.int64, torch.uint64):
        raise TypeError("pcf_sort_u64 needs 64-bit integer keys (read as unsigned)")
    out = torch.empty_like(keys) if out is None else out
    _need_cuda(keys, out)
    wp, wb = _ws_args(ws)
    _check(lib.pcf_sort_u64(_ptr(keys), _ptr(out), keys.numel(), wp, wb, _ptr(d_status),
                            _stream(stream)), "pcf_sort_u64")
    return out


STATIC_SCRATCH_BYTES = 128 << 20  # PCF_STATIC_SCRATCH_BYTES


def pcf_sort_f64_static(keys: torch.Tensor, d_status: torch.Tensor, out: torch.Tensor | None = None,
                        stream=None) -> torch.Tensor:
    """pcf_sort_f64 with the library's static scratch as workspace (no
    allocation by the library); `d_status` (int32 device tensor) is required."""
    lib = load()
    if keys.dtype != torch.float64:
        raise TypeError("pcf_sort_f64_static needs float64 keys")
    out = torch.empty_like(keys) if out is None else out
    _need_cuda(keys, out, d_status)
    _check(lib.pcf_sort_f64_static(_ptr(keys), _ptr(out), keys.numel(), _ptr(d_status),
                                   _stream(stream)), "pcf_sort_f64_static")
    return out


def inplace_workspace_bytes(key_type: int, n: int) -> int:
    return int(load().pcf_inplace_workspace_bytes(key_type, n))


def pcf_sort_inplace(keys: torch.Tensor, ws=None, stream=None) -> torch.Tensor:
    """Sorts `keys` (float64 or 64-bit integer read as unsigned) within its own
    memory; returns `keys`.  Waits for the stream."""
    lib = load()
    kt = _key_type(keys)
    _need_cuda(keys)
    wp, wb = _ws_args(ws)
    _check(lib.pcf_sort_inplace(kt, _ptr(keys), keys.numel(), wp, wb, _stream(stream)),
           "pcf_sort_inplace")
    return keys


def sort(keys: torch.Tensor, out=None, ws=None, d_status=None, stream=None) -> torch.Tensor:
    if _key_type(keys) == KEY_F64:
        return pcf_sort_f64(keys, out, ws, d_status, stream)
    return pcf_sort_u64(keys, out, ws, d_status, stream)


def pcf_argsort(keys: torch.Tensor, keys_out: torch.Tensor | None = None,
                idx_out: torch.Tensor | None = None, ws=None, d_status=None, stream=None,
                want_keys: bool = True):
    """Stable argsort: returns (sorted keys or None, int32 tensor of input positions
    holding uint32 values)."""
    lib = load()
    kt = _key_type(keys)
    n = keys.numel()
    if keys_out is None and want_keys:
        keys_out = torch.empty_like(keys)
    if idx_out is None:
        idx_out = torch.empty(n, dtype=torch.int32, device=keys.device)
    _need_cuda(keys, keys_out, idx_out)
    wp, wb = _ws_args(ws)
    _check(lib.pcf_argsort(kt, _ptr(keys), _ptr(keys_out), _ptr(idx_out), n, wp, wb,
                           _ptr(d_status), _stream(stream)), "pcf_argsort")
    return keys_out, idx_out


def pcf_sort_segmented(keys: torch.Tensor, offsets: torch.Tensor, vals: torch.Tensor | None = None,
                       keys_out=None, vals_out=None, ws=None, d_status=None, stream=None):
    """Each CSR segment [offsets[s], offsets[s+1]) sorted on its own, stably,
    carrying `vals` (int32 tensor holding uint32 words).  offsets: int64 device
    tensor of num_segments + 1 entries."""
    lib = load()
    kt = _key_type(keys)
    keys_out = torch.empty_like(keys) if keys_out is None else keys_out
    if vals is not None and vals_out is None:
        vals_out = torch.empty_like(vals)
    _need_cuda(keys, offsets, vals, keys_out, vals_out)
    nseg = offsets.numel() - 1
    wp, wb = _ws_args(ws)
    _check(lib.pcf_sort_segmented(kt, _ptr(keys), _ptr(keys_out), _ptr(vals), _ptr(vals_out),
                                  _ptr(offsets), nseg, keys.numel(), wp, wb, _ptr(d_status),
                                  _stream(stream)), "pcf_sort_segmented")
    return keys_out, vals_out


def pcf_graph_stats() -> dict:
    """Graph cache counters of the segmented path."""
    c, r, h = _U64(), _U64(), _U64()
    _check(load().pcf_graph_stats(ctypes.byref(c), ctypes.byref(r), ctypes.byref(h)),
           "pcf_graph_stats")
    return {"captures": c.value, "replays": r.value, "cached": h.value}


def pcf_graph_clear() -> None:
    _check(load().pcf_graph_clear(), "pcf_graph_clear")


def pcf_lfail_grid(arrays: torch.Tensor, cells, seed: int = 0, stream=None):
    """Bucketing-failure counts (Sec. 4.2): `arrays` is a (reps, n) float64
    device tensor; `cells` a sequence of (alpha, beta, gamma, delta).  Returns a
    numpy array of failure counts per cell (out of reps)."""
    import numpy as np
    _need_cuda(arrays)
    reps, n = arrays.shape
    hc = np.ascontiguousarray(np.asarray(cells, dtype=np.uint32).reshape(-1, 4))
    out = np.zeros(hc.shape[0], dtype=np.uint32)
    _check(load().pcf_lfail_grid(_ptr(arrays), n, reps, hc.ctypes.data, hc.shape[0], seed,
                                 out.ctypes.data, _stream(stream)), "pcf_lfail_grid")
    return out


def pcf_level_trace(keys: torch.Tensor, alpha: int, beta: int, gamma: int, node_seed: int,
                    vals: torch.Tensor | None = None, stream=None) -> dict:
    """One model-based bucketing on the GPU with explicit parameters; returns
    the model (b, T), bucket sizes and the stable partition."""
    import numpy as np
    lib = load()
    kt = _key_type(keys)
    part = torch.empty_like(keys)
    pvals = torch.empty_like(vals) if vals is not None else None
    _need_cuda(keys, vals)
    hb = np.zeros(beta + 1, dtype=np.uint64)
    hT = np.zeros(beta + 1, dtype=np.uint64)
    hs = np.zeros(gamma + 1, dtype=np.uint64)
    sc = np.zeros(5, dtype=np.uint64)
    _check(lib.pcf_level_trace(kt, _ptr(keys), _ptr(vals), keys.numel(), node_seed, alpha, beta,
                               gamma, _ptr(part), _ptr(pvals), hb.ctypes.data, hT.ctypes.data,
                               hs.ctypes.data, sc.ctypes.data, _stream(stream)),
           "pcf_level_trace")
    return {"b": hb, "T": hT, "sizes": hs, "min_bits": int(sc[0]), "max_bits": int(sc[1]),
            "scale_bits": int(sc[2]), "halves": int(sc[3]), "status": int(sc[4]),
            "part_keys": part, "part_vals": pvals}


def get_policy() -> dict:
    p = Policy()
    _check(load().pcf_get_policy(ctypes.byref(p)), "pcf_get_policy")
    return p.as_dict()


def set_policy(**kw) -> dict:
    p = Policy()
    lib = load()
    _check(lib.pcf_get_policy(ctypes.byref(p)), "pcf_get_policy")
    for k, v in kw.items():
        setattr(p, k, int(v))
    _check(lib.pcf_set_policy(ctypes.byref(p)), "pcf_set_policy")
    return p.as_dict()


def pcf_autotune(key_type: int, with_payload: bool, out_json: str) -> None:
    _check(load().pcf_autotune(key_type, int(with_payload), out_json.encode()), "pcf_autotune")


def pcf_load_tuning(path: str | None) -> None:
    """Installs a tuning table; None clears it."""
    _check(load().pcf_load_tuning(path.encode() if path is not None else None), "pcf_load_tuning")


def policy_for(key_type: int, n: int, with_payload: bool = False) -> dict:
    p = Policy()
    _check(load().pcf_policy_for(key_type, n, int(with_payload), ctypes.byref(p)), "pcf_policy_for")
    return p.as_dict()


def pcf_profile_enable(on: bool = True) -> None:
    _check(load().pcf_profile_enable(int(on)), "pcf_profile_enable")


def pcf_profile_select(kinds=None) -> None:
    """Record events only for the named launch kinds (None: all timed kinds)."""
    timed = KERNEL_KINDS[:KERNEL_KINDS.index("radix_keys")]
    kinds = timed if kinds is None else kinds
    mask = 0
    for k in kinds:
        mask |= 1 << timed.index(k)
    _check(load().pcf_profile_select(mask), "pcf_profile_select")


def pcf_profile_read(reset: bool = False) -> dict:
    """Per-kernel totals: {name: {"launches", "ms", "keys", "fallback_ms"}}
    (fallback_ms: the part of ms apportioned to the standard sort of failed
    buckets by key share)."""
    arr = (KernelStat * len(KERNEL_KINDS))()
    _check(load().pcf_profile_read(arr, int(reset)), "pcf_profile_read")
    return {KERNEL_KINDS[i]: {"launches": int(arr[i].launches), "ms": float(arr[i].ms),
                              "keys": float(arr[i].keys), "fallback_ms": float(arr[i].fallback_ms)}
            for i in range(len(KERNEL_KINDS))}


# ---- serving ------------------------------------------------------------------

class _DevView:
    """A device buffer owned by the server, exposed to torch without a copy."""

    def __init__(self, ptr: int, n: int, typestr: str):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (ptr, False),
                                         "version": 3, "strides": None}


class Server:
    """Continuous-batching sort server (pcf_serve_*).  submit() never blocks;
    results stay in server memory until release()."""

    def __init__(self, hbm_budget_bytes: int, max_streams: int = 2, max_batch_requests: int = 256,
                 max_batch_keys: int = 1 << 28, device: int = 0):
        lib = load()
        cfg = ServeConfig(hbm_budget_bytes, max_streams, max_batch_requests, max_batch_keys, device,
                          0)
        h = ctypes.c_void_p()
        _check(lib.pcf_serve_create(ctypes.byref(cfg), ctypes.byref(h)), "pcf_serve_create")
        self._h = h
        self._inputs = {}

    def submit(self, keys: torch.Tensor, argsort: bool = False) -> int:
        """Returns a ticket; `keys` is kept alive until the request is released.
        An event recorded on torch's current stream orders the server's read
        of `keys` after the work that produced them."""
        _need_cuda(keys)
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream(keys.device))
        t = _U64()
        _check(load().pcf_serve_submit_after(self._h, _key_type(keys), _ptr(keys), keys.numel(),
                                             int(argsort), ctypes.c_void_p(ev.cuda_event),
                                             ctypes.byref(t)), "pcf_serve_submit_after")
        self._inputs[t.value] = (keys, ev)
        return t.value

    def _result(self, r: ServeResult, kt_dtype) -> dict:
        out = {"n": int(r.n), "latency_ns": int(r.latency_ns), "queue_ns": int(r.queue_ns),
               "status": int(r.status), "batch_requests": int(r.batch_requests),
               "keys": None, "idx": None}
        if r.n and r.d_keys_sorted:
            ts = "<f8" if kt_dtype == torch.float64 else "<i8"
            out["keys"] = torch.as_tensor(_DevView(r.d_keys_sorted, r.n, ts), device="cuda")
        if r.n and r.d_idx:
            out["idx"] = torch.as_tensor(_DevView(r.d_idx, r.n, "<i4"), device="cuda")
        return out

    def poll(self, ticket: int):
        """None while pending, else the result dict (tensors view server memory)."""
        r = ServeResult()
        rc = load().pcf_serve_poll(self._h, ticket, ctypes.byref(r))
        if rc == PENDING:
            return None
        _check(rc, "pcf_serve_poll")
        return self._result(r, self._inputs[ticket][0].dtype)

    def poll_status(self, ticket: int):
        """None while pending, else (status, latency_ns, batch_requests) without
        touching the result memory."""
        r = ServeResult()
        rc = load().pcf_serve_poll(self._h, ticket, ctypes.byref(r))
        if rc == PENDING:
            return None
        _check(rc, "pcf_serve_poll")
        return int(r.status), int(r.latency_ns), int(r.batch_requests)

    def wait(self, ticket: int, timeout_ms: int = 60000):
        r = ServeResult()
        rc = load().pcf_serve_wait(self._h, ticket, timeout_ms, ctypes.byref(r))
        if rc == PENDING:
            return None
        _check(rc, "pcf_serve_wait")
        return self._result(r, self._inputs[ticket][0].dtype)

    def release(self, ticket: int) -> None:
        _check(load().pcf_serve_release(self._h, ticket), "pcf_serve_release")
        self._inputs.pop(ticket, None)

    def stats(self) -> dict:
        st = ServeStats()
        _check(load().pcf_serve_get_stats(self._h, ctypes.byref(st)), "pcf_serve_get_stats")
        return st.as_dict()

    def close(self) -> None:
        if self._h:
            _check(load().pcf_serve_destroy(self._h), "pcf_serve_destroy")
            self._h = None
            self._inputs.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
