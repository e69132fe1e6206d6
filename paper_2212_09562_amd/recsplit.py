"""ctypes binding of librecsplit.so (include/recsplit.h).

Argument marshalling only: every step of construction and evaluation runs
in the library's HIP kernels.  Keys are (n, 2) arrays of (w0, w1) words:
numpy uint64 arrays live in host memory; torch tensors on a HIP device
(int64 or uint64, contiguous) are passed by device pointer.  Importing this
module imports torch first (one HIP runtime per process), then loads the
library, and raises if it has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

# torch first: its HIP runtime is then the one this library binds to (by
# soname), so a process never holds two HIP runtimes and device pointers from
# torch tensors and from the library live in the same context.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librecsplit.so")

RS_FLAG_ROTATION = 1
RS_FLAG_KEYS_ON_DEVICE = 2
RS_FLAG_KEEP_VALUES = 4
RS_PENDING = 1
RS_NOALLOC_MAX_KEYS = 1 << 19

ERRORS = {0: "RS_OK", -1: "RS_ERR_INVALID_ARG", -2: "RS_ERR_DUPLICATE", -3: "RS_ERR_OOM",
          -4: "RS_ERR_DEVICE", -5: "RS_ERR_CORRUPT", -6: "RS_ERR_SEARCH_LIMIT",
          -7: "RS_ERR_UNSUPPORTED"}


class RecSplitError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {ERRORS.get(code, code)} ({_lib.rs_strerror(code).decode()})")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("nb", ctypes.c_uint64), ("nodes", ctypes.c_uint64),
                ("split_nodes", ctypes.c_uint64), ("leaf_nodes", ctypes.c_uint64),
                ("useful_evals_split", ctypes.c_uint64), ("useful_evals_leaf", ctypes.c_uint64),
                ("early_exit_evals_leaf", ctypes.c_double),
                ("early_exit_evals_split", ctypes.c_double), ("gr_bits", ctypes.c_uint64), ("bytes", ctypes.c_uint64),
                ("max_bucket", ctypes.c_uint32), ("workers", ctypes.c_uint32),
                ("ms_sort", ctypes.c_double), ("ms_search", ctypes.c_double),
                ("ms_encode", ctypes.c_double), ("ms_total", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ValuRates(ctypes.Structure):
    _fields_ = [("add_u32", ctypes.c_double), ("xor_b32", ctypes.c_double),
                ("mul_lo_u32", ctypes.c_double), ("mul_hi_u32", ctypes.c_double),
                ("mad_u64_u32", ctypes.c_double), ("lshrrev_b64", ctypes.c_double),
                ("lshl_add_u64", ctypes.c_double), ("add3_u32", ctypes.c_double),
                ("hash_evals", ctypes.c_double), ("hash_evals_sustained", ctypes.c_double),
                ("compute_units", ctypes.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                      "(hipcc --offload-arch=gfx950); there is no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)
_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_lib.rs_build.argtypes = [_vp, _u64, _u32, _u32, _u32, ctypes.POINTER(_vp)]
_lib.rs_build_noalloc.argtypes = [_vp, _u64, _u32, _u32, _u32, _vp, _u64, ctypes.POINTER(_u64)]
_lib.rs_query.argtypes = [_vp, _vp, _u64, _vp, _u32]
_lib.rs_serialize.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_u64)]
_lib.rs_deserialize.argtypes = [_vp, _u64, ctypes.POINTER(_vp)]
_lib.rs_debug_node_values.argtypes = [_vp, _u64, _vp, _u64, ctypes.POINTER(_u64)]
_lib.rs_get_stats.argtypes = [_vp, ctypes.POINTER(Stats)]


class Job(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("n", ctypes.c_uint64), ("leaf_size", ctypes.c_uint32),
                ("bucket_size", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


_lib.rs_build_batch.argtypes = [ctypes.POINTER(Job), ctypes.c_uint32, ctypes.POINTER(_vp),
                                ctypes.POINTER(ctypes.c_int)]
_lib.rs_calibrate_valu.argtypes = [ctypes.POINTER(ValuRates)]
_lib.rs_rotation_lookup.argtypes = [_u32, _u32, _u32]
_lib.rs_rotation_lookup.restype = ctypes.c_uint32
_lib.rs_attempt_work.argtypes = [_u32, _u32, _u32]
_lib.rs_attempt_work.restype = ctypes.c_double


class Schedule(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint32) for k in ("chunk_shift_small", "help_after_small",
                                                "inline_leaf_tau_small", "chunk_shift_large",
                                                "help_after_large", "inline_leaf_tau_large",
                                                "small_tasks_per_worker", "bucket_mode_max_leaf",
                                                "stall_guard_us", "max_workers",
                                                "leaf_filter_tau", "join_leaf_tau",
                                                "split_filter_tau", "rotation_lookup",
                                                "bucket_wave")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib.rs_set_schedule.argtypes = [ctypes.POINTER(Schedule)]
_lib.rs_get_schedule.argtypes = [ctypes.POINTER(Schedule)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_uint64), ("max_slots", ctypes.c_uint32),
                ("max_jobs_per_launch", ctypes.c_uint32), ("reserve_per_cu", ctypes.c_uint32)]


class RequestTimes(ctypes.Structure):
    _fields_ = [("submit", ctypes.c_double), ("admit", ctypes.c_double),
                ("done", ctypes.c_double), ("slot", ctypes.c_uint32),
                ("batch_jobs", ctypes.c_uint32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_uint64) for k in ("submitted", "completed", "launches",
                                                "keys_completed", "waiting", "bytes_in_use",
                                                "peak_bytes")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib.rs_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)]
_lib.rs_server_submit.argtypes = [_vp, ctypes.POINTER(Job), ctypes.POINTER(_u64)]
_lib.rs_server_poll.argtypes = [_vp, _u64, ctypes.c_int, ctypes.POINTER(_vp),
                                ctypes.POINTER(ctypes.c_int), ctypes.POINTER(RequestTimes)]
_lib.rs_server_get_stats.argtypes = [_vp, ctypes.POINTER(ServerStats)]
_lib.rs_server_destroy.argtypes = [_vp]
_lib.rs_server_destroy.restype = None
_lib.rs_free.argtypes = [_vp]
_lib.rs_free.restype = None
_lib.rs_strerror.argtypes = [ctypes.c_int]
_lib.rs_strerror.restype = ctypes.c_char_p
for _f in ("rs_build", "rs_build_noalloc", "rs_build_batch", "rs_query", "rs_serialize", "rs_deserialize",
           "rs_debug_node_values", "rs_get_stats", "rs_calibrate_valu", "rs_server_create",
           "rs_server_submit", "rs_server_poll", "rs_server_get_stats", "rs_set_schedule",
           "rs_get_schedule"):
    getattr(_lib, _f).restype = ctypes.c_int


def library():
    return _lib


def _check(rc: int, where: str):
    if rc != 0:
        raise RecSplitError(rc, where)


def _keys_arg(keys):
    """(pointer, n, flags, keepalive) for host numpy or device torch keys."""
    if isinstance(keys, np.ndarray):
        k = np.ascontiguousarray(keys, dtype=np.uint64)
        if k.ndim != 2 or k.shape[1] != 2:
            raise ValueError("keys must have shape (n, 2)")
        return k.ctypes.data if k.size else None, k.shape[0], 0, k
    if not isinstance(keys, torch.Tensor) or keys.device.type != "cuda":
        raise TypeError("keys must be a numpy array or a torch tensor on a HIP device")
    if keys.dim() != 2 or keys.shape[1] != 2 or keys.element_size() != 8 or not keys.is_contiguous():
        raise ValueError("device keys must be a contiguous (n, 2) tensor of 64-bit words")
    return keys.data_ptr() if keys.numel() else None, keys.shape[0], RS_FLAG_KEYS_ON_DEVICE, keys


def _check_out(out, n: int, device):
    """The query kernel writes n 64-bit words through out's pointer: it must be
    a contiguous tensor of 8-byte elements on the keys' device with room for n."""
    if not isinstance(out, torch.Tensor):
        raise TypeError("out must be a torch tensor")
    if out.device != device:
        raise ValueError(f"out is on {out.device}, the keys on {device}")
    if out.element_size() != 8 or out.is_floating_point() or out.is_complex():
        raise ValueError("out must hold 64-bit integers")
    if not out.is_contiguous():
        raise ValueError("out must be contiguous")
    if out.numel() < n:
        raise ValueError(f"out holds {out.numel()} elements, {n} are needed")


class MPHF:
    """A built (or deserialised) minimal perfect hash function."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    def __del__(self):
        self.free()

    def free(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.rs_free(h)
            self._h = ctypes.c_void_p(0)

    def serialize(self) -> bytes:
        p, n = ctypes.c_void_p(), ctypes.c_uint64()
        _check(_lib.rs_serialize(self._h, ctypes.byref(p), ctypes.byref(n)), "rs_serialize")
        return ctypes.string_at(p.value, n.value)

    def query(self, keys, out=None):
        ptr, n, flags, keep = _keys_arg(keys)
        if flags & RS_FLAG_KEYS_ON_DEVICE:
            if out is None:
                out = torch.empty(n, dtype=torch.int64, device=keys.device)
            else:
                _check_out(out, n, keys.device)
            _check(_lib.rs_query(self._h, ptr, n, out.data_ptr() if n else None, flags), "rs_query")
            return out
        if out is not None:
            raise ValueError("out is for device keys only; host queries return a new array")
        res = np.zeros(n, dtype=np.uint64)
        _check(_lib.rs_query(self._h, ptr, n, res.ctypes.data if n else None, 0), "rs_query")
        return res

    def node_values(self, bucket: int) -> np.ndarray:
        cnt = ctypes.c_uint64()
        _lib.rs_debug_node_values(self._h, bucket, None, 0, ctypes.byref(cnt))
        out = np.zeros(max(cnt.value, 1), dtype=np.uint64)
        _check(_lib.rs_debug_node_values(self._h, bucket, out.ctypes.data, len(out),
                                         ctypes.byref(cnt)), "rs_debug_node_values")
        return out[:cnt.value]

    def stats(self) -> dict:
        st = Stats()
        _check(_lib.rs_get_stats(self._h, ctypes.byref(st)), "rs_get_stats")
        return st.as_dict()


def build(keys, leaf_size: int, bucket_size: int, rotation: bool = True,
          keep_values: bool = False) -> MPHF:
    """rs_build on host (numpy) or device (torch) keys."""
    ptr, n, flags, keep = _keys_arg(keys)
    flags |= (RS_FLAG_ROTATION if rotation else 0) | (RS_FLAG_KEEP_VALUES if keep_values else 0)
    h = ctypes.c_void_p()
    _check(_lib.rs_build(ptr, n, leaf_size, bucket_size, flags, ctypes.byref(h)), "rs_build")
    return MPHF(h.value)


def build_noalloc(keys, leaf_size: int, bucket_size: int, rotation: bool = True,
                  cap_words: int | None = None) -> bytes:
    """rs_build_noalloc: the serialised structure (the bytes build(...).serialize()
    gives) built in the library's fixed device array, for callers that may not
    allocate device memory; at most RS_NOALLOC_MAX_KEYS keys.  cap_words sizes
    the host output buffer (default: room for 8 bits per key); a structure that
    needs more is built again into a buffer of the size the library reports."""
    ptr, n, flags, keep = _keys_arg(keys)
    flags |= RS_FLAG_ROTATION if rotation else 0
    cap = cap_words if cap_words is not None else 64 + n // 8 + 4 * (n // max(bucket_size, 1))
    for _ in range(2):
        out = np.zeros(max(int(cap), 1), dtype=np.uint64)
        nw = ctypes.c_uint64()
        rc = _lib.rs_build_noalloc(ptr, n, leaf_size, bucket_size, flags, out.ctypes.data,
                                   len(out), ctypes.byref(nw))
        if rc == -1 and nw.value > len(out):
            cap = nw.value
            continue
        _check(rc, "rs_build_noalloc")
        return out[:nw.value].tobytes()
    raise RecSplitError(-1, "rs_build_noalloc")


def build_batch(jobs):
    """rs_build_batch: jobs is a sequence of dicts with keys, leaf_size,
    bucket_size and optionally rotation (default True) and keep_values.
    Returns (list of MPHF or None, list of status codes)."""
    arr = (Job * max(len(jobs), 1))()
    keep = []
    for i, j in enumerate(jobs):
        ptr, n, flags, k = _keys_arg(j["keys"])
        keep.append(k)
        flags |= RS_FLAG_ROTATION if j.get("rotation", True) else 0
        flags |= RS_FLAG_KEEP_VALUES if j.get("keep_values", False) else 0
        arr[i] = Job(ptr, n, j["leaf_size"], j["bucket_size"], flags)
    outs = (ctypes.c_void_p * max(len(jobs), 1))()
    st = (ctypes.c_int * max(len(jobs), 1))()
    _lib.rs_build_batch(arr, len(jobs), outs, st)
    res = [MPHF(outs[i]) if outs[i] else None for i in range(len(jobs))]
    return res, [int(st[i]) for i in range(len(jobs))]


class Server:
    """rs_server_*: continuous batching of build requests under an HBM budget.

    submit() queues a request and returns its ticket; the key array is kept
    alive here until its result is collected with poll()/wait()."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 4, max_jobs_per_launch: int = 16,
                 reserve_per_cu: int = 0):
        cfg = ServerConfig(hbm_budget_bytes, max_slots, max_jobs_per_launch, reserve_per_cu)
        h = ctypes.c_void_p()
        _check(_lib.rs_server_create(ctypes.byref(cfg), ctypes.byref(h)), "rs_server_create")
        self._h = h
        self._keep = {}

    def submit(self, keys, leaf_size: int, bucket_size: int, rotation: bool = True,
               keep_values: bool = False) -> int:
        ptr, n, flags, k = _keys_arg(keys)
        flags |= (RS_FLAG_ROTATION if rotation else 0) | (RS_FLAG_KEEP_VALUES if keep_values else 0)
        job = Job(ptr, n, leaf_size, bucket_size, flags)
        t = ctypes.c_uint64()
        _check(_lib.rs_server_submit(self._h, ctypes.byref(job), ctypes.byref(t)),
               "rs_server_submit")
        self._keep[t.value] = k
        return t.value

    def poll(self, ticket: int, wait: bool = False):
        """None while pending; else (MPHF or None, status, times dict)."""
        h, st, tm = ctypes.c_void_p(), ctypes.c_int(), RequestTimes()
        rc = _lib.rs_server_poll(self._h, ticket, 1 if wait else 0, ctypes.byref(h),
                                 ctypes.byref(st), ctypes.byref(tm))
        if rc == RS_PENDING:
            return None
        _check(rc, "rs_server_poll")
        self._keep.pop(ticket, None)
        return (MPHF(h.value) if h.value else None), st.value, tm.as_dict()

    def wait(self, ticket: int):
        return self.poll(ticket, wait=True)

    def stats(self) -> dict:
        st = ServerStats()
        _check(_lib.rs_server_get_stats(self._h, ctypes.byref(st)), "rs_server_get_stats")
        return st.as_dict()

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.rs_server_destroy(h)
            self._h = ctypes.c_void_p(0)
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        self.close()


def get_schedule() -> dict:
    """The search schedule (rs_get_schedule)."""
    sc = Schedule()
    _check(_lib.rs_get_schedule(ctypes.byref(sc)), "rs_get_schedule")
    return sc.as_dict()


def set_schedule(schedule=None, **changes) -> dict:
    """rs_set_schedule: None (and no changes) restores the defaults; otherwise
    the given fields replace those of ``schedule`` (default: the current one).
    Returns the schedule now in force."""
    if schedule is None and not changes:
        _check(_lib.rs_set_schedule(None), "rs_set_schedule")
        return get_schedule()
    sc = dict(schedule or get_schedule())
    sc.update(changes)
    _check(_lib.rs_set_schedule(ctypes.byref(Schedule(**sc))), "rs_set_schedule")
    return get_schedule()


def deserialize(data: bytes) -> MPHF:
    buf = np.frombuffer(data, dtype=np.uint8)
    h = ctypes.c_void_p()
    _check(_lib.rs_deserialize(buf.ctypes.data if len(buf) else None, len(buf), ctypes.byref(h)),
           "rs_deserialize")
    return MPHF(h.value)


def strerror(code: int) -> str:
    return _lib.rs_strerror(code).decode()


def attempt_work(leaf_size: int, node_size: int, rotation: bool = True) -> float:
    """Expected hash evaluations of one failed attempt at a node of node_size
    keys when it stops at the first evidence that it fails (host only)."""
    w = _lib.rs_attempt_work(leaf_size, node_size, RS_FLAG_ROTATION if rotation else 0)
    if w < 0:
        raise RecSplitError(-1, "rs_attempt_work")
    return w


def calibrate_valu() -> dict:
    """Issue rates of the VALU instruction classes of a hash evaluation."""
    r = ValuRates()
    _check(_lib.rs_calibrate_valu(ctypes.byref(r)), "rs_calibrate_valu")
    return r.as_dict()


def rotation_lookup(m: int, a: int, b: int) -> int:
    """rs_rotation_lookup: the smallest rotation r with a | rot_m^r(b) filling
    all m bits, found by table lookups (host only); m when none fits."""
    r = _lib.rs_rotation_lookup(m, a, b)
    if r == 0xFFFFFFFF:
        raise RecSplitError(-1, "rs_rotation_lookup")
    return r
