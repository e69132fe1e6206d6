"""CPU oracle for RecSplit construction -- TEST INFRASTRUCTURE ONLY.

ctypes loader for ``recsplit_oracle.c``: a plain, slow, single-threaded C
implementation of what the GPU library computes, written from the paper
(Bez, Kurpicz, Lehmann, Sanders, arXiv 2212.09562).  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package; the product library never does, and shares no code with
it.  Parity pins for each function are in ``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "recsplit_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FLAG_ROTATION = 1
FLAG_NAIVE = 2

ERRORS = {0: "ok", -1: "invalid argument", -2: "duplicate key", -3: "out of memory",
          -5: "corrupt", -6: "search limit"}


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {ERRORS.get(code, code)} ({code})")
        self.code = code


def compile_oracle(force: bool = False) -> str:
    """Compile the oracle with the host C compiler (plain -O2, no vectorising flags)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Stats(ctypes.Structure):
    _fields_ = [("evals_split", ctypes.c_uint64), ("evals_leaf", ctypes.c_uint64),
                ("nodes_split", ctypes.c_uint64), ("nodes_leaf", ctypes.c_uint64),
                ("bf_ee_evals", ctypes.c_uint64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(compile_oracle())
        u64, u32, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        sig = {
            "or_splitmix64_next": (u64, [_u64p]),
            "or_start_seed": (u64, [u32]),
            "or_hash": (u64, [u64, u64]),
            "or_remap": (u32, [u64, u32]),
            "or_bucket_of": (u64, [u64, u64]),
            "or_num_buckets": (u64, [u64, u32]),
            "or_fanouts": (None, [u32, _u32p, _u32p]),
            "or_children": (i32, [u32, u32, _u32p]),
            "or_rot": (u32, [u32, u32, u32]),
            "or_rotation_fit": (i32, [u32, u32, u32, u32, u32]),
            "or_leaf_search": (i32, [_u64p, _u8p, u32, u32, u32, _u64p, _u64p]),
            "or_split_search": (i32, [_u64p, u32, u32, u32, _u64p]),
            "or_tau": (u32, [u32, u32]),
            "or_tau_log2arg": (ctypes.c_double, [u32, u32]),
            "or_preorder_sizes": (i32, [u32, u32, _u32p, u64, _u64p]),
            "or_build": (i32, [_u64p, u64, u32, u32, u32, ctypes.POINTER(ctypes.c_void_p), _u64p,
                               ctypes.POINTER(_Stats)]),
            "or_build_buckets": (i32, [_u64p, u64, u32, u32, u32, _u64p, u32, _u64p, u64, _u64p,
                                       _u64p, u64, _u64p, _u64p, ctypes.POINTER(_Stats)]),
            "or_query": (i32, [_u8p, u64, _u64p, u64, _u64p]),
            "or_bucket_values": (i32, [_u8p, u64, u64, _u64p, u64, _u64p]),
            "or_bucket_record": (i32, [_u8p, u64, u64, _u64p, u64, _u64p]),
            "or_free": (None, [ctypes.c_void_p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p64(a):
    return a.ctypes.data_as(_u64p)


def _keys(keys) -> np.ndarray:
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    if k.ndim != 2 or k.shape[1] != 2:
        raise ValueError("keys must be an (n, 2) uint64 array of (w0, w1)")
    return k


# ---------------------------------------------------------------- primitives
def splitmix64(seed: int, count: int) -> np.ndarray:
    st = ctypes.c_uint64(seed)
    return np.array([lib().or_splitmix64_next(ctypes.byref(st)) for _ in range(count)], dtype=np.uint64)


def start_seed(depth: int) -> int:
    return int(lib().or_start_seed(depth))


def hash64(w1: int, x: int) -> int:
    return int(lib().or_hash(w1, x))


def remap(h: int, M: int) -> int:
    return int(lib().or_remap(h, M))


def bucket_of(w0: int, nb: int) -> int:
    return int(lib().or_bucket_of(w0, nb))


def num_buckets(n: int, b: int) -> int:
    return int(lib().or_num_buckets(n, b))


def fanouts(l: int):
    lo, up = ctypes.c_uint32(), ctypes.c_uint32()
    lib().or_fanouts(l, ctypes.byref(lo), ctypes.byref(up))
    return int(lo.value), int(up.value)


def children(m: int, l: int):
    out = (ctypes.c_uint32 * 64)()
    k = lib().or_children(m, l, out)
    if k < 0:
        raise OracleError(k, "children")
    return [int(out[i]) for i in range(k)]


def rot(x: int, r: int, m: int) -> int:
    return int(lib().or_rot(x, r, m))


def rotation_fit(a: int, b: int, na: int, nb: int, m: int) -> int:
    return int(lib().or_rotation_fit(a, b, na, nb, m))


LEAF_BRUTE, LEAF_BRUTE_NAIVE, LEAF_ROT, LEAF_ROT_NAIVE = 0, 1, 2, 3


def leaf_search(w1, is_b, depth: int, mode: int):
    """Return (value, early-exit evaluations) for one leaf."""
    w = np.ascontiguousarray(w1, dtype=np.uint64)
    b = np.ascontiguousarray(is_b, dtype=np.uint8)
    v, ee = ctypes.c_uint64(), ctypes.c_uint64(0)
    rc = lib().or_leaf_search(_p64(w), b.ctypes.data_as(_u8p), len(w), depth, mode, ctypes.byref(v),
                              ctypes.byref(ee))
    if rc:
        raise OracleError(rc, "leaf_search")
    return int(v.value), int(ee.value)


def split_search(w1, l: int, depth: int) -> int:
    w = np.ascontiguousarray(w1, dtype=np.uint64)
    s = ctypes.c_uint64()
    rc = lib().or_split_search(_p64(w), len(w), l, depth, ctypes.byref(s))
    if rc:
        raise OracleError(rc, "split_search")
    return int(s.value)


def tau(m: int, l: int) -> int:
    return int(lib().or_tau(m, l))


def tau_log2arg(m: int, l: int) -> float:
    return float(lib().or_tau_log2arg(m, l))


def preorder_sizes(m: int, l: int):
    cap = 2 * m + 2
    out = (ctypes.c_uint32 * cap)()
    cnt = ctypes.c_uint64()
    rc = lib().or_preorder_sizes(m, l, out, cap, ctypes.byref(cnt))
    if rc:
        raise OracleError(rc, "preorder_sizes")
    return [int(out[i]) for i in range(cnt.value)]


# ---------------------------------------------------------------- whole build
def build(keys, leaf_size: int, bucket_size: int, rotation: bool, naive: bool = False):
    """Return (serialised bytes, stats dict)."""
    k = _keys(keys)
    ptr, ln = ctypes.c_void_p(), ctypes.c_uint64()
    st = _Stats()
    flags = (FLAG_ROTATION if rotation else 0) | (FLAG_NAIVE if naive else 0)
    rc = lib().or_build(_p64(k), k.shape[0], leaf_size, bucket_size, flags, ctypes.byref(ptr),
                        ctypes.byref(ln), ctypes.byref(st))
    if rc:
        raise OracleError(rc, "build")
    try:
        data = ctypes.string_at(ptr.value, ln.value)
    finally:
        lib().or_free(ptr)
    return data, st.as_dict()


def build_buckets(keys, leaf_size: int, bucket_size: int, rotation: bool, buckets):
    """Build only the selected buckets of a full key set.

    Returns (list of (bucket, size, values, record_words, record_bits), stats).
    """
    k = _keys(keys)
    sel = np.ascontiguousarray(buckets, dtype=np.uint64)
    ns = len(sel)
    vcap = 2 * 8192 * max(ns, 1)
    vals = np.zeros(vcap, dtype=np.uint64)
    counts = np.zeros(max(ns, 1), dtype=np.uint64)
    wcap = 1024 * max(ns, 1)
    grw = np.zeros(wcap, dtype=np.uint64)
    grlen = np.zeros(max(ns, 1), dtype=np.uint64)
    sizes = np.zeros(max(ns, 1), dtype=np.uint64)
    st = _Stats()
    rc = lib().or_build_buckets(_p64(k), k.shape[0], leaf_size, bucket_size,
                                FLAG_ROTATION if rotation else 0, _p64(sel), ns, _p64(vals), vcap,
                                _p64(counts), _p64(grw), wcap, _p64(grlen), _p64(sizes),
                                ctypes.byref(st))
    if rc:
        raise OracleError(rc, "build_buckets")
    out, vo, wo = [], 0, 0
    for i in range(ns):
        c = int(counts[i])
        nw = (int(grlen[i]) + 63) // 64
        out.append((int(sel[i]), int(sizes[i]), vals[vo:vo + c].copy(), grw[wo:wo + nw].copy(),
                    int(grlen[i])))
        vo += c
        wo += nw
    return out, st.as_dict()


def query(data: bytes, keys) -> np.ndarray:
    k = _keys(keys)
    buf = np.frombuffer(data, dtype=np.uint8).copy()
    out = np.zeros(k.shape[0], dtype=np.uint64)
    rc = lib().or_query(buf.ctypes.data_as(_u8p), len(buf), _p64(k), k.shape[0], _p64(out))
    if rc:
        raise OracleError(rc, "query")
    return out


def bucket_values(data: bytes, bucket: int) -> np.ndarray:
    buf = np.frombuffer(data, dtype=np.uint8).copy()
    cap = 65536
    out = np.zeros(cap, dtype=np.uint64)
    cnt = ctypes.c_uint64()
    rc = lib().or_bucket_values(buf.ctypes.data_as(_u8p), len(buf), bucket, _p64(out), cap,
                                ctypes.byref(cnt))
    if rc:
        raise OracleError(rc, "bucket_values")
    return out[:cnt.value].copy()


def bucket_record(data: bytes, bucket: int) -> tuple:
    """(record words, record bits) of one bucket, read out of serialised
    bytes and repacked from bit 0 (zero padded), comparable word for word
    with the records of build_buckets."""
    buf = np.frombuffer(data, dtype=np.uint8).copy()
    cap = 1 << 16
    out = np.zeros(cap, dtype=np.uint64)
    nbits = ctypes.c_uint64()
    rc = lib().or_bucket_record(buf.ctypes.data_as(_u8p), len(buf), bucket, _p64(out), cap,
                                ctypes.byref(nbits))
    if rc:
        raise OracleError(rc, "bucket_record")
    return out[:(nbits.value + 63) // 64].copy(), int(nbits.value)
