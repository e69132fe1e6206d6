"""Seeded synthetic inputs: uniform random 128-bit fingerprints.

The paper measures its own configurations on random 128-bit integers used
directly as the master hash code (Sec. 6, "Experimental Setup"); these
generators stand in for that input.  This module holds no arithmetic of the
construction itself: it only draws keys (and, for the batched and served
workloads, job parameters), so both the GPU library and the CPU oracle are
fed from it.

Keys come from SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): output i of the
stream seeded with s is mix(s + (i + 1) * 0x9E3779B97F4A7C15).  Key j is the
pair (w0, w1) = (output 2j, output 2j + 1).  A key equal (in all 128 bits) to
an earlier one is dropped and the stream continues, so the set is duplicate
free and the same for every caller.
"""
from __future__ import annotations

import math

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def splitmix64_stream(seed: int, start: int, count: int) -> np.ndarray:
    """Outputs start .. start+count-1 (0-based) of SplitMix64 seeded with ``seed``."""
    with np.errstate(over="ignore"):
        idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        state = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * GOLDEN
        return _mix(state)


def fingerprints(n: int, seed: int) -> np.ndarray:
    """n distinct 128-bit fingerprints as an (n, 2) uint64 array of (w0, w1)."""
    if n == 0:
        return np.zeros((0, 2), dtype=np.uint64)
    out = splitmix64_stream(seed, 0, 2 * n).reshape(n, 2)
    drawn = 2 * n
    while True:
        view = out.view(np.dtype((np.void, 16))).ravel()
        _, first = np.unique(view, return_index=True)
        if len(first) == n:
            return out
        keep = np.sort(first)
        missing = n - len(keep)
        extra = splitmix64_stream(seed, drawn, 2 * missing).reshape(missing, 2)
        drawn += 2 * missing
        out = np.concatenate([out[keep], extra])


def _as_signed(x: int) -> int:
    x &= 0xFFFFFFFFFFFFFFFF
    return x - (1 << 64) if x >> 63 else x


def _lsr(z, k: int):
    """Logical right shift of int64 tensors (torch's >> is arithmetic)."""
    return (z >> k) & ((1 << (64 - k)) - 1)


def fingerprints_torch(n: int, seed: int, device="cuda"):
    """The keys of ``fingerprints(n, seed)`` drawn with torch on ``device``, as
    an (n, 2) int64 tensor holding the same 64-bit words (two's complement
    int64 arithmetic wraps exactly like uint64).  If two drawn keys share w0
    the exact host procedure (with its redraws) is used instead."""
    import torch

    if n == 0:
        return torch.zeros((0, 2), dtype=torch.int64, device=device)
    idx = torch.arange(1, 2 * n + 1, dtype=torch.int64, device=device)
    z = idx * _as_signed(int(GOLDEN)) + _as_signed(seed)
    z = z ^ _lsr(z, 30)
    z = z * _as_signed(int(_M1))
    z = z ^ _lsr(z, 27)
    z = z * _as_signed(int(_M2))
    z = z ^ _lsr(z, 31)
    out = z.view(n, 2)
    w0 = torch.sort(out[:, 0])[0]
    if n > 1 and bool((w0[1:] == w0[:-1]).any()):
        return torch.from_numpy(fingerprints(n, seed).view(np.int64)).to(device)
    return out


def _unit(x: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1) from the top 53 bits."""
    return (x >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def batched_jobs(count: int = 64, seed: int = 4, lo: float = 1e3, hi: float = 1e6,
                 leaf_sizes=(8, 12, 16), bucket_sizes=(100, 500, 2000), draw=None):
    """Independent key-set jobs: size log-uniform in [lo, hi], leaf and bucket
    sizes each picked uniformly from the given sets.  Parameters are drawn
    first from one SplitMix64 stream, then every job's keys come from its own
    stream seeded with (seed << 32) + job index, through ``draw(n, seed)``
    (default ``fingerprints``; ``fingerprints_torch`` gives the same keys on a
    device)."""
    draw = draw or fingerprints
    draws = splitmix64_stream(seed, 0, 3 * count).reshape(count, 3)
    u = _unit(draws[:, 0])
    sizes = np.floor(10.0 ** (math.log10(lo) + (math.log10(hi) - math.log10(lo)) * u)).astype(np.int64)
    jobs = []
    for j in range(count):
        n = int(sizes[j])
        l = int(leaf_sizes[int(draws[j, 1] % np.uint64(len(leaf_sizes)))])
        b = int(bucket_sizes[int(draws[j, 2] % np.uint64(len(bucket_sizes)))])
        jobs.append({"n": n, "leaf_size": l, "bucket_size": b,
                     "keys": draw(n, (seed << 32) + j)})
    return jobs


def served_requests(count: int, seed: int = 5, rate: float = 20.0, lo: float = 1e4, hi: float = 1e7):
    """Arrival times (Poisson process of the given rate per second) and sizes
    (log-uniform in [lo, hi]) of construction requests; request i's keys come
    from the stream seeded with (seed << 32) + i (drawn lazily by the caller
    through ``fingerprints``)."""
    draws = splitmix64_stream(seed, 0, 2 * count).reshape(count, 2)
    gaps = -np.log1p(-_unit(draws[:, 0])) / rate
    arrivals = np.cumsum(gaps)
    u = _unit(draws[:, 1])
    sizes = np.floor(10.0 ** (math.log10(lo) + (math.log10(hi) - math.log10(lo)) * u)).astype(np.int64)
    return [{"arrival": float(arrivals[i]), "n": int(sizes[i]), "seed": (seed << 32) + i}
            for i in range(count)]
