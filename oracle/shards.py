"""The oracle over many buckets of one key set, one process per shard -- TEST
INFRASTRUCTURE ONLY.

Only ``tests/`` and the ``cpu_baseline`` leg of ``bench.py`` use this module.
The oracle itself stays single-threaded and unchanged: every shard is a
separate Python process that loads the oracle and runs
``oracle.build_buckets`` (bucket the whole key set, then build the trees of
its buckets) on its share of the selected buckets.  Nothing here computes
any part of the method.
"""
from __future__ import annotations

import json
import os
import subprocess
import sys
import tempfile
import time

import numpy as np

_ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

_SHARD = """
import json, sys, time
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
keys = np.load(sys.argv[2], mmap_mode="r")
out = sys.argv[3]
l, b, rot = int(sys.argv[4]), int(sys.argv[5]), bool(int(sys.argv[6]))
sel = [int(x) for x in sys.argv[7].split(",")]
t0 = time.perf_counter()
recs, st = oracle.build_buckets(np.ascontiguousarray(keys), l, b, rot, sel)
dt = time.perf_counter() - t0
arrs = {}
for (j, size, vals, words, bits) in recs:
    arrs[f"v{j}"] = vals
    arrs[f"w{j}"] = words
    arrs[f"m{j}"] = np.array([size, bits], dtype=np.uint64)
np.savez(out, **arrs)
print(json.dumps({"seconds": dt, "keys": sum(r[1] for r in recs),
                  "evals": st["evals_split"] + st["evals_leaf"], "buckets": sel}))
"""


def host_cores(limit: int = 16) -> int:
    """Cores this process may run on, at most `limit`."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(limit, n))


def build_buckets_parallel(keys, leaf_size: int, bucket_size: int, rotation: bool, buckets,
                           procs: int = 0, contiguous: bool = False):
    """Oracle node values and Golomb-Rice records of the selected buckets of
    the key set `keys` ((n, 2) uint64), computed by `procs` single-threaded
    oracle processes (0: the host's cores, at most 16).

    Buckets are dealt round-robin to the processes, or in contiguous runs
    with contiguous=True.  Returns (results, shards): results maps bucket ->
    (size, values, record words, record bits); shards lists, per process, its
    wall time inside the oracle, its keys, its hash evaluations (the paper's
    count) and its buckets."""
    sel = [int(j) for j in buckets]
    if not sel:
        return {}, []
    procs = min(len(sel), procs or host_cores())
    if contiguous:
        per = -(-len(sel) // procs)
        groups = [sel[i * per:(i + 1) * per] for i in range(procs)]
    else:
        groups = [sel[i::procs] for i in range(procs)]
    groups = [g for g in groups if g]
    results, shards = {}, []
    with tempfile.TemporaryDirectory() as tmp:
        path = os.path.join(tmp, "keys.npy")
        np.save(path, np.ascontiguousarray(keys, dtype=np.uint64))
        env = dict(os.environ, OMP_NUM_THREADS="1")
        running = []
        for i, g in enumerate(groups):
            out = os.path.join(tmp, f"shard{i}.npz")
            cmd = [sys.executable, "-c", _SHARD, _ROOT, path, out, str(leaf_size),
                   str(bucket_size), "1" if rotation else "0", ",".join(str(j) for j in g)]
            running.append((subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True, env=env), out))
        for p, out in running:
            text = p.communicate()[0]
            if p.returncode:
                raise RuntimeError(f"oracle shard failed with status {p.returncode}")
            shards.append(json.loads(text.strip().splitlines()[-1]))
            with np.load(out) as z:
                for j in shards[-1]["buckets"]:
                    size, bits = (int(x) for x in z[f"m{j}"])
                    results[j] = (size, z[f"v{j}"].copy(), z[f"w{j}"].copy(), bits)
    return results, shards


def timed_shards(keys, leaf_size: int, bucket_size: int, rotation: bool, per_proc: int,
                 procs: int):
    """The first per_proc * procs buckets, per_proc contiguous buckets per
    process; returns (results, shards, wall seconds including start-up)."""
    t0 = time.perf_counter()
    res, shards = build_buckets_parallel(keys, leaf_size, bucket_size, rotation,
                                         range(per_proc * procs), procs, contiguous=True)
    return res, shards, time.perf_counter() - t0
