"""Writes tests/golden/large_leaf_sets.txt: the oracle's serialised structure
of small key sets at the space-efficient leaf sizes 19 to 24 (Sec. 6,
tab:showcaseOverall uses l = 18 and 24), each a bucket large enough for a
fanout-2 root, upper and lower splits and full leaves (Sec. 2.2 "Splitting
Trees").  The oracle needs minutes to an hour per set at these leaf sizes, so
the GPU tests compare with these stored bytes instead of rebuilding them.

Only the oracle and the seeded key generator are called.  Each set is built
by its own single-threaded oracle process, all sets at once:

    python tests/golden/make_large_leaf_sets.py
"""
from __future__ import annotations

import json
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
OUT = os.path.join(HERE, "large_leaf_sets.txt")

# (n, leaf size, bucket size, rotation fitting, key seed).  One bucket each
# (n <= b), above the upper aggregation unit where a fanout-2 root is wanted:
# l=19: ua 760; l=20: ua 960 (b = 500 gives two buckets of upper splits);
# l=21: ua 1008; l=22: ua 1188; l=24: ua 1296.
SETS = [
    (800, 19, 800, True, 1901),
    (1000, 20, 500, True, 2001),
    (600, 20, 600, False, 2002),
    (1100, 21, 1100, True, 2101),
    (1300, 22, 1300, True, 2201),
    (2000, 24, 2000, True, 2401),
]

_ONE = """
import json, sys, time
sys.path.insert(0, sys.argv[1])
import oracle
from paper_2212_09562_amd import keygen
n, l, b, rot, seed = (int(x) for x in sys.argv[2:7])
keys = keygen.fingerprints(n, seed)
t0 = time.perf_counter()
data, st = oracle.build(keys, l, b, bool(rot))
print(json.dumps({"hex": data.hex(), "seconds": time.perf_counter() - t0,
                  "evals": st["evals_split"] + st["evals_leaf"]}))
"""


def main():
    procs = []
    for n, l, b, rot, seed in SETS:
        cmd = [sys.executable, "-c", _ONE, ROOT, str(n), str(l), str(b), str(int(rot)), str(seed)]
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, text=True,
                                      env=dict(os.environ, OMP_NUM_THREADS="1")))
    rows = []
    for (n, l, b, rot, seed), p in zip(SETS, procs):
        text = p.communicate()[0]
        if p.returncode:
            raise SystemExit(f"oracle failed on n={n} l={l} b={b}: status {p.returncode}")
        r = json.loads(text.strip().splitlines()[-1])
        print(f"n={n} l={l} b={b} rot={rot}: {r['seconds']:.0f} s, {r['evals']:.3e} evaluations",
              flush=True)
        rows.append(f"{n} {l} {b} {int(rot)} {seed} {r['hex']}")
    with open(OUT, "w") as f:
        f.write("# Serialised structures built by the oracle (make_large_leaf_sets.py).\n"
                "# Keys: keygen.fingerprints(n, seed).  Columns: n  leaf_size  bucket_size\n"
                "# rotation  seed  bytes (hex)\n")
        for row in rows:
            f.write(row + "\n")
    print(f"wrote {OUT} at {time.strftime('%H:%M:%S')}")


if __name__ == "__main__":
    main()
