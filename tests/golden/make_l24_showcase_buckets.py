"""Writes tests/golden/l24_b2000_n5e6_buckets.txt: the oracle's node values and
Golomb-Rice records of three buckets of the paper's most space-efficient
configuration (tab:showcaseOverall: l = 24, b = 2000, rotation fitting,
n = 5 million random 128-bit keys), on the key set the GPU build of that
configuration uses (keygen.fingerprints(5_000_000, 55)).  Each bucket costs
the oracle an hour or more on one core (55 to 89 minutes for these three), so
the check of the GPU build reads these stored results.

Only the oracle and the seeded key generator are called, one
single-threaded oracle process per bucket:

    python tests/golden/make_l24_showcase_buckets.py
"""
from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "l24_b2000_n5e6_buckets.txt")
N, L, B, SEED = 5_000_000, 24, 2000, 55
BUCKETS = [0, 1250, 2499]


def main():
    from oracle import shards
    from paper_2212_09562_amd import keygen

    keys = keygen.fingerprints(N, SEED)
    t0 = time.perf_counter()
    res, runs = shards.build_buckets_parallel(keys, L, B, True, BUCKETS, procs=len(BUCKETS))
    with open(OUT, "w") as f:
        f.write("# Oracle results for buckets of keygen.fingerprints(5000000, 55) at l = 24,\n"
                "# b = 2000, rotation fitting (make_l24_showcase_buckets.py).  Per bucket three\n"
                "# lines: 'bucket size record_bits', the record words (hex), and the node\n"
                "# values in preorder (decimal).\n")
        for j in BUCKETS:
            size, vals, words, bits = res[j]
            f.write(f"{j} {size} {bits}\n")
            f.write(" ".join(f"{int(w):016x}" for w in words) + "\n")
            f.write(" ".join(str(int(v)) for v in vals) + "\n")
    for r in runs:
        print(f"buckets {r['buckets']}: {r['seconds']:.0f} s, {r['evals']:.3e} evaluations")
    print(f"wrote {OUT} in {time.perf_counter() - t0:.0f} s")


if __name__ == "__main__":
    main()
