"""Autotuner of the seed-search schedule (rs_set_schedule).

The schedule decides how the persistent search kernel hands out attempts --
the chunk length of a split search relative to its expected length, how
soon idle workers join a long search, the grid size, the bucket-to-workgroup
mapping of small trees (one wave and 64 seeds a round, or four waves and
256), how a rotation is fitted -- and never what it finds: every schedule
yields the same structure.  Small launches (few nodes
per worker, e.g. one small request) are latency bound and want short chunks
that idle workers share early; large launches are throughput bound and want
few claims (little scheduling traffic) as long as that costs no time.

``tune()`` times the search kernel (HIP events around the launch, reported
in the build statistics) on synthetic key sets for every candidate setting
of each launch class; the cost of a setting is the sum over the sets of its
time relative to the defaults' (every set weighs the same), and among the
settings within ``tol`` of the cheapest it keeps the one with the longest
chunks; ``python -m
paper_2212_09562_amd.autotune`` prints it as JSON, and ``apply()`` installs
a schedule for the process.  The library's built-in defaults are this
tuner's result on an MI355X.
"""
from __future__ import annotations

import argparse
import json
import statistics

from . import keygen, recsplit

# (n, leaf size, bucket size) of the key sets each launch class is timed on
SMALL_SETS = [(10_000, 12, 1000), (30_000, 12, 1000), (20_000, 16, 2000)]
LARGE_SETS = [(1_000_000, 12, 1000), (10_000_000, 12, 1000), (1_000_000, 8, 100),
              (1_000_000, 10, 500), (1_000_000, 16, 2000), (3_000_000, 16, 2000)]
SHIFTS = (10, 12, 13, 14, 15, 16, 63)
HELP_AFTER = (1, 4, 16, 64)
INLINE_TAU = (0, 10, 13, 16, 20)
BUCKET_LEAF = (0, 8, 10, 12)
# bucket-to-workgroup mapping in whole-bucket mode: 0 = four waves share a
# bucket (256 seeds per round), 1 = one wave per bucket (64 seeds per round)
BUCKET_WAVE = (0, 1)
# rotation leaves: 0 = the wave tests every rotation, 1 = two table lookups
ROTATION_LOOKUP = (0, 1)


def _time_sets(sets, keys, reps, ref=None):
    """Median search time of each set; with ``ref`` (times of a reference
    schedule) the sum of the ratios, so every set weighs the same."""
    times = []
    for (n, l, b), k in zip(sets, keys):
        ms = []
        for _ in range(reps):
            f = recsplit.build(k, l, b, True)
            ms.append(f.stats()["ms_search"])
            f.free()
        times.append(statistics.median(ms))
    if ref is None:
        return times
    return sum(t / r for t, r in zip(times, ref))


def tune(small_sets=SMALL_SETS, large_sets=LARGE_SETS, shifts=SHIFTS, help_after=HELP_AFTER,
         inline_tau=INLINE_TAU, bucket_leaf=BUCKET_LEAF, bucket_wave=BUCKET_WAVE,
         rotation_lookup=ROTATION_LOOKUP, reps=3, seed=11, tol=0.01, log=None):
    """Per launch class: the fastest (chunk_shift, help_after), then the
    fastest inline_leaf_tau with those; then, on the large sets, the
    whole-bucket threshold (the smallest within tol of the fastest), the
    bucket-to-workgroup mapping (seeds per wave and round) and the rotation
    test (wave or lookup tables), each kept at its default unless another
    value is faster by more than tol.  Returns the schedule dict and the
    timing table."""
    import torch

    base = recsplit.set_schedule(None)
    keys = {id(s): [keygen.fingerprints_torch(n, seed + i, "cuda") for i, (n, _, _) in enumerate(s)]
            for s in (small_sets, large_sets)}
    torch.cuda.synchronize()
    table = {}
    best = dict(base)
    try:
        for cls, sets in (("small", small_sets), ("large", large_sets)):
            ks = keys[id(sets)]
            # force every set into this class
            force = {"small_tasks_per_worker": 1 << 30} if cls == "small" else {
                "small_tasks_per_worker": 1}
            _time_sets(sets, ks, 1)  # warm-up
            recsplit.set_schedule(base, **force)
            ref = _time_sets(sets, ks, reps)
            if log:
                log(f"{cls} reference (defaults): " + ", ".join(f"{t:.3f}" for t in ref) + " ms")
            results = []
            for r in shifts:
                for h in help_after:
                    recsplit.set_schedule(base, **force, **{f"chunk_shift_{cls}": r,
                                                            f"help_after_{cls}": h})
                    t = _time_sets(sets, ks, reps, ref)
                    results.append((t, r, h))
                    if log:
                        log(f"{cls} chunk_shift={r} help_after={h}: {t:.4f}")
            results.sort()
            table[cls] = [{"cost": t, "chunk_shift": r, "help_after": h} for t, r, h in results]
            near = [x for x in results if x[0] <= results[0][0] * (1.0 + tol)]
            _, r, h = min(near, key=lambda x: (x[1], -x[2]))
            best[f"chunk_shift_{cls}"] = r
            best[f"help_after_{cls}"] = h
            # then the leaf inlining threshold with those
            results = []
            for it in inline_tau:
                recsplit.set_schedule(best, **force, **{f"inline_leaf_tau_{cls}": it})
                t = _time_sets(sets, ks, reps, ref)
                results.append((t, it))
                if log:
                    log(f"{cls} inline_leaf_tau={it}: {t:.4f}")
            results.sort()
            table[cls + "_inline"] = [{"cost": t, "inline_leaf_tau": it} for t, it in results]
            table[cls + "_reference_ms"] = ref
            best[f"inline_leaf_tau_{cls}"] = results[0][1]
            if cls == "large":
                results = []
                for bl in bucket_leaf:
                    recsplit.set_schedule(best, **force, bucket_mode_max_leaf=bl)
                    t = _time_sets(sets, ks, reps, ref)
                    results.append((t, bl))
                    if log:
                        log(f"{cls} bucket_mode_max_leaf={bl}: {t:.4f}")
                table["bucket_mode"] = [{"cost": t, "bucket_mode_max_leaf": bl} for t, bl in results]
                low = min(t for t, _ in results)
                best["bucket_mode_max_leaf"] = min(bl for t, bl in results if t <= low * (1.0 + tol))
                for name, values in (("bucket_wave", bucket_wave),
                                     ("rotation_lookup", rotation_lookup)):
                    results = []
                    for v in values:
                        recsplit.set_schedule(best, **force, **{name: v})
                        t = _time_sets(sets, ks, reps, ref)
                        results.append((t, v))
                        if log:
                            log(f"{cls} {name}={v}: {t:.4f}")
                    table[name] = [{"cost": t, name: v} for t, v in results]
                    at_default = [t for t, v in results if v == base[name]]
                    low_t, low_v = min(results)
                    if not at_default or low_t < at_default[0] * (1.0 - tol):
                        best[name] = low_v
    finally:
        recsplit.set_schedule(None)
    return best, table


def apply(schedule: dict) -> dict:
    """Install a schedule for this process."""
    return recsplit.set_schedule(None, **schedule) if schedule else recsplit.set_schedule(None)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", help="write the schedule and timing table as JSON")
    args = ap.parse_args()
    best, table = tune(reps=args.reps, log=lambda s: print(s, flush=True))
    out = {"schedule": best, "timings_ms": table, "defaults": recsplit.get_schedule()}
    text = json.dumps(out, indent=1)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text + "\n")
    print(json.dumps({"schedule": best}), flush=True)


if __name__ == "__main__":
    main()
