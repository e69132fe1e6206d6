"""GPU: many key sets in one persistent launch (rs_build_batch).

Every job's result must be the same bytes as its solo build and as the
oracle's; a job that fails (duplicate keys, arguments out of range) reports
its own code and leaves the others untouched.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from oracle import shards
from paper_2212_09562_amd import keygen

pytestmark = pytest.mark.gpu


def rs():
    from paper_2212_09562_amd import recsplit

    return recsplit


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _bucket_sizes(keys, nb):
    """Keys per bucket, bucket = floor(w0 * nb / 2^64) from 32-bit halves
    (exact for nb < 2^31); used only to pick buckets for the oracle, which
    reports each bucket's size itself."""
    w0 = keys[:, 0]
    hi, lo = w0 >> np.uint64(32), w0 & np.uint64(0xFFFFFFFF)
    nbu = np.uint64(nb)
    bucket = (hi * nbu + ((lo * nbu) >> np.uint64(32))) >> np.uint64(32)
    return np.bincount(bucket.astype(np.int64), minlength=nb)


def test_mixed_batch_matches_solo_and_oracle():
    import torch

    _case("mixed batch of 9 jobs")
    specs = [(5000, 8, 100, True), (0, 8, 100, True), (1, 5, 7, False), (20000, 12, 500, True),
             (3000, 4, 30, False), (7000, 6, 1, True), (12000, 8, 4096, True), (4000, 16, 2000, True),
             (2500, 3, 50, True)]
    jobs, wants = [], []
    for i, (n, l, b, rot) in enumerate(specs):
        keys = keygen.fingerprints(n, 700 + i)
        dev = i % 2 == 1
        jobs.append({"keys": torch.from_numpy(keys.view(np.int64)).cuda() if dev else keys,
                     "leaf_size": l, "bucket_size": b, "rotation": rot, "host": keys})
        wants.append(oracle.build(keys, l, b, rot)[0])
    # a duplicate and a bad argument in the middle of the batch
    dup = keygen.fingerprints(3000, 799)
    dup[3, 1] = dup[4, 1]
    dup[3, 0] = dup[4, 0] ^ np.uint64(1)
    jobs.insert(4, {"keys": dup, "leaf_size": 8, "bucket_size": 100, "rotation": True})
    jobs.insert(6, {"keys": keygen.fingerprints(10, 798), "leaf_size": 30, "bucket_size": 100})
    outs, st = rs().build_batch(jobs)
    assert st[4] == -2 and outs[4] is None
    assert st[6] == -1 and outs[6] is None
    k = 0
    for i, j in enumerate(jobs):
        if i in (4, 6):
            continue
        assert st[i] == 0, (i, st[i])
        got = outs[i].serialize()
        assert got == wants[k], i
        solo = rs().build(j["host"], j["leaf_size"], j["bucket_size"], j["rotation"]).serialize()
        assert got == solo
        r = outs[i].query(j["host"])
        assert np.array_equal(r, oracle.query(wants[k], j["host"]))
        k += 1


def test_batched_configuration_same_as_solo():
    """The 64-set batch (sizes log-uniform in [10^3, 10^6], l in {8,12,16}, b in
    {100,500,2000}, seed 4): every set's bytes equal its solo build, the ranks of
    every set form a permutation, and the oracle agrees on the small sets and,
    bucket by bucket (node values and Golomb-Rice records), on the largest
    bucket of every large set and the first and last of most of them."""
    import torch

    jobs = keygen.batched_jobs(64, seed=4)
    _case(f"64-job batch, {sum(j['n'] for j in jobs)} keys")
    batch = [{"keys": torch.from_numpy(j["keys"].view(np.int64)).cuda(), "leaf_size": j["leaf_size"],
              "bucket_size": j["bucket_size"], "keep_values": True} for j in jobs]
    outs, st = rs().build_batch(batch)
    assert all(s == 0 for s in st), st
    checks = []  # (set, buckets) the oracle rebuilds from the large sets
    for i, j in enumerate(jobs):
        data = outs[i].serialize()
        solo = rs().build(batch[i]["keys"], j["leaf_size"], j["bucket_size"], True).serialize()
        assert data == solo, i
        r = outs[i].query(batch[i]["keys"])
        assert torch.equal(torch.sort(r)[0], torch.arange(j["n"], device=r.device, dtype=r.dtype))
        cheap = (j["leaf_size"] == 8 and j["n"] <= 300000) or \
            (j["leaf_size"] == 12 and j["n"] <= 20000) or j["n"] <= 2000
        if cheap:
            assert data == oracle.build(j["keys"], j["leaf_size"], j["bucket_size"], True)[0], i
        else:
            # the largest bucket of every large set (one bucket of the l = 16,
            # b = 2000 sets, whose buckets cost the oracle seconds each), and
            # the first and last of the others
            nb = oracle.num_buckets(j["n"], j["bucket_size"])
            sizes = _bucket_sizes(j["keys"], nb)
            sel = {int(np.argmax(sizes))}
            if not (j["leaf_size"] == 16 and j["bucket_size"] == 2000):
                sel |= {0, nb - 1}
            checks.append((i, sorted(sel)))
    _case(f"oracle on {sum(len(c[1]) for c in checks)} buckets of {len(checks)} large sets")

    def rebuild(check):
        i, sel = check
        j = jobs[i]
        res, _ = shards.build_buckets_parallel(j["keys"], j["leaf_size"], j["bucket_size"], True,
                                               sel, procs=len(sel))
        return i, res

    with ThreadPoolExecutor(max_workers=max(1, shards.host_cores() // 2)) as ex:
        done = list(ex.map(rebuild, checks))
    assert any(jobs[i]["leaf_size"] == 16 and jobs[i]["bucket_size"] == 2000 for i, _ in done)
    for i, res in done:
        data = outs[i].serialize()
        for bk, (size, vals, words, nbits) in res.items():
            assert size == _bucket_sizes(jobs[i]["keys"], outs[i].stats()["nb"])[bk], (i, bk)
            assert np.array_equal(outs[i].node_values(bk), vals), (i, bk)
            gw, gb = oracle.bucket_record(data, bk)
            assert gb == nbits and np.array_equal(gw, words), (i, bk)


def test_autotuner_runs_and_leaves_defaults():
    from paper_2212_09562_amd import autotune

    _case("autotune on tiny sets")
    before = rs().get_schedule()
    best, table = autotune.tune(small_sets=[(5000, 12, 1000)], large_sets=[(20000, 8, 100)],
                                shifts=(8, 63), help_after=(1, 2), inline_tau=(0, 16),
                                bucket_leaf=(0, 8), reps=1)
    assert len(table["bucket_wave"]) == 2 and len(table["rotation_lookup"]) == 2
    assert best["bucket_wave"] in (0, 1) and best["rotation_lookup"] in (0, 1)
    assert rs().get_schedule() == before
    assert best["chunk_shift_small"] in (8, 63) and best["help_after_large"] in (1, 2)
    assert len(table["small"]) == 4 and len(table["large"]) == 4
    keys = keygen.fingerprints(20000, 5)
    want = rs().build(keys, 8, 100, True).serialize()
    try:
        autotune.apply(best)
        assert rs().build(keys, 8, 100, True).serialize() == want
    finally:
        rs().set_schedule(None)
