"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Bit-exact is the bar everywhere (construction is integer work): the same
serialised bytes, the same node values, the same query results -- also for
keys outside the set, since both sides evaluate the same function.  Small
cases cover several buckets, ragged last leaves, singleton children, empty
and one-key sets, l from 2 to 16 and b from 1 to 4096; the benchmark
configurations follow at full size (the l = 16, b = 2000 build on a sample
of buckets the oracle can afford).
"""
import math
import os

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


def _first_diff_bucket(f, data, nb):
    for j in range(nb):
        a = f.node_values(j)
        b = oracle.bucket_values(data, j)
        if not np.array_equal(a, b):
            return j, a, b
    return None


def _check_parity(keys, l, b, rot, tag=""):
    _case(f"n={len(keys)} l={l} b={b} rot={rot} {tag}")
    want, st = oracle.build(keys, l, b, rot)
    f = rs().build(keys, l, b, rot, keep_values=True)
    got = f.serialize()
    if got != want:
        nb = oracle.num_buckets(len(keys), b)
        d = _first_diff_bucket(f, want, nb)
        raise AssertionError(f"bytes differ ({len(got)} vs {len(want)}); first bucket with other "
                             f"values: {d}")
    gs = f.stats()
    assert gs["useful_evals_split"] == st["evals_split"]
    assert gs["useful_evals_leaf"] == st["evals_leaf"]
    assert gs["split_nodes"] == st["nodes_split"] and gs["leaf_nodes"] == st["nodes_leaf"]
    r = f.query(keys)
    assert np.array_equal(np.sort(r), np.arange(len(keys), dtype=np.uint64))
    assert np.array_equal(r, oracle.query(want, keys))
    return f, want


SMALL = [
    (0, 8, 100, True), (1, 8, 100, True), (2, 8, 2, False), (3, 2, 1, True), (17, 5, 7, False),
    (1000, 8, 100, False), (1000, 8, 100, True), (3000, 2, 7, True), (3000, 3, 50, False),
    (4000, 4, 30, True), (5000, 5, 100, True), (5000, 7, 300, False), (6000, 10, 500, True),
    (8000, 12, 1000, True), (3000, 12, 60, False), (20000, 8, 100, True), (20000, 6, 1, True),
]


@pytest.mark.parametrize("n,l,b,rot", SMALL)
def test_small_parity(n, l, b, rot):
    _check_parity(keygen.fingerprints(n, 100 + n + l), l, b, rot)


def test_non_members_match_oracle():
    keys = keygen.fingerprints(30000, 9)
    _case("non-member queries, n=30000 l=8 b=100")
    f, data = _check_parity(keys, 8, 100, True)
    other = keygen.fingerprints(20000, 10)
    assert np.array_equal(f.query(other), oracle.query(data, other))


def test_query_through_elias_fano_selects():
    """A query reads the bucket offsets C_j, C_j+1 and the record offset P_j
    from a decoded copy of both Elias-Fano sequences when that copy is no
    larger than the structure (or 1 MiB), else by select on the sequences
    themselves.  80 000 buckets of 5 keys take the select path (1.28 MB of
    offsets against 0.16 MB of structure)."""
    keys = keygen.fingerprints(400_000, 31)
    f, data = _check_parity(keys, 5, 5, True, "select path")
    other = keygen.fingerprints(50_000, 32)
    assert np.array_equal(f.query(other), oracle.query(data, other))


def test_device_keys_and_determinism():
    import torch

    keys = keygen.fingerprints(50000, 12)
    _case("device keys, repeat, other launch shapes: n=50000 l=8 b=100")
    want, _ = oracle.build(keys, 8, 100, True)
    dk = torch.from_numpy(keys.view(np.int64)).cuda()
    f = rs().build(dk, 8, 100, True)
    assert f.serialize() == want
    r = f.query(dk)
    torch.cuda.synchronize()
    assert np.array_equal(r.cpu().numpy().view(np.uint64), oracle.query(want, keys))
    # a shuffled copy and other chunk schedules give the same bytes
    perm = np.random.default_rng(0).permutation(len(keys))
    k16 = keys[:2500]
    want16 = oracle.build(k16, 16, 2000, True)[0]
    try:
        for sched in ({"chunk_shift_small": 3, "chunk_shift_large": 3, "help_after_small": 1,
                       "help_after_large": 1, "max_workers": 37, "inline_leaf_tau_small": 0,
                       "inline_leaf_tau_large": 0},
                      {"chunk_shift_small": 0, "chunk_shift_large": 63, "help_after_small": 5,
                       "help_after_large": 1, "small_tasks_per_worker": 1000,
                       "inline_leaf_tau_small": 64, "inline_leaf_tau_large": 64},
                      {"small_tasks_per_worker": 1, "inline_leaf_tau_large": 9}):
            rs().set_schedule(None)
            rs().set_schedule(**sched)
            assert rs().build(keys[perm], 8, 100, True).serialize() == want
            assert rs().build(k16, 16, 2000, True).serialize() == want16
    finally:
        rs().set_schedule(None)
    assert rs().build(keys, 8, 100, True).serialize() == want


def test_device_keygen_matches_host():
    _case("keys drawn on the device equal the host draw")
    for n, seed in ((1, 0), (100_000, 3), (77_777, (5 << 32) + 9)):
        d = keygen.fingerprints_torch(n, seed, "cuda").cpu().numpy().view(np.uint64)
        assert np.array_equal(d, keygen.fingerprints(n, seed)), (n, seed)


BUCKET_MODE = [(5000, 8, 100, True), (5000, 8, 100, False), (3000, 2, 7, True), (4000, 4, 30, False),
               (20000, 12, 1000, True), (6000, 10, 60, True), (2000, 16, 20, True), (1500, 5, 1, True)]


@pytest.mark.parametrize("n,l,b,rot", BUCKET_MODE)
def test_whole_bucket_mode(n, l, b, rot):
    """One worker per bucket, the tree built in LDS (forced with a small
    grid), the worker four waves or one."""
    keys = keygen.fingerprints(n, 300 + n + l)
    try:
        for wave in (0, 1):
            rs().set_schedule(None)
            rs().set_schedule(max_workers=4, bucket_mode_max_leaf=24, bucket_wave=wave)
            _check_parity(keys, l, b, rot, f"whole-bucket workers, bucket_wave={wave}")
    finally:
        rs().set_schedule(None)


FILTERED = [(5000, 8, 100, True), (5000, 8, 100, False), (3000, 2, 7, True), (4000, 4, 30, False),
            (20000, 12, 1000, True), (3000, 12, 200, False), (2500, 16, 2000, True),
            (400, 18, 50, True), (1500, 5, 1, True)]


@pytest.mark.parametrize("n,l,b,rot", FILTERED)
def test_filtered_leaf_search(n, l, b, rot):
    """Every leaf of three or more keys through the staged early-exit search
    (leaf_filter_tau=1), alone or in claimed chunks that idle workers join
    (join_leaf_tau=1; with leaf_filter_tau=12 the shorter leaves are joined
    unfiltered), then none: the same bytes as the oracle."""
    keys = keygen.fingerprints(n, 500 + n + l)
    try:
        for filt, join in ((1, 0), (1, 1), (12, 1), (0, 0)):
            rs().set_schedule(None)
            # joining happens in small launches: make every launch small
            rs().set_schedule(leaf_filter_tau=filt, join_leaf_tau=join,
                              small_tasks_per_worker=1000)
            _check_parity(keys, l, b, rot, f"leaf_filter_tau={filt} join_leaf_tau={join}")
    finally:
        rs().set_schedule(None)


SPLIT_FILTERED = [(20000, 12, 1000, True), (6000, 16, 2000, True), (4000, 10, 500, False),
                  (3000, 8, 100, True), (2000, 18, 50, True), (5000, 6, 300, True),
                  (3000, 13, 777, True), (600, 20, 100, True), (150, 22, 150, True)]


@pytest.mark.parametrize("n,l,b,rot", SPLIT_FILTERED)
def test_filtered_split_search(n, l, b, rot):
    """Lower and upper split searches through the staged early-exit search
    (split_filter_tau=1; chunk_shift 0 makes chunks long enough for it early;
    at leaf sizes 20 and 22 the counter fields need more than 32 bits and the
    splits keep the plain rounds), with and without filtered leaves, then
    without: the oracle's bytes."""
    keys = keygen.fingerprints(n, 700 + n + l)
    try:
        for sched in ({"split_filter_tau": 1, "chunk_shift_small": 0, "chunk_shift_large": 0},
                      {"split_filter_tau": 1, "leaf_filter_tau": 1, "bucket_mode_max_leaf": 0},
                      {"split_filter_tau": 0, "leaf_filter_tau": 0}):
            rs().set_schedule(None)
            rs().set_schedule(**sched)
            _check_parity(keys, l, b, rot, str(sched))
    finally:
        rs().set_schedule(None)


LOOKUP = [(5000, 8, 100), (3000, 4, 30), (20000, 12, 1000), (6000, 10, 60), (2500, 16, 2000),
          (1500, 5, 1), (4000, 6, 7), (3000, 14, 500), (2000, 2, 3)]


@pytest.mark.parametrize("n,l,b", LOOKUP)
def test_rotation_lookup_tables(n, l, b):
    """Rotation-fitting leaves that find their rotation by table lookups
    (Sec. 4 "Lookup Tables"; rotation_lookup=1): in the plain kernel with
    node tasks, in whole-bucket workers, and with the filters on (whose
    kernel keeps the wave test): the oracle's bytes every time."""
    keys = keygen.fingerprints(n, 1100 + n + l)
    try:
        for sched in ({"rotation_lookup": 1, "bucket_mode_max_leaf": 0, "leaf_filter_tau": 0,
                       "split_filter_tau": 0},
                      {"rotation_lookup": 1, "max_workers": 4, "bucket_mode_max_leaf": 24},
                      {"rotation_lookup": 1, "max_workers": 4, "bucket_mode_max_leaf": 24,
                       "bucket_wave": 0},
                      {"rotation_lookup": 1}):
            rs().set_schedule(None)
            rs().set_schedule(**sched)
            _check_parity(keys, l, b, True, str(sched))
    finally:
        rs().set_schedule(None)


def test_early_exit_work_figures():
    """The early-exit work the library reports equals the closed form summed
    over the oracle's leaf values, and the per-size split table
    (rs_attempt_work, pinned on the CPU) summed over its split values."""
    from closed_forms import leaf_early_exit_evals

    for n, l, b, rot in ((20000, 12, 500, True), (20000, 8, 100, False), (4000, 16, 2000, True),
                         (1500, 18, 300, True)):
        keys = keygen.fingerprints(n, 41)
        _case(f"early-exit work n={n} l={l} b={b} rot={rot}")
        data, _ = oracle.build(keys, l, b, rot)
        f = rs().build(keys, l, b, rot)
        nb = oracle.num_buckets(len(keys), b)
        sizes = np.bincount([oracle.bucket_of(int(w0), nb) for w0 in keys[:, 0]], minlength=nb)
        want, want_split = 0.0, 0.0
        for j in range(nb):
            vals = oracle.bucket_values(data, j)
            ms = oracle.preorder_sizes(int(sizes[j]), l)
            assert len(ms) == len(vals)
            for m, v in zip(ms, vals):
                if m <= l:
                    failed = int(v) // m if rot else int(v)
                    want += failed * leaf_early_exit_evals(m, rot) + m
                else:
                    want_split += int(v) * rs().attempt_work(l, m) + m
        st = f.stats()
        assert st["early_exit_evals_leaf"] == pytest.approx(want, rel=2e-4), (l, b, rot)
        assert st["early_exit_evals_leaf"] < st["useful_evals_leaf"]
        assert st["early_exit_evals_split"] == pytest.approx(want_split, rel=1e-5), (l, b, rot)
        assert st["early_exit_evals_split"] <= st["useful_evals_split"]


def test_serialise_roundtrip_and_corruption():
    keys = keygen.fingerprints(10000, 13)
    _case("deserialise, n=10000 l=8 b=100")
    f = rs().build(keys, 8, 100, True)
    data = f.serialize()
    g = rs().deserialize(data)
    assert g.serialize() == data
    assert np.array_equal(g.query(keys), f.query(keys))
    bad = bytearray(data)
    bad[0] ^= 1
    with pytest.raises(rs().RecSplitError) as e:
        rs().deserialize(bytes(bad))
    assert e.value.code == -5
    with pytest.raises(rs().RecSplitError) as e:
        rs().deserialize(data[:-8])
    assert e.value.code == -5


def test_duplicates_and_bad_arguments():
    keys = keygen.fingerprints(2000, 14)
    _case("duplicate w1 in one bucket")
    dup = keys.copy()
    dup[5, 1] = dup[6, 1]
    dup[5, 0] = dup[6, 0] ^ np.uint64(1)
    with pytest.raises(rs().RecSplitError) as e:
        rs().build(dup, 8, 100, True)
    assert e.value.code == -2
    for l, b in ((1, 100), (25, 100), (8, 0), (8, 4097)):
        with pytest.raises(rs().RecSplitError) as e:
            rs().build(keys, l, b, True)
        assert e.value.code == -1
    # the library is still usable after the errors
    _check_parity(keys, 8, 100, True, "after errors")


def test_extreme_w1_values_and_their_duplicates():
    """Keys whose second word is 0 or 2^64 - 1 (the duplicate check pads each
    bucket's sorted w1 words with the latter): one in each of several buckets
    builds as the oracle does; two equal ones in one bucket are a duplicate."""
    n, b = 5000, 100
    keys = keygen.fingerprints(n, 23)
    nb = oracle.num_buckets(n, b)
    bucket = [(int(w) * nb) >> 64 for w in keys[:, 0]]
    first = {}
    for i, j in enumerate(bucket):
        first.setdefault(j, i)
    picks = list(first.values())[::5]
    keys[picks[0::2], 1] = 0
    keys[picks[1::2], 1] = np.uint64(0xFFFFFFFFFFFFFFFF)
    _check_parity(keys, 8, b, True, "w1 = 0 or 2^64-1 in %d buckets" % len(picks))
    for i in picks[:2]:
        k = next(t for t in range(n) if t != i and bucket[t] == bucket[i])
        dup = keys.copy()
        dup[k, 1] = dup[i, 1]
        _case("two keys with w1 = %#x in one bucket" % int(dup[i, 1]))
        with pytest.raises(rs().RecSplitError) as e:
            rs().build(dup, 8, b, True)
        assert e.value.code == -2


def test_stall_guard_stops_a_launch_and_the_library_recovers():
    """The bug guard on idle time, forced from the host with a 1 microsecond
    limit: the launch ends with RS_ERR_DEVICE instead of finishing, every
    worker exits, and the next build is exact."""
    keys = keygen.fingerprints(20000, 17)
    _case("stall guard at 1 us")
    try:
        rs().set_schedule(None)
        rs().set_schedule(stall_guard_us=1)
        with pytest.raises(rs().RecSplitError) as e:
            rs().build(keys, 12, 1000, True)
        assert e.value.code == -4
    finally:
        rs().set_schedule(None)
    _check_parity(keys, 12, 1000, True, "after a stopped launch")


def test_progress_lines(capfd):
    """RS_PROGRESS=<seconds>: while a search runs, the library prints the
    number of finished nodes to stderr at that interval.  The counts never
    decrease and never exceed the node total, and the structure is the same
    as without the lines."""
    keys = keygen.fingerprints_torch(1_000_000, 77, "cuda")
    _case("progress lines, l=20 b=100 n=1e6")
    ref = rs().build(keys, 20, 100, True).serialize()
    os.environ["RS_PROGRESS"] = "0.1"
    try:
        data = rs().build(keys, 20, 100, True).serialize()
    finally:
        del os.environ["RS_PROGRESS"]
    err = capfd.readouterr().err
    lines = [ln.split() for ln in err.splitlines() if ln.startswith("[rs progress]")]
    assert len(lines) >= 2, err
    done = [int(w[3]) for w in lines]
    total = {int(w[5]) for w in lines}
    assert len(total) == 1
    assert done == sorted(done) and done[-1] <= total.pop()
    assert data == ref


def _skewed(n, seed, nb, big):
    """n keys whose first `big` fall into bucket 0 of nb (w0 below 2^64/nb)."""
    keys = keygen.fingerprints(n, seed).copy()
    keys[:big, 0] >>= np.uint64(8)
    return keys


def test_bucket_beyond_the_first_duplicate_check():
    """The duplicate check's LDS is sized from the expected bucket size before
    the sizes are known; a far larger bucket (600 keys where b = 100) is
    checked after the first wait, with a second check sized to it."""
    n, b = 3000, 100
    keys = _skewed(n, 41, oracle.num_buckets(n, b), 600)
    _check_parity(keys, 8, b, True, "one bucket of 600+ keys")
    dup = keys.copy()
    dup[599] = dup[3]  # two equal keys in the large bucket
    with pytest.raises(rs().RecSplitError) as e:
        rs().build(dup, 8, b, True)
    assert e.value.code == -2


def test_largest_buckets():
    _case("b=4096, n=12000, l=8")
    _check_parity(keygen.fingerprints(12000, 15), 8, 4096, True)


@pytest.mark.parametrize("n,l,b,rot", [(2000, 18, 50, True), (150, 18, 50, False),
                                       (600, 20, 100, True), (30, 24, 30, True)])
def test_leaf_sizes_above_16(n, l, b, rot):
    """The space-efficient leaf sizes of Sec. 6 (l = 18, 20, 24) on sets the
    oracle can afford; l = 24 leaves need values above 2^32."""
    _check_parity(keygen.fingerprints(n, 910 + l + n), l, b, rot)


def _large_leaf_sets():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large_leaf_sets.txt")
    rows = []
    if not os.path.exists(path):  # written by tests/golden/make_large_leaf_sets.py
        return [pytest.param(0, 0, 0, True, 0, "", marks=pytest.mark.skip(reason=f"{path} missing"))]
    with open(path) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                n, l, b, rot, seed, hexbytes = line.split()
                rows.append((int(n), int(l), int(b), bool(int(rot)), int(seed), hexbytes))
    return rows


@pytest.mark.parametrize("n,l,b,rot,seed,hexbytes", _large_leaf_sets(),
                         ids=lambda v: str(v)[:12])
def test_large_leaf_sets_against_stored_oracle_bytes(n, l, b, rot, seed, hexbytes):
    """Leaf sizes 19 to 24 on buckets large enough for a fanout-2 root and
    upper and lower splits (the oracle needs minutes to an hour per set; its
    bytes are stored by tests/golden/make_large_leaf_sets.py): the default
    schedule (staged leaf and split searches, 64-bit split counters from
    l = 19 on), the staged split search forced onto every split, and neither
    filter all give the oracle's bytes."""
    want = bytes.fromhex(hexbytes)
    keys = keygen.fingerprints(n, seed)
    try:
        for sched in ({}, {"split_filter_tau": 1, "chunk_shift_small": 0, "chunk_shift_large": 0},
                      {"split_filter_tau": 0, "leaf_filter_tau": 0}):
            _case(f"stored oracle bytes n={n} l={l} b={b} rot={rot} {sched}")
            rs().set_schedule(None)
            rs().set_schedule(**sched)
            f = rs().build(keys, l, b, rot)
            assert f.serialize() == want, sched
            r = f.query(keys)
            assert np.array_equal(np.sort(r), np.arange(n, dtype=np.uint64))
            assert np.array_equal(r, oracle.query(want, keys))
    finally:
        rs().set_schedule(None)


def test_leaf16_two_buckets():
    _case("l=16 b=2000 n=4000 (two buckets)")
    _check_parity(keygen.fingerprints(4000, 16), 16, 2000, True)


@pytest.mark.parametrize("rot,seed,n", [(False, 1, 100000), (True, 2, 1000000)])
def test_configs_l8_b100_full(rot, seed, n):
    """Plain RecSplit on 10^5 keys and rotation fitting on 10^6 keys, l=8, b=100."""
    keys = keygen.fingerprints(n, seed)
    _check_parity(keys, 8, 100, rot, "full configuration")


def _record_bits(words, gr_off, start, nbits):
    out = np.zeros((nbits + 63) // 64, dtype=np.uint64)
    for i in range(len(out)):
        lo = start + 64 * i
        w, s = lo // 64, lo % 64
        v = int(words[gr_off + w]) >> s
        if s and gr_off + w + 1 < len(words):
            v |= int(words[gr_off + w + 1]) << (64 - s)
        take = min(64, nbits - 64 * i)
        out[i] = v & ((1 << take) - 1)
    return out


def _parse_offsets(data):
    """Bucket prefix sums C and record offsets P decoded from the bytes."""
    w = np.frombuffer(data, dtype=np.uint64)
    at = 5
    seqs = []
    for _ in range(2):
        N, U, L, lw, ub, uw = (int(x) for x in w[at:at + 6])
        lower = w[at + 6:at + 6 + lw]
        upper = w[at + 6 + lw:at + 6 + lw + uw]
        bits = np.unpackbits(upper.view(np.uint8), bitorder="little")[:ub]
        ones = np.flatnonzero(bits)
        hi = ones - np.arange(N)
        lows = np.unpackbits(lower.view(np.uint8), bitorder="little")[:N * L].reshape(N, L) \
            if L else np.zeros((N, 0), dtype=np.uint8)
        lo = (lows.astype(np.uint64) << np.arange(L, dtype=np.uint64)).sum(axis=1) if L else 0
        seqs.append((hi.astype(np.uint64) << np.uint64(L)) | lo)
        at += 6 + lw + uw
    return seqs[0], seqs[1], at + 2, w


def test_config_l16_b2000_sampled():
    """10^7 keys, l=16, b=2000, rotation fitting: the whole build on the GPU,
    checked on 48 buckets rebuilt by the oracle (values and their Golomb-Rice
    records; the largest and smallest bucket among them), on the bucket sizes,
    and on the ranks of all keys."""
    import torch

    n, l, b = 10_000_000, 16, 2000
    keys = keygen.fingerprints(n, 3)
    _case("n=1e7 l=16 b=2000 rot, sampled buckets")
    dk = torch.from_numpy(keys.view(np.int64)).cuda()
    f = rs().build(dk, l, b, True, keep_values=True)
    data = f.serialize()
    nb = oracle.num_buckets(n, b)
    C, P, gr_off, words = _parse_offsets(data)
    bucket = ((keys[:, 0].astype(object) * nb) >> 64).astype(np.int64)
    assert np.array_equal(np.diff(C.astype(np.int64)), np.bincount(bucket, minlength=nb))
    # 48 buckets the oracle rebuilds, one single-threaded oracle process per
    # host core: the largest and the smallest bucket, the first and the last,
    # and 44 spread evenly over the rest
    sizes = np.bincount(bucket, minlength=nb)
    sel = {0, nb - 1, int(np.argmax(sizes)), int(np.argmin(sizes))}
    for j in np.linspace(1, nb - 2, 60).astype(int):
        if len(sel) == 48:
            break
        sel.add(int(j))
    assert len(sel) == 48
    res, _ = shards.build_buckets_parallel(keys, l, b, True, sorted(sel))
    assert sorted(res) == sorted(sel)
    for j, (size, vals, rec_words, rec_bits) in sorted(res.items()):
        assert size == sizes[j], j
        assert np.array_equal(f.node_values(j), vals), j
        assert int(P[j + 1] - P[j]) == rec_bits
        assert np.array_equal(_record_bits(words, gr_off, int(P[j]), rec_bits), rec_words), j
    r = f.query(dk)
    rs_sorted = torch.sort(r)[0]
    assert torch.equal(rs_sorted, torch.arange(n, device=r.device, dtype=r.dtype))
    # ranks of a sample of keys against the oracle's evaluation of the same bytes
    idx = np.random.default_rng(1).choice(n, 2000, replace=False)
    assert np.array_equal(r[torch.from_numpy(idx).cuda()].cpu().numpy().view(np.uint64),
                          oracle.query(data, keys[idx]))
    bits = len(data) * 8 / n
    assert math.log2(math.e) <= bits < 1.56 + 0.06
