"""Rotation fitting by lookup tables (Sec. 4 "Lookup Tables"), host side.

The library's table path (rs_rotation_lookup: the same tables and formula
its search kernels use when the rotation_lookup schedule option is on) must
return, for every pair of hash-position words a (keys of A) and b (keys of B)
whose popcounts pass the rotation test's gate, the smallest rotation r with
a | rot_m^r(b) = 2^m - 1 -- what the oracle's plain rotation test finds by
trying every r -- including words that repeat under rotation, where several
rotations fit and r - t must be reduced modulo the period.
"""
import itertools
import random

import pytest

import oracle


def lib_r(m, a, b):
    from paper_2212_09562_amd import recsplit

    return recsplit.rotation_lookup(m, a, b)


def oracle_r(m, a, b):
    r = oracle.rotation_fit(a, b, bin(a).count("1"), bin(b).count("1"), m)
    return m if r < 0 else r


def _words(m, k):
    for bits in itertools.combinations(range(m), k):
        yield sum(1 << p for p in bits)


@pytest.mark.parametrize("m", range(2, 10))
def test_every_gated_pair_small_leaves(m):
    """All pairs with popcount(a) + popcount(b) = m (the pairs the popcount
    gate lets through when |A| + |B| = m)."""
    n = 0
    for k in range(m + 1):
        bs = list(_words(m, m - k))
        for a in _words(m, k):
            for b in bs:
                assert lib_r(m, a, b) == oracle_r(m, a, b), (m, a, b)
                n += 1
    assert n > 0


@pytest.mark.parametrize("m", [10, 12, 14, 16])
def test_sampled_pairs_and_periodic_words(m):
    rng = random.Random(m)
    full = (1 << m) - 1
    pairs = []
    for _ in range(20000):
        k = rng.randrange(m + 1)
        a = sum(1 << p for p in rng.sample(range(m), k))
        if rng.random() < 0.5:
            # b fits a after some rotation: its complement is a rotation of a
            r = rng.randrange(m)
            na = ((a << (m - r)) | (a >> r)) & full if r else a  # rot^-r(a)
            b = ~na & full
        else:
            b = sum(1 << p for p in rng.sample(range(m), m - k))
        pairs.append((a, b))
    # words with a period below m (several rotations fit; the smallest counts)
    for p in [d for d in range(1, m) if m % d == 0]:
        for _ in range(200):
            unit = rng.randrange(1 << p)
            a = 0
            for i in range(m // p):
                a |= unit << (i * p)
            for r in range(m):
                na = ((a << (m - r)) | (a >> r)) & full if r else a
                pairs.append((a, ~na & full))
    for a, b in pairs:
        assert lib_r(m, a, b) == oracle_r(m, a, b), (m, a, b)


def test_out_of_range_leaf_sizes_refused():
    from paper_2212_09562_amd import recsplit

    for m in (0, 1, 17, 24):
        with pytest.raises(recsplit.RecSplitError):
            recsplit.rotation_lookup(m, 0, 0)
