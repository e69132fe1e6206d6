"""Pins for the oracle's primitives: hash, remap, buckets, tree shape, rotation.

Each test ties a function of the CPU oracle to something other than the
oracle itself: a published reference vector, the paper's formulas evaluated
in exact arithmetic, invariants the paper states, or brute force over all
small inputs.
"""
import math

import numpy as np
import pytest

import oracle
from closed_forms import fanouts_exact
from conftest import golden
from paper_2212_09562_amd import keygen

GOLDEN = 0x9E3779B97F4A7C15


def test_splitmix64_reference_vector():
    ref = [int(r[0], 16) for r in golden("splitmix64_seed0.txt")]
    assert [int(x) for x in oracle.splitmix64(0, 5)] == ref
    # the seeded input generator is a second, independent implementation
    assert [int(x) for x in keygen.splitmix64_stream(0, 0, 5)] == ref


def test_keygen_matches_oracle_stream():
    for seed in (1, 2, 3, 12345):
        a = keygen.splitmix64_stream(seed, 0, 64)
        b = oracle.splitmix64(seed, 64)
        assert np.array_equal(a, b)


def test_hash_is_splitmix_mixer():
    # hash(w1, x) = mixer(w1 + x); SplitMix64 output i of seed 0 is mixer((i+1) * golden)
    ref = [int(r[0], 16) for r in golden("splitmix64_seed0.txt")]
    for i, r in enumerate(ref):
        assert oracle.hash64(0, (i + 1) * GOLDEN % 2 ** 64) == r
        # the sum wraps modulo 2^64
        assert oracle.hash64(GOLDEN, i * GOLDEN % 2 ** 64) == r
        assert oracle.hash64((i + 1) * GOLDEN % 2 ** 64 + 5, 2 ** 64 - 5) == r


def test_start_seeds_are_splitmix_outputs():
    ref = [int(r[0], 16) for r in golden("splitmix64_seed0.txt")]
    assert [oracle.start_seed(d) for d in range(5)] == ref


def test_remap_exact_multiply_high():
    rng = np.random.default_rng(7)
    for M in (1, 2, 3, 7, 16, 24, 112, 560, 4095):
        assert oracle.remap(0, M) == 0
        assert oracle.remap(0xFFFFFFFF << 32, M) == M - 1
        for h in rng.integers(0, 2 ** 63, 50, dtype=np.uint64):
            h = int(h) * 2 + 1
            p = oracle.remap(h, M)
            # p is the unique integer with p <= (h >> 32) * M / 2^32 < p + 1
            assert p * 2 ** 32 <= (h >> 32) * M < (p + 1) * 2 ** 32


def test_remap_equal_share():
    # every position receives floor or ceil of 2^32 / M top words
    for M in (3, 5, 7, 16, 24):
        counts = [0] * M
        for p in range(M):
            lo = -(-p * 2 ** 32 // M)
            hi = -(-(p + 1) * 2 ** 32 // M)
            counts[p] = hi - lo
            assert oracle.remap(lo << 32, M) == p
            assert oracle.remap((hi - 1) << 32, M) == p
        assert sum(counts) == 2 ** 32
        assert max(counts) - min(counts) <= 1


def test_bucket_map():
    for nb in (1, 2, 3, 1000, 10 ** 7):
        assert oracle.bucket_of(0, nb) == 0
        assert oracle.bucket_of(2 ** 64 - 1, nb) == nb - 1
        w0 = [0, 1, 2 ** 32, 2 ** 63, 2 ** 64 - 2]
        bs = [oracle.bucket_of(w, nb) for w in w0]
        assert bs == sorted(bs)  # monotone in w0
        for w in w0:
            assert oracle.bucket_of(w, nb) == (w * nb) >> 64
    assert oracle.num_buckets(0, 100) == 1
    assert oracle.num_buckets(100000, 100) == 1000
    assert oracle.num_buckets(10 ** 7, 2000) == 5000
    assert oracle.num_buckets(101, 100) == 2


def test_bucket_sizes_are_balanced():
    k = keygen.fingerprints(200000, 11)
    nb = 2000
    b = np.array([oracle.bucket_of(int(w), nb) for w in k[:, 0]])
    cnt = np.bincount(b, minlength=nb)
    # Poisson(100): chi-square with nb - 1 degrees of freedom stays near nb
    chi2 = ((cnt - 100.0) ** 2 / 100.0).sum()
    assert abs(chi2 - nb) < 6 * math.sqrt(2 * nb)


@pytest.mark.parametrize("l", list(range(2, 25)))
def test_fanouts_match_formula(l):
    assert oracle.fanouts(l) == fanouts_exact(l)


def test_fanout_values():
    # values of the two formulas of Sec. 2.2 at the leaf sizes the paper uses
    assert oracle.fanouts(8) == (4, 3)
    assert oracle.fanouts(12) == (5, 4)
    assert oracle.fanouts(16) == (7, 5)
    assert oracle.fanouts(24) == (9, 6)
    # 0.35*7 + 0.55 = 3 and 0.21*10 + 0.9 = 3 exactly
    assert oracle.fanouts(7)[0] == 3
    assert oracle.fanouts(10)[1] == 3


def _leaf_level(m, l):
    """Sizes of all children at the leaf level (including size-1 ones), in order."""
    if m <= l:
        return [m]
    out = []
    for c in oracle.children(m, l):
        out += _leaf_level(c, l)
    return out


@pytest.mark.parametrize("l", [2, 3, 4, 5, 8, 12, 16, 24])
def test_tree_shape_invariants(l):
    rng = np.random.default_rng(l)
    ms = sorted(set([2, 3, l, l + 1, 2 * l, 2 * l + 1] + list(rng.integers(2, 5000, 60))))
    lf, uf = oracle.fanouts(l)
    for m in ms:
        m = int(m)
        leaves = _leaf_level(m, l)
        assert sum(leaves) == m
        # every leaf but possibly the last holds exactly l objects (Sec. 2.2)
        assert all(x == l for x in leaves[:-1])
        assert 1 <= leaves[-1] <= l
        parts = oracle.children(m, l)
        if m <= l:
            assert parts == []
        else:
            assert sum(parts) == m and min(parts) >= 1
            if m <= lf * l:
                assert len(parts) == -(-m // l)
            elif m <= uf * lf * l:
                assert len(parts) == -(-m // (lf * l))
            else:
                assert len(parts) == 2
                # the left subtree is full: a multiple of the upper unit
                assert parts[0] % (uf * lf * l) == 0


def _rotation_fit_by_sets(a, b, na, nb_, m):
    """Definition by sets: the na keys of A land on the set bits of a, the nb_
    keys of B on those of b (fewer bits than keys means a collision).  The
    value is the smallest r with A and (B + r) mod m partitioning Z_m."""
    A = {p for p in range(m) if a >> p & 1}
    B = {p for p in range(m) if b >> p & 1}
    if len(A) != na or len(B) != nb_:
        return None
    for r in range(m):
        Bs = {(p + r) % m for p in B}
        if A.isdisjoint(Bs) and (A | Bs) == set(range(m)):
            return r
    return None


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6])
def test_rotation_fit_exhaustive(m):
    for na in range(m + 1):
        nb_ = m - na
        for a in range(1 << m):
            if bin(a).count("1") > na or (na > 0) != (a > 0):
                continue
            for b in range(1 << m):
                if bin(b).count("1") > nb_ or (nb_ > 0) != (b > 0):
                    continue
                want = _rotation_fit_by_sets(a, b, na, nb_, m)
                got = oracle.rotation_fit(a, b, na, nb_, m)
                assert got == (-1 if want is None else want), (a, b, na)


def test_rot_moves_bits_up_cyclically():
    for m in (2, 5, 8, 16, 24):
        for p in range(m):
            for r in range(m):
                assert oracle.rot(1 << p, r, m) == 1 << ((p + r) % m)
