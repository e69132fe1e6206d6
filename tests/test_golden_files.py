"""CPU: the stored oracle results that the GPU tests compare against are
consistent with the paper's rules, independently of the search that made
them.

* tests/golden/large_leaf_sets.txt (whole structures, l = 19 to 24): every
  stored structure is a minimal perfect hash function of its key set (the
  ranks the oracle's query gives form a permutation of [0, n)).
* tests/golden/l24_b2000_n5e6_buckets.txt (three buckets of the l = 24,
  b = 2000, n = 5 million configuration of tab:showcaseOverall): the bucket
  sizes agree with a count of the keys (Sec. 2.2, buckets by the
  multiply-high of the first key word), there is one value per node of the
  splitting tree, and each record is exactly the Golomb-Rice code of those
  values (Sec. 2.2 "Representation": the fixed parts of all nodes in
  preorder, then their unary parts), decoded here bit by bit.
"""
import os

import numpy as np
import pytest

import oracle
from paper_2212_09562_amd import keygen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not written")
    return [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]


def test_large_leaf_structures_are_minimal_perfect():
    rows = _rows("large_leaf_sets.txt")
    assert rows
    for n, l, b, rot, seed, hexbytes in rows:
        n, seed = int(n), int(seed)
        keys = keygen.fingerprints(n, seed)
        ranks = oracle.query(bytes.fromhex(hexbytes), keys)
        assert np.array_equal(np.sort(ranks), np.arange(n)), (n, l, b, rot, seed)


def _bit(words, pos):
    return (int(words[pos >> 6]) >> (pos & 63)) & 1


def _gr_decode(words, nbits, sizes, l):
    """Values of the nodes (sizes in preorder) from one bucket's record."""
    taus = [oracle.tau(m, l) for m in sizes]
    pos, fixed = 0, []
    for t in taus:
        f = 0
        for i in range(t):
            f |= _bit(words, pos + i) << i
        fixed.append(f)
        pos += t
    vals = []
    for t, f in zip(taus, fixed):
        q = 0
        while not _bit(words, pos):
            q += 1
            pos += 1
        pos += 1
        vals.append((q << t) | f)
    assert pos == nbits
    return vals


def test_l24_showcase_buckets_consistent():
    rows = _rows("l24_b2000_n5e6_buckets.txt")
    assert len(rows) == 9
    n, l, b = 5_000_000, 24, 2000
    keys = keygen.fingerprints(n, 55)
    nb = oracle.num_buckets(n, b)
    w0 = keys[:, 0]
    hi, lo = w0 >> np.uint64(32), w0 & np.uint64(0xFFFFFFFF)
    nbu = np.uint64(nb)
    bucket = ((hi * nbu + ((lo * nbu) >> np.uint64(32))) >> np.uint64(32)).astype(np.int64)
    for i in (0, 1, n // 2, n - 1):
        assert bucket[i] == oracle.bucket_of(int(w0[i]), nb)
    counts = np.bincount(bucket, minlength=nb)
    for i in range(0, len(rows), 3):
        j, size, bits = (int(x) for x in rows[i])
        words = np.array([int(w, 16) for w in rows[i + 1]], dtype=np.uint64)
        vals = [int(v) for v in rows[i + 2]]
        assert counts[j] == size
        sizes = oracle.preorder_sizes(size, l)
        assert len(vals) == len(sizes)
        assert len(words) == (bits + 63) // 64
        assert _gr_decode(words, bits, sizes, l) == vals, j
