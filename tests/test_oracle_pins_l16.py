"""Pins of the oracle's searches at the headline leaf size l = 16 (b = 2000).

The expected number of attempts of every node kind follows from the paper's
probability analysis: m^m / (m! F) rotation attempts per leaf (Appendix A,
F the mean rotation-orbit size of the B positions), and 1 / p seeds per
lower or upper split, p the multinomial probability that the seed sends
exactly the part sizes to the children (Sec. 2.2).  The oracle's means over
many random nodes of the l = 16 tree must match them within 4 sigma
(sigma = sqrt(mu^2 - mu) / sqrt(N) for a geometric count).  A wrong child
rule, a dropped hash term or a rotation applied the wrong way moves these
means by far more.  The nodes are searched by several processes; each node
is still one plain single-threaded oracle call.
"""
import math
import multiprocessing as mp

import numpy as np
import pytest

import oracle
from closed_forms import rotation_attempts, split_success
from paper_2212_09562_amd import keygen

pytestmark = pytest.mark.slow

PROCS = 8


def _leaf_attempts(args):
    w1, isb, depth = args
    m = len(w1)
    v, _ = oracle.leaf_search(w1, isb, depth, oracle.LEAF_ROT)
    return v // m + 1


def _split_trials(args):
    w1, l, depth = args
    return oracle.split_search(w1, l, depth) + 1


def _pool_map(fn, items):
    with mp.get_context("fork").Pool(PROCS) as pool:
        return np.array(pool.map(fn, items, chunksize=1), dtype=np.float64)


def _check_geometric_mean(t, want):
    sigma = math.sqrt(want * want - want) / math.sqrt(len(t))
    assert abs(t.mean() - want) < 4 * sigma, (t.mean(), want, sigma)


def test_l16_rotation_leaf_attempts():
    """Full leaves of 16 keys with rotation fitting: mean attempts 55,240."""
    m, N = 16, 6400
    want = rotation_attempts(m)
    assert abs(want - 55240) < 1.0
    k = keygen.fingerprints(m * N, 1601).reshape(N, m, 2)
    items = [(k[i, :, 1].copy(), (k[i, :, 0] & np.uint64(1)).astype(np.uint8), 1 + i % 4)
             for i in range(N)]
    _check_geometric_mean(_pool_map(_leaf_attempts, items), want)


@pytest.mark.parametrize("m,N,paper", [(112, 240, 397_978), (560, 96, 222_260)])
def test_l16_split_trials(m, N, paper):
    """Lower splits (112 keys into 7 parts of 16) and upper splits (560 keys
    into 5 parts of 112) of the l = 16 tree: mean seeds 1 / p."""
    l = 16
    sizes = oracle.children(m, l)
    assert sizes == [m // len(sizes)] * len(sizes)
    want = 1.0 / split_success(sizes)
    assert abs(want - paper) < 1.0
    k = keygen.fingerprints(m * N, 1700 + m)
    items = [(k[i * m:(i + 1) * m, 1].copy(), l, 1 + i % 3) for i in range(N)]
    _check_geometric_mean(_pool_map(_split_trials, items), want)
