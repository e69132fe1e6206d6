"""Pins for the oracle's searches against the paper's probability analysis.

The expected number of trials of each search has a closed form (Sec. 2.2,
Appendix A); the oracle's means over many random nodes must match it within
Monte-Carlo error, and the printed values of fig:prob and
fig:hashFunctionEvals must follow.  A dropped term in the hash, a wrong
rotation, or a split that counts the wrong child shifts these means by far
more than the tolerance.
"""
import math

import numpy as np
import pytest

import oracle
from closed_forms import (brute_early_exit_evals_per_trial, brute_trials, fig_prob_factor,
                          fig_prob_overhead, hash_evals_ratio, lemma_factor, orbit_mean,
                          rotation_attempts, rotation_attempts_given_a, split_success)
from conftest import golden
from paper_2212_09562_amd import keygen


def _leaves(m, count, seed):
    k = keygen.fingerprints(m * count, seed).reshape(count, m, 2)
    return k[:, :, 1], (k[:, :, 0] & np.uint64(1)).astype(np.uint8)


@pytest.mark.parametrize("m", [2, 3, 5, 8])
def test_leaf_naive_equals_bitmask(m):
    w1, isb = _leaves(m, 300, 100 + m)
    for i in range(300):
        d = i % 4
        v0, _ = oracle.leaf_search(w1[i], isb[i], d, oracle.LEAF_BRUTE)
        v1, _ = oracle.leaf_search(w1[i], isb[i], d, oracle.LEAF_BRUTE_NAIVE)
        assert v0 == v1
        r0, _ = oracle.leaf_search(w1[i], isb[i], d, oracle.LEAF_ROT)
        r1, _ = oracle.leaf_search(w1[i], isb[i], d, oracle.LEAF_ROT_NAIVE)
        assert r0 == r1


def test_leaf_trials_brute_force():
    """Mean (v + 1) of brute-force leaves = m^m / m! (Sec. 2.2, Appendix A)."""
    m, N = 8, 4000
    w1, isb = _leaves(m, N, 21)
    t = np.array([oracle.leaf_search(w1[i], isb[i], 0, oracle.LEAF_BRUTE)[0] + 1 for i in range(N)])
    want = brute_trials(m)  # 416.1
    assert abs(want - 416.1) < 0.1
    sigma = math.sqrt(want * want - want) / math.sqrt(N)
    assert abs(t.mean() - want) < 4 * sigma


def test_leaf_attempts_rotation_by_class():
    """Rotation attempts given |A| = a follow m^m / (m! F(m, m - a)), F the mean
    rotation-orbit size (Appendix A: P(R) = P(B) times that factor)."""
    m, N = 8, 6000
    w1, isb = _leaves(m, N, 22)
    att = np.array([oracle.leaf_search(w1[i], isb[i], 1, oracle.LEAF_ROT)[0] // m + 1
                    for i in range(N)])
    na = m - isb.sum(axis=1)
    for a in range(m + 1):
        sel = att[na == a]
        if len(sel) < 200:
            continue
        want = rotation_attempts_given_a(m, a)
        sigma = math.sqrt(want * want - want) / math.sqrt(len(sel))
        assert abs(sel.mean() - want) < 4 * sigma, (a, sel.mean(), want)
    want = rotation_attempts(m)
    assert abs(want - 56.48) < 0.01
    sigma = math.sqrt(want * want) / math.sqrt(N)
    assert abs(att.mean() - want) < 4 * sigma


def test_fig_prob_values_reproduced():
    """The lemma's bound, averaged over |A|, reproduces fig:prob exactly."""
    for m, factor, overhead in golden("fig_prob.txt"):
        m = int(m)
        assert fig_prob_factor(m) == pytest.approx(float(factor), rel=2e-5, abs=1e-6)
        assert fig_prob_overhead(m) == pytest.approx(float(overhead), rel=2e-5, abs=1e-9)


def test_lemma_bound_and_exact_factor():
    """P(R)/P(B) = F(m, m-a) >= bound, with equality when gcd(a, m-a) = 1."""
    for m in range(2, 13):
        for a in range(m + 1):
            exact = orbit_mean(m, m - a) * 1.0
            bound = lemma_factor(m, a)
            assert exact >= bound - 1e-12
            if math.gcd(a, m - a) == 1:
                assert exact == pytest.approx(bound, rel=1e-12)


def test_rotation_success_factor_monte_carlo():
    """Measured P(R)/P(B) over leaves of size 6 matches the exact factor."""
    m, N = 6, 8000
    w1, isb = _leaves(m, N, 23)
    rot = np.array([oracle.leaf_search(w1[i], isb[i], 0, oracle.LEAF_ROT)[0] // m + 1
                    for i in range(N)], dtype=float)
    brute = np.array([oracle.leaf_search(w1[i], isb[i], 0, oracle.LEAF_BRUTE)[0] + 1
                      for i in range(N)], dtype=float)
    want = brute_trials(m) / rotation_attempts(m)
    got = brute.mean() / rot.mean()
    assert abs(got / want - 1) < 4 * math.sqrt(2.0 / N)


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6, 7, 8])
def test_fig_hash_evals(m):
    """Hash evaluations of rotation fitting relative to brute force with early
    exit (fig:hashFunctionEvals): closed form, oracle and printed value agree."""
    printed = {int(r[0]): float(r[1]) for r in golden("fig_hash_evals.txt")}[m]
    closed = hash_evals_ratio(m)
    assert closed == pytest.approx(printed, rel=0.01)
    N = 6000
    w1, isb = _leaves(m, N, 300 + m)
    rot_evals = brute_ee = 0
    for i in range(N):
        v, _ = oracle.leaf_search(w1[i], isb[i], 0, oracle.LEAF_ROT)
        rot_evals += (v // m + 1) * m
        _, ee = oracle.leaf_search(w1[i], isb[i], 0, oracle.LEAF_BRUTE)
        brute_ee += ee
    got = rot_evals / brute_ee
    assert abs(got / printed - 1) < 4 * math.sqrt(2.0 / N) + 0.01, (got, printed)


def _children_by_definition(w1s, m, l, s, depth):
    """Child index of each key, written from readings R6-R8 with Python ints."""
    lf, uf = oracle.fanouts(l)
    la, ua = lf * l, uf * lf * l
    x = (s + oracle.start_seed(depth)) % 2 ** 64
    out = []
    for w in w1s:
        h = oracle.hash64(int(w), x)
        p = ((h >> 32) * m) >> 32
        if m > ua:
            left = ua * (-(-(m // 2) // ua))
            out.append(1 if p >= left else 0)
        else:
            out.append(p // (l if m <= la else la))
    return out


@pytest.mark.parametrize("m,l", [(32, 8), (20, 8), (96, 8), (60, 8), (140, 8), (300, 8), (60, 12)])
def test_split_seed_is_minimal(m, l):
    k = keygen.fingerprints(m * 6, 40 + m)
    sizes = oracle.children(m, l)
    for i in range(6):
        w1 = k[i * m:(i + 1) * m, 1]
        s = oracle.split_search(w1, l, i)
        for t in range(s + 1):
            ch = _children_by_definition(w1, m, l, t, i)
            cnt = [ch.count(j) for j in range(len(sizes))]
            assert (cnt == sizes) == (t == s), (t, s, cnt, sizes)


@pytest.mark.parametrize("m,l", [(32, 8), (96, 8), (200, 8)])
def test_split_trials_match_multinomial(m, l):
    """Mean (s + 1) = 1 / p with p the multinomial probability of the exact
    part sizes (the splitting search of Sec. 2.2)."""
    N = 1500
    k = keygen.fingerprints(m * N, 500 + m)
    t = np.array([oracle.split_search(k[i * m:(i + 1) * m, 1], l, i % 3) + 1 for i in range(N)])
    want = 1.0 / split_success(oracle.children(m, l))
    sigma = math.sqrt(want * want - want) / math.sqrt(N)
    assert abs(t.mean() - want) < 4 * sigma, (t.mean(), want)
