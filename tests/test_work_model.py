"""The early-exit work model of the roofline against enumeration.

The roofline counts a failed attempt at the expected evaluations of an
attempt that stops at the first evidence that it fails: a collision within a
class of a leaf's keys, a split child above its part size.  These tests
check the leaf closed form and the library's table (rs_attempt_work) by
enumerating every class assignment and every hash outcome of small nodes,
and the split table at l = 16 by simulation.
"""
import itertools

import numpy as np
import pytest

from closed_forms import brute_early_exit_evals_per_trial, leaf_early_exit_evals


def _enumerate(m: int, rotation: bool) -> float:
    total, count = 0.0, 0
    classes = itertools.product((0, 1), repeat=m) if rotation else [(0,) * m]
    for cls in classes:
        a = [i for i in range(m) if cls[i] == 0]
        b = [i for i in range(m) if cls[i] == 1]
        first, second = (a, b) if len(a) >= len(b) else (b, a)
        for pos in itertools.product(range(m), repeat=m):
            evals = 0
            ok = True
            for group in (first, second):
                seen = set()
                for i in group:
                    evals += 1
                    if pos[i] in seen:
                        ok = False
                        break
                    seen.add(pos[i])
                if not ok:
                    break
            total += evals
            count += 1
    return total / count


@pytest.mark.parametrize("m", [2, 3, 4, 5])
@pytest.mark.parametrize("rotation", [False, True])
def test_leaf_early_exit_model_matches_enumeration(m, rotation):
    assert leaf_early_exit_evals(m, rotation) == pytest.approx(_enumerate(m, rotation), rel=1e-12)


def test_brute_model_is_the_papers_early_exit_count():
    for m in range(2, 17):
        assert leaf_early_exit_evals(m, False) == pytest.approx(brute_early_exit_evals_per_trial(m))


# ---------------------------------------------------------------- the library's table
def _lib():
    from paper_2212_09562_amd import recsplit

    return recsplit


def _split_parts(l: int, m: int):
    """Part sizes of a node of m keys: fanouts ceil(0.35 l + 0.55) and
    ceil(0.21 l + 0.9) (at least 2) above the leaves, 2 above those."""
    lo = max(2, -(-(35 * l + 55) // 100))
    up = max(2, -(-(21 * l + 90) // 100))
    la, ua = lo * l, lo * l * up
    if m <= l:
        return None
    if m > ua:
        return "binary"
    unit = l if m <= la else la
    k = -(-m // unit)
    return [unit] * (k - 1) + [m - unit * (k - 1)]


def _enumerate_split(parts):
    """Mean keys hashed by an attempt that stops once some child holds more
    keys than its part size, over every assignment of the m keys to
    positions 0..m-1 (child = position // unit)."""
    m = sum(parts)
    unit = parts[0]
    total, count = 0, 0
    for pos in itertools.product(range(m), repeat=m):
        cnt = [0] * len(parts)
        evals = 0
        for p in pos:
            evals += 1
            ch = min(p // unit, len(parts) - 1)
            cnt[ch] += 1
            if cnt[ch] > parts[ch]:
                break
        total += evals
        count += 1
    return total / count


@pytest.mark.parametrize("l,m", [(2, 3), (2, 4), (2, 5), (2, 6), (3, 4), (3, 5), (3, 6), (3, 7)])
def test_split_attempt_work_matches_enumeration(l, m):
    parts = _split_parts(l, m)
    assert isinstance(parts, list)
    assert _lib().attempt_work(l, m) == pytest.approx(_enumerate_split(parts), rel=1e-9)


def test_split_attempt_work_matches_simulation_at_l16():
    rng = np.random.default_rng(7)
    for m, trials in ((112, 20000), (100, 20000), (560, 4000)):
        parts = _split_parts(16, m)
        bounds = np.cumsum(parts)
        ch = np.searchsorted(bounds, rng.integers(0, m, size=(trials, m)), side="right")
        onehot = np.zeros((trials, m, len(parts)), dtype=np.int16)
        np.put_along_axis(onehot, ch[..., None], 1, axis=2)
        over = (np.cumsum(onehot, axis=1) > np.array(parts)).any(axis=2)
        evals = np.where(over.any(axis=1), over.argmax(axis=1) + 1, m)
        se = evals.std() / np.sqrt(trials)
        assert abs(_lib().attempt_work(16, m) - evals.mean()) < 5 * se + 1e-9, m


def test_leaf_and_binary_attempt_work():
    for m in range(2, 17):
        assert _lib().attempt_work(16, m, rotation=True) == pytest.approx(
            leaf_early_exit_evals(m, True), abs=2e-4)
        assert _lib().attempt_work(16, m, rotation=False) == pytest.approx(
            leaf_early_exit_evals(m, False), abs=2e-4)
    assert _split_parts(16, 2000) == "binary" and _lib().attempt_work(16, 2000) == 2000.0
    with pytest.raises(Exception):
        _lib().attempt_work(1, 5)
