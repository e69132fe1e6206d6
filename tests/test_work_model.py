"""The early-exit leaf work model against exhaustive enumeration.

The roofline counts a failed leaf attempt at the expected evaluations of an
attempt that stops at the first collision within a class of its keys; this
checks that closed form by enumerating every class assignment and every
hash outcome of small leaves.
"""
import itertools

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
