"""The packed child counters of the staged split search, restated in Python.

The first k-1 children of a split count in fields of fe bits (fe the bit
length of the part size u); the last child adds above them.  A child above
its part size is found for all fields at once: adding u' = 2^fe - 1 - u to
every field carries out of exactly the fields holding more than u, and
(acc + c) ^ acc ^ c is the carry vector of that addition.  The final test
compares the low (k-1)*fe bits with u in every field.  Checked here over
every count vector of small splits, including fields that overflow.
"""
import itertools

import pytest


def _layout(k, u):
    fe = u.bit_length()
    comp = carries = target = 0
    for j in range(k - 1):
        target |= u << (fe * j)
        comp |= ((1 << fe) - 1 - u) << (fe * j)
        carries |= 1 << (fe * (j + 1))
    return fe, comp, carries, target, (1 << (fe * (k - 1))) - 1


def _pack(counts, fe):
    acc = 0
    for j, c in enumerate(counts):
        acc += c << (fe * j)  # the last child lands above the fields
    return acc & 0xFFFFFFFF


@pytest.mark.parametrize("k,u", [(3, 2), (4, 3), (3, 5), (5, 4), (2, 7), (4, 8)])
def test_overfull_child_found_by_one_add(k, u):
    fe, comp, carries, target, low = _layout(k, u)
    assert (k - 1) * fe <= 31
    top = (1 << fe) - 1  # counts of the explicit fields before they wrap
    for counts in itertools.product(range(top + 1), repeat=k - 1):
        for last in range(0, u + 3):
            acc = _pack(list(counts) + [last], fe)
            dead = (((acc + comp) ^ acc ^ comp) & carries) != 0
            assert dead == any(c > u for c in counts), (counts, last)
            # the final word test: exact when no field has wrapped
            assert ((acc & low) == target) == all(c == u for c in counts)


def test_wrapped_field_is_only_a_missed_exit():
    # a field past 2^fe - 1 carries into the next one; the attempt is dead
    # anyway, and a test that misses it only evaluates more keys
    k, u = 3, 5
    fe, comp, carries, target, low = _layout(k, u)
    for c0 in range(1 << fe, 3 << fe):
        for c1 in range(0, u + 1):
            acc = _pack([c0, c1, 0], fe)
            dead = (((acc + comp) ^ acc ^ comp) & carries) != 0
            if not dead:
                assert c0 > u  # missed: the attempt is dead and is verified exactly later
