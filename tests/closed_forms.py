"""Closed forms from the paper's analysis, computed independently of the oracle.

Used as pins: the oracle's Monte-Carlo behaviour must match these, and these
must reproduce the numbers the paper prints.
"""
from __future__ import annotations

import math
from fractions import Fraction
from functools import lru_cache

import numpy as np


def totient(d: int) -> int:
    return sum(1 for j in range(1, d + 1) if math.gcd(d, j) == 1)


def lemma_factor(m: int, a: int) -> float:
    """Appendix A lemma: lower bound of P(R)/P(B) given |A| = a, |B| = m - a,
    i.e. C(m, a) * m / sum_{d | gcd(a, m-a)} phi(d) C(m/d, (m-a)/d)."""
    g = math.gcd(a, m - a)
    s = sum(totient(d) * math.comb(m // d, (m - a) // d) for d in range(1, g + 1) if g % d == 0)
    return math.comb(m, a) * m / s


def fig_prob_factor(m: int) -> float:
    """Left plot of fig:prob: the bound averaged over |A| ~ Binomial(m, 1/2)."""
    return sum(math.comb(m, a) / 2 ** m * lemma_factor(m, a) for a in range(m + 1))


def fig_prob_overhead(m: int) -> float:
    """Right plot of fig:prob: log2(E_a[m / factor_a]) / m bits per object."""
    return math.log2(sum(math.comb(m, a) / 2 ** m * m / lemma_factor(m, a) for a in range(m + 1))) / m


@lru_cache(maxsize=None)
def _periods(m: int):
    """Period (orbit size under rotation) of every m-bit mask, by enumeration."""
    x = np.arange(1 << m, dtype=np.uint64)
    full = np.uint64((1 << m) - 1)
    per = np.full(1 << m, m, dtype=np.int64)
    for r in range(m - 1, 0, -1):
        if m % r:
            continue
        rot = ((x << np.uint64(r)) | (x >> np.uint64(m - r))) & full
        per[rot == x] = r
    pop = np.array([bin(i).count("1") for i in range(1 << m)])
    return per, pop


def orbit_mean(m: int, k: int) -> float:
    """F(m, k): mean orbit size of a uniform k-subset of Z_m under rotation."""
    per, pop = _periods(m)
    return float(per[pop == k].mean())


def rotation_attempts_given_a(m: int, a: int) -> float:
    """Expected rotation-fitting attempts of a leaf with |A| = a:
    m^m / (m! F(m, m - a)), since P(success) = P(B) * F (Appendix A)."""
    return m ** m / (math.factorial(m) * orbit_mean(m, m - a))


def rotation_attempts(m: int) -> float:
    return sum(math.comb(m, a) / 2 ** m * rotation_attempts_given_a(m, a) for a in range(m + 1))


def brute_trials(m: int) -> float:
    """Expected brute-force trials of a leaf: m^m / m! (Sec. 2.2, Appendix A)."""
    return m ** m / math.factorial(m)


def brute_early_exit_evals_per_trial(m: int) -> float:
    """Evaluations of one trial that stops at the first collision:
    key j+1 is hashed iff the first j keys landed on distinct positions."""
    return sum(math.factorial(m) / (math.factorial(m - j) * m ** j) for j in range(m))


def hash_evals_ratio(m: int) -> float:
    """fig:hashFunctionEvals: rotation fitting hashes all m keys per attempt;
    brute force with early exit, by Wald's identity, E_ee * m^m / m!."""
    return m * rotation_attempts(m) / (brute_early_exit_evals_per_trial(m) * brute_trials(m))


def split_success(sizes) -> float:
    """Probability that one seed sends exactly sizes[j] keys to child j when
    each key goes to child j with probability sizes[j] / m (multinomial)."""
    m = sum(sizes)
    lp = math.lgamma(m + 1) + sum(-math.lgamma(s + 1) + s * math.log(s / m) for s in sizes)
    return math.exp(lp)


def rice_length(p: float, tau: int) -> float:
    """Expected Golomb-Rice code length of a geometric(p) value on {0,1,...}:
    tau fixed bits + 1 stop bit + E[floor(X / 2^tau)] = sum_j (1-p)^(j 2^tau)."""
    q = math.exp((2 ** tau) * math.log1p(-p))
    return tau + 1 + q / (1 - q)


def fanouts_exact(l: int):
    lo = max(2, math.ceil(Fraction(35 * l + 55, 100)))
    up = max(2, math.ceil(Fraction(21 * l + 90, 100)))
    return lo, up


def _distinct_prefix(j: int, m: int) -> float:
    """P(j keys hashed uniformly into m slots are pairwise distinct)."""
    return math.prod(1 - t / m for t in range(j))


def early_exit_keys(j: int, m: int) -> float:
    """Keys hashed when j keys are hashed in turn until the first collision."""
    return sum(_distinct_prefix(i, m) for i in range(j))


def leaf_early_exit_evals(m: int, rotation: bool) -> float:
    """Expected evaluations of one leaf attempt that stops at the first
    collision within a class: brute force has one class of m keys; rotation
    fitting has A, |A| ~ Binomial(m, 1/2), and B, the larger hashed first and
    the other only when the first has no collision (Sec. 4: a class's word
    rules the attempt out by its popcount)."""
    if not rotation:
        return early_exit_keys(m, m)
    tot = 0.0
    for a in range(m + 1):
        n1 = max(a, m - a)
        tot += math.comb(m, a) / 2 ** m * (early_exit_keys(n1, m) +
                                           _distinct_prefix(n1, m) * early_exit_keys(m - n1, m))
    return tot
