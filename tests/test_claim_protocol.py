"""Exhaustive model of the search kernel's claim and finalize protocol (CPU).

The persistent search kernel shares one split search among workers: a
64-bit claim word per task holds the chunks in flight (low 32 bits), the
rounds handed out so far (the cursor) and a found bit (bit 63); a worker
claims a chunk of rounds with one atomic add, evaluates it with its waves,
and thread 0 then publishes a value (atomicMin on the task's best, then the
found bit), drops its chunk and claims the next with one atomic, or leaves.
Whoever drops the in-flight count to zero with the found bit set finalizes
the task (a compare-and-swap closes it).  Inside a worker, thread 0 passes
its decision (evaluate the next chunk, or stop and maybe finalize) to the
other waves through LDS between two barriers.

This file models that protocol step by step -- every global atomic, every
LDS access and barrier of the kernel's claim loop is one step of one wave --
and explores every interleaving of two workers of two waves each, or of
three workers (the owner with two waves, two helpers with one), explicit
states breadth first, on small searches with chosen valid attempts.  In every reachable final state: no wave waits at a barrier its
partner left (no deadlock), exactly one worker finalizes, the value it
finalizes is the smallest valid attempt (no chunk below it was skipped), the
found bit is set and no chunk is in flight.  The owner's claim-ahead (two
chunks in flight) and helpers that leave at any decision are included, and
so is the attempt cap (an error ends the search without a value).

The same model with the barrier between the chunk's evaluation and thread
0's rewrite of the decision taken out -- the ordering the kernel had before
that barrier was added -- must reach a bad state, and so must a drop that
finalizes without the found bit; the tests check that it does, so the model
is able to see those classes of bug.
"""
from __future__ import annotations

from collections import deque

import pytest

INF = 1 << 62
FOUND = 1 << 63
MASK32 = (1 << 32) - 1


def cursor(np_):
    return (np_ >> 32) & 0x7FFFFFFF


class Config:
    def __init__(self, workers, valid, rmax=2, cap_rounds=5, owner_ahead=True, b2=True,
                 helper_leaves=True, helper_waves=2, found_check=True):
        self.workers = workers        # worker 0 owns the task, the others help
        self.helper_waves = helper_waves  # waves of each helper (the owner has two)
        self.valid = frozenset(valid)  # valid attempts; attempt = 2 * round + wave
        self.rmax = rmax              # longest claim, in rounds
        self.cap_rounds = cap_rounds  # claims past this cursor hit the attempt cap
        self.owner_ahead = owner_ahead  # the owner claims its next chunk before evaluating
        self.b2 = b2                  # barrier between evaluation and the rewritten decision
        self.helper_leaves = helper_leaves
        self.found_check = found_check  # a drop finalizes only with the found bit set


# Global state: (np, best, closed, error).
# Per worker LDS: (go, fin, first, rounds, s_best, barrier arrivals (w0, w1),
#   barrier generation).
# Wave 0 locals (thread 0): (pc, r, have_next, next_old, next_r, held, v, claims, tmp)
# Wave 1 locals: (pc, round index)
# The finalizers are recorded as (worker, value).

def _initial(cfg):
    glob = (0, INF, 0, 0)
    lds = tuple((0, 0, 0, 0, INF, (0, 0), 0) for _ in range(cfg.workers))
    w0 = tuple(("init", 1, False, 0, 0, 0, INF, 0, 0) for _ in range(cfg.workers))
    w1 = tuple(("top", 0) if k == 0 or cfg.helper_waves == 2 else ("done", 0)
               for k in range(cfg.workers))
    return (glob, lds, w0, w1, ())


def _decide(cfg, k, old, rr, glob, lds):
    """Thread 0 turns a claim's old word into a decision.  Returns
    (glob, lds, next pc, extra) where extra carries a pending release."""
    first = cursor(old)
    go, fin, f0, r0, sb, arr, gen = lds[k]
    if old & FOUND:
        return glob, lds, ("release", 1), None
    if first >= cfg.cap_rounds:
        np_, best, closed, err = glob
        glob = (np_, best, closed, 1)
        return glob, lds, ("release", 1), None
    lds = lds[:k] + ((1, fin, first, rr, sb, arr, gen),) + lds[k + 1:]
    return glob, lds, ("to_top",), None


def _successors(cfg, state):
    glob, lds, w0s, w1s, fins = state
    out = []
    for k in range(cfg.workers):
        own = k == 0
        # ---------------------------------------------------------- wave 0
        pc, r, have_next, next_old, next_r, held, v, claims, tmp = w0s[k]
        go, fin, first, rounds, sb, arr, gen = lds[k]

        def put(glob2, lds2, w0new, fins2=fins, _k=k):
            out.append((glob2, lds2, w0s[:_k] + (w0new,) + w0s[_k + 1:], w1s, fins2))

        def setl(newl, _k=k):
            return lds[:_k] + (newl,) + lds[_k + 1:]

        np_, best, closed, err = glob
        if pc == "init":
            # sh.fin = 0, sh.best = inf, sh.go = 0 (LDS, before the first barrier)
            lds2 = setl((0, 0, first, rounds, INF, arr, gen))
            if not own and cfg.helper_leaves:
                put(glob, lds2, ("top", r, have_next, next_old, next_r, held, v, claims, 0))
            put(glob, lds2, ("claim0", r, have_next, next_old, next_r, held, v, claims, 0))
        elif pc == "claim0":
            old = np_
            glob2 = (np_ + ((r << 32) | 1), best, closed, err)
            rr = r
            r2 = min(r * 2, cfg.rmax)
            g3, l3, nxt, _ = _decide(cfg, k, old, rr, glob2, lds)
            if nxt[0] == "release":
                put(g3, l3, ("rel", r2, have_next, next_old, next_r, nxt[1], v, claims + 1, 0))
            else:
                put(g3, l3, ("top", r2, have_next, next_old, next_r, held, v, claims + 1, 0))
        elif pc == "rel":
            # release_chunk(held): the drop; the close follows as its own step
            n = held
            old = np_
            glob2 = (np_ - n, best, closed, err)
            if (old & MASK32) == n and ((old & FOUND) or not cfg.found_check):
                put(glob2, lds, ("close", r, have_next, next_old, next_r, held, v, claims, 0))
            else:
                put(glob2, setl((go, 0, first, rounds, sb, arr, gen)),
                    ("top", r, have_next, next_old, next_r, held, v, claims, 0))
        elif pc == "close":
            if closed == 0:
                put((np_, best, 1, err), setl((go, 1, first, rounds, sb, arr, gen)),
                    ("top", r, have_next, next_old, next_r, held, v, claims, 0))
            else:
                put(glob, setl((go, 0, first, rounds, sb, arr, gen)),
                    ("top", r, have_next, next_old, next_r, held, v, claims, 0))
        elif pc == "top":
            # barrier B1
            a0, a1 = arr
            if a0 == 0:
                put(glob, setl((go, fin, first, rounds, sb, (1, a1), gen)),
                    ("b1wait", r, have_next, next_old, next_r, held, v, claims, gen))
        elif pc == "b1wait":
            if gen != tmp:  # the barrier opened
                put(glob, lds, ("readgo", r, have_next, next_old, next_r, held, v, claims, 0))
        elif pc == "readgo":
            if not go:
                put(glob, lds, ("exit", r, have_next, next_old, next_r, held, v, claims, 0))
            elif own and cfg.owner_ahead:
                # claim the next chunk before evaluating this one
                old = np_
                put((np_ + ((r << 32) | 1), best, closed, err), lds,
                    ("eval", min(r * 2, cfg.rmax), True, old, r, held, v, claims + 1, 0))
            else:
                put(glob, lds, ("eval", r, have_next, next_old, next_r, held, v, claims, 0))
        elif pc == "eval":
            # tmp = rounds of the chunk done by this wave
            if tmp >= rounds:
                put(glob, lds, ("b2" if cfg.b2 else "dec", r, have_next, next_old, next_r, held, v,
                                claims, 0))
            else:
                a = 2 * (first + tmp) + 0
                if a >= sb:
                    put(glob, lds, ("b2" if cfg.b2 else "dec", r, have_next, next_old, next_r,
                                    held, v, claims, 0))
                elif a in cfg.valid:
                    put(glob, setl((go, fin, first, rounds, min(sb, a), arr, gen)),
                        ("b2" if cfg.b2 else "dec", r, have_next, next_old, next_r, held, v,
                         claims, 0))
                else:
                    put(glob, lds, ("eval", r, have_next, next_old, next_r, held, v, claims,
                                    tmp + 1))
        elif pc == "b2":
            a0, a1 = arr
            if a0 == 0:
                put(glob, setl((go, fin, first, rounds, sb, (1, a1), gen)),
                    ("b2wait", r, have_next, next_old, next_r, held, v, claims, gen))
        elif pc == "b2wait":
            if gen != tmp:
                put(glob, lds, ("dec", r, have_next, next_old, next_r, held, v, claims, 0))
        elif pc == "dec":
            # v = sh.best; sh.best = inf; sh.fin = 0; sh.go = 0
            hold = 2 if have_next else 1
            lds2 = setl((0, 0, first, rounds, INF, arr, gen))
            base = (r, False, next_old, next_r, hold, sb, claims)
            if sb != INF:
                put(glob, lds2, ("pubmin",) + base + (0,))
            else:
                if not own and cfg.helper_leaves:
                    put(glob, lds2, ("rel",) + base + (0,))
                if hold == 2:
                    if next_old & FOUND:
                        put(glob, lds2, ("rel",) + base + (0,))
                    else:
                        put(glob, lds2, ("dropone",) + base + (0,))
                else:
                    put(glob, lds2, ("claimnext",) + base + (0,))
        elif pc == "pubmin":
            put((np_, min(best, v), closed, err), lds,
                ("pubfound", r, have_next, next_old, next_r, held, v, claims, 0))
        elif pc == "pubfound":
            put((np_ | FOUND, best, closed, err), lds,
                ("rel", r, have_next, next_old, next_r, held, v, claims, 0))
        elif pc == "dropone":
            glob2 = (np_ - 1, best, closed, err)
            g3, l3, nxt, _ = _decide(cfg, k, next_old, next_r, glob2, lds)
            if nxt[0] == "release":
                put(g3, l3, ("rel", r, have_next, next_old, next_r, 1, v, claims, 0))
            else:
                put(g3, l3, ("top", r, have_next, next_old, next_r, 1, v, claims, 0))
        elif pc == "claimnext":
            old = np_
            glob2 = (np_ + (r << 32), best, closed, err)
            g3, l3, nxt, _ = _decide(cfg, k, old, r, glob2, lds)
            r2 = min(r * 2, cfg.rmax)
            if nxt[0] == "release":
                put(g3, l3, ("rel", r2, have_next, next_old, next_r, 1, v, claims + 1, 0))
            else:
                put(g3, l3, ("top", r2, have_next, next_old, next_r, 1, v, claims + 1, 0))
        elif pc == "exit":
            if fin:
                put(glob, lds, ("done", r, have_next, next_old, next_r, held, v, claims, 0),
                    fins + ((k, best),))
            else:
                put(glob, lds, ("done", r, have_next, next_old, next_r, held, v, claims, 0))
        # ---------------------------------------------------------- wave 1
        pc1, t1 = w1s[k]

        def put1(lds2, w1new, _k=k):
            out.append((glob, lds2, w0s, w1s[:_k] + (w1new,) + w1s[_k + 1:], fins))

        if pc1 == "top":
            a0, a1 = arr
            if a1 == 0:
                put1(setl((go, fin, first, rounds, sb, (a0, 1), gen)), ("b1wait", gen))
        elif pc1 == "b1wait":
            if gen != t1:
                put1(lds, ("readgo", 0))
        elif pc1 == "readgo":
            put1(lds, ("eval", 0) if go else ("exit", 0))
        elif pc1 == "eval":
            if t1 >= rounds:
                put1(lds, ("b2", 0) if cfg.b2 else ("top", 0))
            else:
                a = 2 * (first + t1) + 1
                if a >= sb:
                    put1(lds, ("b2", 0) if cfg.b2 else ("top", 0))
                elif a in cfg.valid:
                    put1(setl((go, fin, first, rounds, min(sb, a), arr, gen)),
                         ("b2", 0) if cfg.b2 else ("top", 0))
                else:
                    put1(lds, ("eval", t1 + 1))
        elif pc1 == "b2":
            a0, a1 = arr
            if a1 == 0:
                put1(setl((go, fin, first, rounds, sb, (a0, 1), gen)), ("b2wait", gen))
        elif pc1 == "b2wait":
            if gen != t1:
                put1(lds, ("top", 0))
        elif pc1 == "exit":
            put1(lds, ("done", 0))
        # ---------------------------------------------------------- barrier opens
        if arr == (1, 1) or (arr[0] == 1 and k and cfg.helper_waves == 1):
            lds2 = setl((go, fin, first, rounds, sb, (0, 0), gen + 1))
            out.append((glob, lds2, w0s, w1s, fins))
    return out


def explore(cfg, limit=3_000_000):
    """All reachable states; returns (final states, bad states with reasons)."""
    start = _initial(cfg)
    seen = {start}
    todo = deque([start])
    finals, bad = [], []
    valid_min = min(cfg.valid) if cfg.valid else None
    while todo:
        s = todo.popleft()
        nxt = _successors(cfg, s)
        if not nxt:
            glob, lds, w0s, w1s, fins = s
            done = all(w[0] == "done" for w in w0s) and all(w[0] == "done" for w in w1s)
            if not done:
                bad.append(("deadlock: waves wait for partners that left", s))
                continue
            finals.append(s)
            np_, best, closed, err = glob
            if err:
                continue  # the attempt cap ended the search: an error, no value
            if len(fins) != 1:
                bad.append((f"{len(fins)} finalizers", s))
            elif fins[0][1] != valid_min:
                bad.append((f"finalized {fins[0][1]}, smallest valid attempt {valid_min}", s))
            if not (np_ & FOUND):
                bad.append(("found bit lost", s))
            if np_ & MASK32:
                bad.append(("chunks still in flight at the end", s))
            continue
        for t in nxt:
            if t not in seen:
                seen.add(t)
                todo.append(t)
                if len(seen) > limit:
                    raise RuntimeError("state space larger than the limit")
    return finals, bad, len(seen)


CASES = [
    # (workers, waves per helper, valid attempts, rmax, cap rounds, owner claims ahead)
    (2, 2, {0}, 2, 4, True),
    (2, 2, {3}, 2, 4, True),
    (2, 2, {5}, 2, 5, True),
    (2, 2, {2, 5}, 2, 5, True),
    (2, 2, {4}, 1, 4, False),
    (2, 2, {6}, 2, 5, False),
    (3, 1, {3}, 1, 3, True),
    (3, 1, {2, 4}, 2, 4, False),
]


@pytest.mark.parametrize("workers,hwaves,valid,rmax,cap,ahead", CASES)
def test_claim_protocol_all_interleavings(workers, hwaves, valid, rmax, cap, ahead):
    cfg = Config(workers, valid, rmax=rmax, cap_rounds=cap, owner_ahead=ahead,
                 helper_waves=hwaves)
    finals, bad, n = explore(cfg)
    assert not bad, bad[0][0]
    assert finals, "no final state reached"
    # some interleavings end with the value, not only by the attempt cap
    assert any(f[0][3] == 0 for f in finals)


def test_model_finds_a_finalize_without_the_found_bit():
    """A drop that finalizes whenever the in-flight count reaches zero (found
    bit ignored) lets a worker close the task between two chunks, before any
    value exists: the model reaches a state that finalizes a wrong value."""
    cfg = Config(2, {3}, rmax=1, cap_rounds=4, owner_ahead=False, found_check=False)
    _, bad, _ = explore(cfg)
    assert any("finalized" in reason or "finalizers" in reason for reason, _ in bad)


def test_model_finds_the_missing_barrier():
    """Without the barrier between the chunk's evaluation and thread 0's
    rewrite of the decision, a wave can evaluate past a value that thread 0
    has already consumed, or read the next decision: a bad state exists."""
    cfg = Config(2, {3}, rmax=2, cap_rounds=4, owner_ahead=True, b2=False)
    _, bad, _ = explore(cfg)
    assert bad
