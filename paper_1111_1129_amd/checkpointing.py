"""Binomial ("revolve") checkpointing for the reverse sweep of the adjoint.

Reversing T forward steps needs the state entering every step, in reverse
order.  With c snapshot slots besides the stored initial state, the fewest
forward steps that deliver them follow from the recursion

    F(1, c) = 0,    F(l, 0) = l (l - 1) / 2,
    F(l, c) = min over 1 <= m < l of  m + F(l - m, c - 1) + F(m, c),

(advance m steps and keep that state in a slot, reverse the last l - m steps
with one slot fewer, free the slot, reverse the first m steps), whose value
is Griewank and Walther's optimal count for binomial checkpointing (Algorithm
799, "revolve", ACM TOMS 2000): with c + 1 checkpoints counting the initial
one and r the least integer with C(c + 1 + r, c + 1) >= l,
F(l, c) = r l - C(c + 1 + r, c + 2).

This module holds the table and a schedule walker that calls back for the
two actions (advance a state from one slot into another, take one adjoint
step); it does no arithmetic of the method and touches no device memory
itself.
"""
from __future__ import annotations

import math

import numpy as np


def forward_cost_table(T: int, c_max: int) -> tuple[np.ndarray, np.ndarray]:
    """(F, split): F[l, c] = fewest forward steps to reverse l steps with c
    free slots, split[l, c] = the first advance m that attains it (0 where
    l <= 1 or c = 0), for 0 <= l <= T, 0 <= c <= c_max."""
    F = np.zeros((T + 1, c_max + 1), dtype=np.int64)
    split = np.zeros((T + 1, c_max + 1), dtype=np.int64)
    ls = np.arange(T + 1, dtype=np.int64)
    F[:, 0] = ls * (ls - 1) // 2
    F[0, 0] = 0
    for c in range(1, c_max + 1):
        for l in range(2, T + 1):
            m = np.arange(1, l, dtype=np.int64)
            cost = m + F[l - m, c - 1] + F[m, c]
            k = int(np.argmin(cost))  # the smallest advance among the optima
            F[l, c] = cost[k]
            split[l, c] = m[k]
    return F, split


def revolve_closed_form(l: int, checkpoints: int) -> int:
    """Griewank and Walther's minimal number of forward steps to reverse l
    steps with `checkpoints` checkpoints (the initial state included, >= 1)."""
    if l <= 1:
        return 0
    c = checkpoints
    r = 0
    while math.comb(c + r, c) < l:
        r += 1
    return r * l - math.comb(c + r, c + 1)


class Revolve:
    """Schedule for reversing T steps with `slots` snapshot slots (plus the
    slot holding the initial state).

    run(advance, adjoint) drives it:
      advance(src, dst, t, k) the state at time t in slot src -> time t + k in
                              slot dst (src != dst; src is left unchanged)
      adjoint(slot, t)        one adjoint step of step t from the state at time t
    Slot 0 holds the initial state on entry and is never overwritten; slot
    `slots + 1` is the work slot used when no snapshot slot is left.  The
    adjoint steps come in the order T - 1, ..., 0, and advance is asked for
    exactly forward_steps steps in total."""

    def __init__(self, T: int, slots: int):
        assert T >= 0 and slots >= 0
        self.T, self.slots = T, slots
        self.F, self.split = forward_cost_table(max(T, 1), slots)
        self.forward_steps = int(self.F[T, slots]) if T > 0 else 0

    def run(self, advance, adjoint):
        work = self.slots + 1
        free = list(range(self.slots, 0, -1))

        def reverse(a: int, b: int, slot: int):
            l = b - a
            if l <= 0:
                return
            if l == 1:
                adjoint(slot, a)
                return
            if not free:
                # no slot left: recompute every state from the one at a
                for t in range(b - 1, a - 1, -1):
                    if t == a:
                        adjoint(slot, a)
                    else:
                        advance(slot, work, a, t - a)
                        adjoint(work, t)
                return
            m = int(self.split[l, len(free)])
            s = free.pop()
            advance(slot, s, a, m)
            reverse(a + m, b, s)
            free.append(s)
            reverse(a, a + m, slot)

        reverse(0, self.T, 0)
