"""Binomial checkpointing schedule of the adjoint's reverse sweep (host logic,
no GPU): the optimal forward-step counts against Griewank and Walther's
closed form, and the schedule replayed on integer "states"."""
import math

import pytest

from paper_1111_1129_amd.checkpointing import Revolve, forward_cost_table, revolve_closed_form


def test_closed_form_small_values_by_hand():
    # one checkpoint (the initial state): every state recomputed from t = 0
    assert revolve_closed_form(5, 1) == 0 + 1 + 2 + 3 + 4
    # l = 3 with one snapshot besides the initial state: advance 1, keep it,
    # reverse step 2 from it (1 more step), step 1 from it, step 0 from t = 0
    assert revolve_closed_form(3, 2) == 2
    # enough checkpoints for every state: each step computed once, the last
    # state is never needed (the adjoint of step l - 1 starts from state l - 1)
    assert revolve_closed_form(10, 10) == 9
    assert revolve_closed_form(1, 1) == 0


def test_dynamic_program_equals_the_closed_form():
    F, split = forward_cost_table(120, 8)
    for l in range(1, 121):
        for c in range(0, 9):
            assert F[l, c] == revolve_closed_form(l, c + 1), (l, c)
            if l >= 2 and c >= 1:
                m = split[l, c]
                assert 1 <= m < l
                assert F[l, c] == m + F[l - m, c - 1] + F[m, c]


def replay(T, slots):
    """Run the schedule on integer states; return (adjoint order, forward
    steps, largest slot index, most slots live at once)."""
    plan = Revolve(T, slots)
    state = {0: 0}
    order, fwd, top = [], [0], [0]

    def advance(src, dst, t, k):
        assert dst != 0, "the initial state is never overwritten"
        assert src != dst and state[src] == t and k >= 1
        state[dst] = t + k
        fwd[0] += k
        top[0] = max(top[0], dst)

    def adjoint(slot, t):
        assert state[slot] == t
        order.append(t)

    plan.run(advance, adjoint)
    assert state[0] == 0
    return order, fwd[0], top[0], plan.forward_steps


@pytest.mark.parametrize("T,slots", [(0, 0), (1, 0), (2, 0), (6, 0), (7, 1), (23, 3), (50, 4),
                                     (100, 7), (500, 10), (500, 45)])
def test_schedule_delivers_every_state_in_reverse(T, slots):
    order, fwd, top, planned = replay(T, slots)
    assert order == list(range(T - 1, -1, -1))
    assert fwd == planned
    if T >= 1:
        assert fwd == revolve_closed_form(T, slots + 1)
    assert top <= slots + 1  # the snapshot slots and the work slot


def test_more_memory_never_costs_more_recomputation():
    F, _ = forward_cost_table(300, 12)
    for l in range(1, 301):
        assert all(F[l, c + 1] <= F[l, c] for c in range(12))
    # with as many slots as steps every state is computed once
    assert F[300, 12] >= 299
    r = next(r for r in range(20) if math.comb(13 + r, 13) >= 300)
    assert F[300, 12] == r * 300 - math.comb(13 + r, 14)
