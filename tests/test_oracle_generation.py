"""Pins of the generation oracle (thesis Ch.7 "generation": Game of Life
with dying cells, rule Burst 0235678/3468/255).

The rule table is checked exhaustively on a 3 x 3 torus, where the eight
neighbours of a cell are the eight other cells: for every live-neighbour
count 0..8 and every state of the centre, with dying neighbours mixed in
(they must not count), against the survive and birth sets the thesis states.
Further pins: the dying countdown (blocked for exactly D generations, no
birth into a dying cell), a lone live cell that survives forever (0 is in the
survive set), a full torus that stays full, and a domino that dies without
offspring and is gone after D generations.
"""

import itertools

import numpy as np
import pytest

from oracle import generation_steps

# the thesis's statement of the rule
SURVIVE = {0, 2, 3, 5, 6, 7, 8}
BIRTH = {3, 4, 6, 8}


@pytest.mark.parametrize("centre", ["empty", "live", "dying3", "dying1"])
def test_rule_table_on_3x3_torus(centre):
    rng = np.random.default_rng(7)
    for count in range(9):
        for trial in range(4):
            others = np.zeros(8, np.uint8)
            others[rng.choice(8, count, replace=False)] = 1
            # some of the non-live neighbours are dying: they must not count
            free = np.flatnonzero(others == 0)
            dying = free[rng.random(free.size) < 0.5]
            others[dying] = 2
            state = np.insert(others, 4, 0).astype(np.uint8)
            left = np.where(state == 2, 5, 0).astype(np.int32)
            if centre == "live":
                state[4] = 1
            elif centre.startswith("dying"):
                state[4] = 2
                left[4] = int(centre[5:])
            s, lf = generation_steps(3, 3, state, left, 1, dying=10)
            if centre == "empty":
                assert s[4] == (1 if count in BIRTH else 0), (count, trial)
            elif centre == "live":
                want = 1 if count in SURVIVE else 2
                assert s[4] == want and lf[4] == (0 if want == 1 else 10), (count, trial)
            elif centre == "dying3":
                assert s[4] == 2 and lf[4] == 2, count          # still blocked, whatever the count
            else:
                assert s[4] == 0 and lf[4] == 0, count          # its last dying generation
            # the dying neighbours count down
            assert np.all(lf[np.flatnonzero(state == 2)[np.flatnonzero(state == 2) != 4]] == 4)


@pytest.mark.parametrize("D", [1, 3, 255])
def test_domino_dies_without_offspring_and_expires(D):
    W = H = 12
    state = np.zeros(W * H, np.uint8)
    state[5 * W + 5] = state[5 * W + 6] = 1          # each has one live neighbour: 1 is not in S
    left = np.zeros(W * H, np.int32)
    s, lf = generation_steps(W, H, state, left, 1, dying=D)
    assert set(np.flatnonzero(s)) == {5 * W + 5, 5 * W + 6} and np.all(s[s > 0] == 2) and np.all(lf[s > 0] == D)
    # dead at step 1 with D left: still blocking after D steps (one left) ...
    s, lf = generation_steps(W, H, state, left, D, dying=D)
    assert s.sum() == 2 * 2 and np.all(lf[s > 0] == 1)
    # ... and gone after D + 1
    s, lf = generation_steps(W, H, state, left, D + 1, dying=D)
    assert s.sum() == 0 and lf.sum() == 0


def test_lone_cell_survives_and_full_torus_stays_full():
    W = H = 9
    state = np.zeros(W * H, np.uint8)
    state[40] = 1
    s, lf = generation_steps(W, H, state, np.zeros(W * H, np.int32), 25)
    assert np.array_equal(s, state) and lf.sum() == 0
    full = np.ones(W * H, np.uint8)
    s, lf = generation_steps(W, H, full, np.zeros(W * H, np.int32), 5)
    assert np.all(s == 1)


def test_birth_blocked_by_dying_cell():
    # the centre of a 5 x 5 torus is dying; three live cells around it would
    # give birth (3 is in B) to an empty centre, but not to a dying one
    W = H = 5
    state = np.zeros(W * H, np.uint8)
    left = np.zeros(W * H, np.int32)
    c = 2 * W + 2
    state[c], left[c] = 2, 4
    for i in (1 * W + 1, 1 * W + 2, 1 * W + 3):
        state[i] = 1
    s, lf = generation_steps(W, H, state, left, 1, dying=4)
    assert s[c] == 2 and lf[c] == 3
    state[c], left[c] = 0, 0
    s, _ = generation_steps(W, H, state, left, 1, dying=4)
    assert s[c] == 1


@pytest.mark.parametrize("W,H", [(16, 16), (7, 13), (1, 9), (32, 3)])
def test_invariants_on_random_tori(W, H):
    rng = np.random.default_rng(W * 100 + H)
    state = (rng.random(W * H) < 0.3).astype(np.uint8)
    left = np.zeros(W * H, np.int32)
    for _ in range(30):
        state, left = generation_steps(W, H, state, left, 1, dying=6)
        assert set(np.unique(state)) <= {0, 1, 2}
        assert np.array_equal(left > 0, state == 2) and left.max(initial=0) <= 6
    # stepping k times at once equals k single steps
    s0 = (rng.random(W * H) < 0.3).astype(np.uint8)
    a, la = generation_steps(W, H, s0, np.zeros(W * H, np.int32), 9, dying=6)
    b, lb = s0, np.zeros(W * H, np.int32)
    for _ in range(9):
        b, lb = generation_steps(W, H, b, lb, 1, dying=6)
    assert np.array_equal(a, b) and np.array_equal(la, lb)
