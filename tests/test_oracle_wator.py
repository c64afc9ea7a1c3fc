"""Pins of the wa-tor oracle (thesis Ch.7 "wa-tor").

The oracle keeps Cell, Fish and Shark objects and runs the eight do-alls of
an iteration.  It is checked against:
  * hand-worked cases: a lone fish's move (its direction drawn from an
    independent splitmix64 implementation), a fish that cannot move, a
    shark's starvation time, a fish's first spawn, four sharks contending
    for one fish;
  * a brute-force version written on per-cell arrays (no objects, no
    handles, no snapshots) from the same rules, every iteration, on random
    small tori;
  * bookkeeping invariants (one agent per occupied cell, counts).
"""

import numpy as np
import pytest

from inputs import config_seed, wator_init
from inputs.rng import raw
from oracle import WatorWorld

SEED = config_seed(7)


def nbrs(i, W, H):
    x, y = i % W, i // W
    return [((y - 1) % H) * W + x, y * W + (x + 1) % W, ((y + 1) % H) * W + x, y * W + (x - 1) % W]


def pick(seed, stream, cell, n):
    return int(raw(seed, stream, [cell])[0] % np.uint64(n))


def brute_iteration(W, H, seed, t, prm, kind, timer, energy):
    """One iteration on per-cell arrays, straight from the rules."""
    fs, ss, e0, boost = prm
    N = W * H
    kind, timer, energy = kind.copy(), timer.copy(), energy.copy()
    for ak, phase in ((1, 0), (2, 2)):
        agents = [c for c in range(N) if kind[c] == ak]
        for c in agents:
            timer[c] += 1
            if ak == 2:
                energy[c] -= 1
        req = np.zeros((N, 5), bool)
        for c in agents:
            nb = nbrs(c, W, H)
            cand = [i for i in range(4) if kind[nb[i]] == 1] if ak == 2 else []
            if not cand:
                cand = [i for i in range(4) if kind[nb[i]] == 0]
            if not cand:
                req[c, 4] = True
            else:
                s = cand[pick(seed, 4 * t + phase, c, len(cand))]
                req[nb[s], (s + 2) % 4] = True
        target = {c: c for c in agents}
        for c in range(N):
            if req[c, 4]:
                continue
            cand = [i for i in range(4) if req[c, i]]
            if cand:
                s = cand[pick(seed, 4 * t + phase + 1, c, len(cand))]
                target[nbrs(c, W, H)[s]] = c
        nk, nt, ne = kind.copy(), timer.copy(), energy.copy()
        for c in agents:
            if ak == 2 and energy[c] <= 0:
                nk[c], nt[c], ne[c] = 0, 0, 0
                continue
            d = target[c]
            if d == c:
                continue
            en = energy[c] + (boost if ak == 2 and kind[d] == 1 else 0)
            thr = fs if ak == 1 else ss
            if timer[c] > thr:
                nk[d], nt[d], ne[d] = ak, 0, en if ak == 2 else 0
                nk[c], nt[c], ne[c] = ak, 0, e0 if ak == 2 else 0
            else:
                nk[d], nt[d], ne[d] = ak, timer[c], en if ak == 2 else 0
                nk[c], nt[c], ne[c] = 0, 0, 0
        kind, timer, energy = nk, nt, ne
    return kind, timer, energy


def empty(W, H):
    return {"kind": np.zeros(W * H, np.uint8), "timer": np.zeros(W * H, np.int32),
            "energy": np.zeros(W * H, np.int32)}


def test_lone_fish_moves_to_the_drawn_neighbour():
    W = H = 3
    init = empty(W, H)
    init["kind"][4] = 1
    w = WatorWorld(W, H, SEED, (4, 12, 8, 4), init)
    w.step(1)
    kind, timer, _, counts = w.read()
    # four empty neighbours, candidates in direction order; only one request,
    # so the target cell grants it
    want = nbrs(4, W, H)[pick(SEED, 0, 4, 4)]
    assert counts == (1, 0)
    assert np.flatnonzero(kind).tolist() == [want] and timer[want] == 1


def test_fish_without_empty_neighbour_stays():
    W = H = 3
    init = empty(W, H)
    init["kind"][:] = 1
    w = WatorWorld(W, H, SEED, (4, 12, 8, 4), init)
    w.step(3)
    kind, timer, _, counts = w.read()
    assert counts == (9, 0) and np.all(kind == 1) and np.all(timer == 3)


def test_shark_starves_after_energy0_iterations():
    W = H = 5
    init = empty(W, H)
    init["kind"][12] = 2
    init["energy"][12] = 3
    w = WatorWorld(W, H, SEED, (4, 12, 3, 4), init)
    w.step(2)
    kind, _, energy, counts = w.read()
    assert counts == (0, 1) and energy[kind == 2].tolist() == [1]
    w.step(1)
    assert w.read()[3] == (0, 0)


def test_fish_spawns_when_it_moves_after_the_threshold():
    W = H = 9
    init = empty(W, H)
    init["kind"][40] = 1
    w = WatorWorld(W, H, SEED, (2, 12, 8, 4), init)
    w.step(2)
    assert w.read()[3] == (1, 0)
    w.step(1)             # timer reaches 3 > 2 in this iteration's prepare
    kind, timer, _, counts = w.read()
    assert counts == (2, 0) and timer[kind == 1].tolist() == [0, 0]


def test_four_sharks_contend_for_one_fish():
    W = H = 3
    init = empty(W, H)
    init["kind"][4] = 1
    for c in (1, 3, 5, 7):
        init["kind"][c] = 2
        init["energy"][c] = 5
    w = WatorWorld(W, H, SEED, (4, 12, 5, 4), init)
    w.step(1)
    kind, timer, energy, counts = w.read()
    # the fish cannot move; every shark asks for the fish's cell, which
    # grants one requester drawn on stream 3 at cell 4
    winner = nbrs(4, W, H)[pick(SEED, 3, 4, 4)]
    assert counts == (0, 4)
    assert kind[4] == 2 and energy[4] == 5 - 1 + 4 and kind[winner] == 0
    for c in (1, 3, 5, 7):
        if c != winner:
            assert kind[c] == 2 and energy[c] == 4


@pytest.mark.parametrize("W,H,prm,seed", [(7, 5, (2, 5, 4, 3), 1), (8, 8, (3, 6, 5, 2), 2),
                                          (16, 9, (4, 12, 8, 4), 3), (1, 6, (1, 3, 3, 2), 4)])
def test_matches_brute_force_every_iteration(W, H, prm, seed):
    init = wator_init(W, H, seed=seed, p_fish=0.35, p_shark=0.1, fish_spawn=prm[0], shark_spawn=prm[1],
                      energy0=prm[2])
    w = WatorWorld(W, H, seed, prm, init)
    kind, timer, energy = init["kind"].copy(), init["timer"].copy(), init["energy"].copy()
    for t in range(60):
        kind, timer, energy = brute_iteration(W, H, seed, t, prm, kind, timer, energy)
        w.step(1)
        k, tm, en, counts = w.read()
        assert np.array_equal(k, kind), t
        assert np.array_equal(tm, timer), t
        assert np.array_equal(en, energy), t
        assert counts == (int((kind == 1).sum()), int((kind == 2).sum()))
