"""Pins of the Game-of-Life oracle (thesis Ch.7 "gol", rule B3/S23).

The oracle runs the SMMO decomposition (Cell::count, Alive::death,
Cell::birth over Cell and Alive objects).  It is pinned to facts that do not
come from it: well-known still lifes, oscillators and the glider; the
birth/survival rule table stated in the thesis over all 512 neighbourhoods;
and brute force against a plain array stencil on every 4x4 torus and on
random 8x8 tori.
"""

import numpy as np
import pytest

from oracle import GolWorld


def grid(W, H, cells):
    g = np.zeros((H, W), np.uint8)
    for (x, y) in cells:
        g[y, x] = 1
    return g


def run(g, n):
    H, W = g.shape
    w = GolWorld(W, H, g.reshape(-1))
    w.step(n)
    st, ct, al = w.read()
    assert np.array_equal(np.flatnonzero(st), al), "Alive set must equal the live cells"
    return st.reshape(H, W)


def stencil_step(g):
    """Independent array implementation (neighbour sum by torus rolls)."""
    n = sum(np.roll(np.roll(g, dy, 0), dx, 1)
            for dy in (-1, 0, 1) for dx in (-1, 0, 1) if dx or dy)
    return (((g == 1) & ((n == 2) | (n == 3))) | ((g == 0) & (n == 3))).astype(np.uint8)


@pytest.mark.parametrize("cells", [
    [(3, 3), (4, 3), (3, 4), (4, 4)],                               # block
    [(4, 3), (5, 3), (3, 4), (6, 4), (4, 5), (5, 5)],               # beehive
    [(4, 3), (5, 3), (3, 4), (6, 4), (4, 5), (6, 5), (5, 6)],       # loaf
])
def test_still_lifes(cells):
    g = grid(10, 10, cells)
    for n in (1, 2, 7):
        assert np.array_equal(run(g, n), g)


@pytest.mark.parametrize("cells", [
    [(4, 5), (5, 5), (6, 5)],                                       # blinker
    [(4, 4), (5, 4), (6, 4), (3, 5), (4, 5), (5, 5)],               # toad
    [(2, 2), (3, 2), (2, 3), (5, 4), (4, 5), (5, 5)],               # beacon
])
def test_period_two_oscillators(cells):
    g = grid(10, 10, cells)
    g1 = run(g, 1)
    assert not np.array_equal(g1, g)
    assert np.array_equal(run(g, 2), g)
    assert np.array_equal(run(g, 10), g)


def test_blinker_phases():
    g = grid(7, 7, [(2, 3), (3, 3), (4, 3)])
    assert np.array_equal(run(g, 1), grid(7, 7, [(3, 2), (3, 3), (3, 4)]))


def test_glider_moves_one_diagonal_cell_every_four_generations():
    # glider heading towards +x, +y
    cells = [(1, 0), (2, 1), (0, 2), (1, 2), (2, 2)]
    g = grid(16, 16, cells)
    g4 = run(g, 4)
    assert np.array_equal(g4, np.roll(np.roll(g, 1, 0), 1, 1))
    # on a 16x16 torus it returns after 4*16 generations
    assert np.array_equal(run(g, 64), g)


def test_glider_returns_on_256_torus():
    cells = [(101, 100), (102, 101), (100, 102), (101, 102), (102, 102)]
    g = grid(256, 256, cells)
    assert np.array_equal(run(g, 1024), g)


def test_rule_table_all_512_neighbourhoods():
    # birth with exactly three live neighbours, survival with two or three
    for code in range(512):
        bits = np.array([(code >> i) & 1 for i in range(9)], np.uint8).reshape(3, 3)
        g = np.zeros((5, 5), np.uint8)
        g[1:4, 1:4] = bits
        centre = bits[1, 1]
        nb = int(bits.sum()) - int(centre)
        expect = 1 if (nb == 3 or (centre == 1 and nb == 2)) else 0
        assert run(g, 1)[2, 2] == expect, code


def test_exhaustive_4x4_tori_one_step():
    for code in range(1 << 16):
        g = np.array([(code >> i) & 1 for i in range(16)], np.uint8).reshape(4, 4)
        assert np.array_equal(run(g, 1), stencil_step(g)), code


def test_random_8x8_tori_100_steps():
    rng = np.random.default_rng(8)
    for t in range(2000):
        g = (rng.random((8, 8)) < 0.35).astype(np.uint8)
        ref = g
        for _ in range(100):
            ref = stencil_step(ref)
        assert np.array_equal(run(g, 100), ref), t


def test_counts_are_neighbour_sums():
    rng = np.random.default_rng(3)
    g = (rng.random((13, 11)) < 0.4).astype(np.uint8)
    w = GolWorld(11, 13, g.reshape(-1))
    w.step(1)
    _, ct, _ = w.read()
    n = sum(np.roll(np.roll(g, dy, 0), dx, 1)
            for dy in (-1, 0, 1) for dx in (-1, 0, 1) if dx or dy)
    assert np.array_equal(ct.reshape(13, 11), n)


def test_rectangular_and_degenerate_tori():
    rng = np.random.default_rng(5)
    for (W, H) in [(1, 1), (1, 7), (7, 1), (2, 2), (3, 5), (37, 23)]:
        g = (rng.random((H, W)) < 0.4).astype(np.uint8)
        ref = g
        for _ in range(5):
            ref = stencil_step(ref)
        assert np.array_equal(run(g, 5), ref), (W, H)
