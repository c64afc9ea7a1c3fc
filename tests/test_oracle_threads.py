"""The oracle's parallel do-alls (methods that write only their own object,
run on host threads) give the same results, bit for bit, at one thread and
at eight: spring steps with springs breaking, n-body steps, the adjoint's
reverse sweep, and structure compute steps with breaking.  Each comparison
runs the same call twice, changing only the thread count."""

import numpy as np
import pytest

from inputs import nbody_init, spring_mesh, structure_mesh
from oracle import nbody_steps, set_threads, spring_adjoint, spring_steps, structure_pull, structure_step, threads


@pytest.fixture
def at_threads():
    before = threads()

    def run(n, fn):
        set_threads(n)
        try:
            return fn()
        finally:
            set_threads(before)
    return run


def same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        va, vb = np.atleast_1d(np.asarray(a[k])), np.atleast_1d(np.asarray(b[k]))
        assert va.dtype == vb.dtype and va.shape == vb.shape, k
        assert np.array_equal(np.ascontiguousarray(va).view(np.uint8), np.ascontiguousarray(vb).view(np.uint8)), k


def test_spring_steps_with_breaking(at_threads):
    mesh = spring_mesh(60, 40, seed=31, v_sigma=1.0)
    run = lambda: spring_steps(mesh, 1e-4, 0.3, 200)
    one, eight = at_threads(1, run), at_threads(8, run)
    assert one["nbroken"] > 0
    same(one, eight)


def test_nbody_steps(at_threads):
    s = nbody_init(700, seed=4)
    run = lambda: nbody_steps(s["x"], s["y"], s["vx"], s["vy"], s["m"], 1.0 / 700, 1e-3, 1e-4, 3)
    same(at_threads(1, run), at_threads(8, run))


def test_adjoint_sweep(at_threads):
    mesh = spring_mesh(20, 16, seed=8, v_sigma=0.5)
    run = lambda: spring_adjoint(mesh, 1e-3, 60, every=20)
    one, eight = at_threads(1, run), at_threads(8, run)
    assert np.any(one["gk"] != 0)
    same(one, eight)


def test_structure_steps_with_breaking(at_threads):
    mesh = structure_mesh(40, 16, seed=3, pull_speed=2.0, break_strain=0.02, v_sigma=0.05)
    S = np.asarray(mesh["p1"]).size
    start = dict(mesh, fx=np.zeros(S), fy=np.zeros(S), sdel=np.zeros(S, np.uint8))

    def run():
        cur = structure_pull(start, 30e-4)
        broken = 0
        for _ in range(30):
            cur = structure_step(cur, 1e-4)
            broken += cur["nbroken"]
        return cur, broken

    (one, b1), (eight, b8) = at_threads(1, run), at_threads(8, run)
    assert b1 > 0 and b1 == b8
    same(one, eight)
