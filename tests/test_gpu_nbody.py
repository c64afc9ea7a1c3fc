"""GPU parity of n-body (thesis Ch.7 "nbody") against the float64 oracle.

Per checked step k the GPU's float32 state is read back; the oracle takes
exactly those values and computes one step in float64.  Tolerance (1e-5 per
step, relative to the conditioning scale of each quantity):
  force    |f_gpu - f_ref| <= 1e-5 * sum_j |term_ij|
  velocity |v_gpu - v_ref| <= 1e-5 * (|v_k| + dt * S_f / m)
  position |x_gpu - x_ref| <= 1e-5 * (|x_k| + dt * S_v)
"""

import numpy as np
import pytest

from inputs import nbody_init
from oracle import nbody_force_at, nbody_steps, nbody_update
from paper_1908_05845_amd.sims import NbodySim

pytestmark = pytest.mark.gpu

TOL = 1e-5


def check_force(s0, f, G, eps, idx):
    fx, fy, sx, sy = nbody_force_at(s0["x"], s0["y"], s0["m"], G, eps, idx)
    ex = np.abs(f["fx"][idx] - fx)
    ey = np.abs(f["fy"][idx] - fy)
    assert np.all(ex <= TOL * sx), float(np.max(ex / sx))
    assert np.all(ey <= TOL * sy), float(np.max(ey / sy))
    return sx, sy


def check_full_step(sim, G, eps, dt, sample=None):
    s0 = sim.read()
    n = s0["x"].size
    idx = np.arange(n) if sample is None else sample
    sim.force()
    f = sim.read()
    sx, sy = check_force(s0, f, G, eps, idx)
    sim.update()
    s1 = sim.read()
    # update from the GPU's own forces, every body
    up = nbody_update(s0["x"], s0["y"], s0["vx"], s0["vy"], f["fx"], f["fy"], s0["m"], dt)
    svx = np.abs(s0["vx"]) + dt * np.abs(f["fx"]) / s0["m"]
    svy = np.abs(s0["vy"]) + dt * np.abs(f["fy"]) / s0["m"]
    assert np.all(np.abs(s1["vx"] - up["vx"]) <= TOL * svx)
    assert np.all(np.abs(s1["vy"] - up["vy"]) <= TOL * svy)
    assert np.all(np.abs(s1["x"] - up["x"]) <= TOL * (np.abs(s0["x"]) + dt * svx))
    assert np.all(np.abs(s1["y"] - up["y"]) <= TOL * (np.abs(s0["y"]) + dt * svy))
    # one full oracle step from the same state, on the checked bodies
    if sample is None:
        ref = nbody_steps(s0["x"], s0["y"], s0["vx"], s0["vy"], s0["m"], G, eps, dt, 1)
        Svx = np.abs(s0["vx"]) + dt * ref["sfx"] / s0["m"]
        Svy = np.abs(s0["vy"]) + dt * ref["sfy"] / s0["m"]
        assert np.all(np.abs(s1["vx"] - ref["vx"]) <= TOL * Svx)
        assert np.all(np.abs(s1["vy"] - ref["vy"]) <= TOL * Svy)
        assert np.all(np.abs(s1["x"] - ref["x"]) <= TOL * (np.abs(s0["x"]) + dt * Svx))
        assert np.all(np.abs(s1["y"] - ref["y"]) <= TOL * (np.abs(s0["y"]) + dt * Svy))


@pytest.mark.parametrize("n", [1, 2, 63, 1000, 3000])
def test_small_every_body_every_step(dev, n):
    print("nbody n=%d" % n, flush=True)
    st = nbody_init(n, seed=100 + n)
    G, eps, dt = 1.0 / max(n, 1), 1e-3, 1e-4
    sim = NbodySim(st, G, eps, dt)
    for _ in range(4):
        check_full_step(sim, G, eps, dt)


def test_unsoftened_force_skips_self(dev):
    st = nbody_init(500, seed=9)
    sim = NbodySim(st, 1.0 / 500, 0.0, 1e-5)
    check_full_step(sim, 1.0 / 500, 0.0, 1e-5)
    assert np.all(np.isfinite(sim.read()["fx"]))


def test_config_65536_bodies_sampled(dev):
    print("nbody 65536", flush=True)
    n = 65536
    G, eps, dt = 1.0 / n, 1e-3, 1e-4
    sim = NbodySim(nbody_init(n), G, eps, dt)
    rng = np.random.default_rng(5)
    for step in range(50):
        if step in (0, 1, 25, 49):
            sample = np.sort(rng.choice(n, 384, replace=False))
            sample[0], sample[-1] = 0, n - 1
            check_full_step(sim, G, eps, dt, sample=sample)
        else:
            sim.step(1)
    # momentum stays near zero (started at rest): a property at any size
    s = sim.read()
    p = np.array([np.sum(s["m"] * s["vx"]), np.sum(s["m"] * s["vy"])])
    assert np.all(np.abs(p) <= 1e-4 * np.sum(s["m"] * np.hypot(s["vx"], s["vy"])))
