"""Pins of the n-body oracle (thesis Ch.7 "nbody": gravitational force
F = G m1 m2 / r^2, then v += F/m dt and x += v dt).

Pinned by hand-computed steps with exactly representable results, by the
softened two-body circular orbit (closed form of the angular velocity), by
momentum conservation, pairwise antisymmetry and translation invariance.
"""

import math

import numpy as np

from oracle import nbody_force_at, nbody_steps, nbody_update


def test_single_body_feels_no_force():
    r = nbody_steps([0.3], [-0.2], [0.5], [0.25], [2.0], G=1.0, eps=1e-3, dt=0.5, steps=3)
    assert r["fx"][0] == 0 and r["fy"][0] == 0
    assert r["x"][0] == 0.3 + 3 * 0.25 and r["y"][0] == -0.2 + 3 * 0.125


def test_two_bodies_hand_computed_unsoftened():
    # bodies at x = -1 and x = +1, unit masses, G = 1: |F| = 1/2^2 = 0.25
    # dt = 0.5: v = +-0.125, x = -1 + 0.0625
    r = nbody_steps([-1.0, 1.0], [0.0, 0.0], [0.0, 0.0], [0.0, 0.0], [1.0, 1.0],
                    G=1.0, eps=0.0, dt=0.5)
    assert r["fx"].tolist() == [0.25, -0.25]
    assert r["vx"].tolist() == [0.125, -0.125]
    assert r["x"].tolist() == [-0.9375, 0.9375]
    assert r["y"].tolist() == [0.0, 0.0]


def test_two_bodies_hand_computed_softened():
    # separation 3, softening 4: (9 + 16)^(3/2) = 125; masses 2 and 5, G = 1
    # force on body 0 = 2*5*3/125 = 0.24 towards body 1
    r = nbody_steps([0.0, 3.0], [1.0, 1.0], [0.0, 0.0], [0.0, 0.0], [2.0, 5.0],
                    G=1.0, eps=4.0, dt=1.0)
    assert abs(r["fx"][0] - 0.24) < 1e-15 and abs(r["fx"][1] + 0.24) < 1e-15
    assert abs(r["vx"][0] - 0.12) < 1e-15 and abs(r["vx"][1] + 0.048) < 1e-15


def test_pairwise_antisymmetry():
    # Newton's third law: equal and opposite, up to the rounding of G*m_i*m_j
    rng = np.random.default_rng(1)
    for _ in range(50):
        x, y = rng.random(2), rng.random(2)
        m = 0.5 + rng.random(2)
        fx, fy, _, _ = nbody_force_at(x, y, m, 0.7, 1e-3, [0, 1])
        assert abs(fx[0] + fx[1]) <= 1e-15 * abs(fx[0])
        assert abs(fy[0] + fy[1]) <= 1e-15 * abs(fy[0])


def test_momentum_conserved():
    rng = np.random.default_rng(2)
    n = 300
    x, y = rng.random(n), rng.random(n)
    vx, vy = 0.01 * rng.standard_normal(n), 0.01 * rng.standard_normal(n)
    m = 0.5 + rng.random(n)
    p0 = np.array([np.sum(m * vx), np.sum(m * vy)])
    r = nbody_steps(x, y, vx, vy, m, G=1.0 / n, eps=1e-3, dt=1e-4, steps=20)
    p1 = np.array([np.sum(m * r["vx"]), np.sum(m * r["vy"])])
    scale = np.sum(m * np.hypot(r["vx"], r["vy"]))
    assert np.all(np.abs(p1 - p0) <= 1e-12 * scale)


def test_translation_invariance():
    rng = np.random.default_rng(3)
    n = 100
    x, y, m = rng.random(n), rng.random(n), 0.5 + rng.random(n)
    idx = np.arange(n)
    f0 = nbody_force_at(x, y, m, 1.0 / n, 1e-3, idx)
    f1 = nbody_force_at(x + 0.5, y - 0.25, m, 1.0 / n, 1e-3, idx)
    for a, b, s in ((f0[0], f1[0], f0[2]), (f0[1], f1[1], f0[3])):
        assert np.all(np.abs(a - b) <= 1e-12 * s)


def test_circular_two_body_orbit():
    # equal masses m at separation D orbit their centre at radius D/2 when
    # m w^2 D/2 = G m^2 D / (D^2 + eps^2)^(3/2)
    G, m, D, eps = 1.0, 1.0, 1.0, 0.1
    w = math.sqrt(2 * G * m / (D * D + eps * eps) ** 1.5)
    v = w * D / 2
    T = 2 * math.pi / w
    steps = 20000
    dt = (T / 4) / steps
    r = nbody_steps([-D / 2, D / 2], [0.0, 0.0], [0.0, 0.0], [-v, v], [m, m],
                    G=G, eps=eps, dt=dt, steps=steps)
    # after a quarter period body 1 sits at (0, D/2) and body 0 at (0, -D/2)
    sep = math.hypot(r["x"][1] - r["x"][0], r["y"][1] - r["y"][0])
    assert abs(sep - D) < 1e-4
    ang = math.atan2(r["y"][1], r["x"][1])
    assert abs(ang - math.pi / 2) < 1e-3


def test_sampled_force_equals_full_step_force():
    rng = np.random.default_rng(4)
    n = 257
    x, y, m = rng.random(n), rng.random(n), 0.5 + rng.random(n)
    z = np.zeros(n)
    r = nbody_steps(x, y, z, z, m, G=1.0 / n, eps=1e-3, dt=1e-4)
    idx = np.array([0, 5, 256, 100])
    fx, fy, sx, sy = nbody_force_at(x, y, m, 1.0 / n, 1e-3, idx)
    assert np.array_equal(fx, r["fx"][idx]) and np.array_equal(fy, r["fy"][idx])
    assert np.all(sx >= np.abs(fx)) and np.all(sy >= np.abs(fy))


def test_update_alone_matches_full_step():
    rng = np.random.default_rng(6)
    n = 50
    x, y, m = rng.random(n), rng.random(n), 0.5 + rng.random(n)
    vx, vy = 0.1 * rng.standard_normal(n), 0.1 * rng.standard_normal(n)
    full = nbody_steps(x, y, vx, vy, m, G=0.3, eps=1e-2, dt=1e-3)
    up = nbody_update(x, y, vx, vy, full["fx"], full["fy"], m, dt=1e-3)
    for k in ("x", "y", "vx", "vy"):
        assert np.array_equal(up[k], full[k])
    # worked example: f = 2, m = 4, dt = 0.5 -> v = 0.25, x = 1 + 0.125
    r = nbody_update([1.0], [0.0], [0.0], [0.0], [2.0], [0.0], [4.0], dt=0.5)
    assert r["vx"][0] == 0.25 and r["x"][0] == 1.125
