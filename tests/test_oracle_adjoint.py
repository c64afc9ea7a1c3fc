"""Pins of the float64 adjoint oracle (reverse mode through the spring-mesh
step, breaking off, L = 1/2 sum |x_T - xhat|^2).

Pinned by a single-spring example whose loss is written out by hand as a
function of k, v0 and x0 (so its derivatives do not use the reverse
formulas), by central finite differences of the forward oracle on every
stiffness and initial velocity of an 8x8 mesh over 200 steps, and by the
checkpoint interval not changing any bit of the result.
"""

import numpy as np
import pytest

from inputs import spring_mesh
from oracle import spring_adjoint, spring_steps


def line2(x0b=1.5, k=2.0, L0=1.0):
    adj = -np.ones((2, 8), np.int32)
    adj[0, 0] = 0
    adj[1, 0] = 0
    adjb = np.zeros((2, 8), np.uint8)
    adjb[1, 0] = 1
    return dict(x=np.array([0.0, x0b]), y=np.zeros(2), vx=np.zeros(2), vy=np.zeros(2), m=np.ones(2),
                adj=adj, adj_is_b=adjb, a=np.array([0], np.int32), b=np.array([1], np.int32),
                k=np.array([k]), L0=np.array([L0]), slot_a=np.zeros(1, np.int32),
                slot_b=np.zeros(1, np.int32))


def test_single_spring_one_step_by_hand():
    # one step, dt = 1/2, m = 1: x1_a = dt^2 k (x0_b - x0_a - L0) = k/8 with the
    # nodes at 0 and 1.5, x1_b = 1.5 - k/8, so with xhat = x0:
    #   L(k) = (k/8)^2 = k^2/64 -> L = 1/16, dL/dk = k/32 = 1/16 at k = 2
    #   dL/dv0_a = (x1_a - xhat_a) * dt = 1/8, dL/dv0_b = -1/8
    #   dL/dx0_a = (x1_a - xhat_a)(1 - dt^2 k) + (x1_b - xhat_b) dt^2 k = 0
    r = spring_adjoint(line2(), dt=0.5, steps=1, every=1)
    assert r["loss"] == 0.0625
    assert r["gk"][0] == 0.0625
    assert r["gvx"].tolist() == [0.125, -0.125]
    assert r["gx"].tolist() == [0.0, 0.0]
    assert r["gvy"].tolist() == [0.0, 0.0] and r["gy"].tolist() == [0.0, 0.0]


def test_zero_steps():
    m = line2()
    xh = np.array([0.5, 1.0])
    r = spring_adjoint(m, dt=0.1, steps=0, xhat=xh, yhat=np.zeros(2))
    assert r["gk"][0] == 0.0 and r["gvx"].tolist() == [0.0, 0.0]
    assert r["gx"].tolist() == [-0.5, 0.5]


def _loss(mesh, dt, steps, xh, yh):
    r = spring_steps(mesh, dt, 1e30, steps)
    assert r["nbroken"] == 0
    return 0.5 * np.sum((r["x"] - xh) ** 2 + (r["y"] - yh) ** 2)


def _as64(m):
    return {k: (v.astype(np.float64) if isinstance(v, np.ndarray) and v.dtype == np.float32 else v)
            for k, v in m.items()}


def test_finite_differences_8x8_200_steps():
    mesh = _as64(spring_mesh(8, 8, seed=31, v_sigma=0.5))
    dt, T = 1e-3, 200
    xh, yh = mesh["x"].copy(), mesh["y"].copy()
    r = spring_adjoint(mesh, dt, T, every=20)
    assert r["loss"] > 0
    # every stiffness
    fd = np.zeros(mesh["S"])
    for s in range(mesh["S"]):
        h = 1e-6 * mesh["k"][s]
        mp, mm = dict(mesh), dict(mesh)
        mp["k"] = mesh["k"].copy()
        mm["k"] = mesh["k"].copy()
        mp["k"][s] += h
        mm["k"][s] -= h
        fd[s] = (_loss(mp, dt, T, xh, yh) - _loss(mm, dt, T, xh, yh)) / (2 * h)
    scale = np.max(np.abs(r["gk"]))
    assert np.all(np.abs(fd - r["gk"]) <= 1e-6 * np.abs(r["gk"]) + 1e-8 * scale)
    # every initial velocity component
    for comp in ("vx", "vy"):
        g = r["g" + comp]
        fdv = np.zeros(mesh["N"])
        for i in range(mesh["N"]):
            # step 1e-5 relative: the loss is O(1), so central differences carry
            # ~1e-16 / h of rounding noise; the floor below covers that
            h = 1e-5 * max(abs(mesh[comp][i]), 1e-2)
            mp, mm = dict(mesh), dict(mesh)
            mp[comp] = mesh[comp].copy()
            mm[comp] = mesh[comp].copy()
            mp[comp][i] += h
            mm[comp][i] -= h
            fdv[i] = (_loss(mp, dt, T, xh, yh) - _loss(mm, dt, T, xh, yh)) / (2 * h)
        sc = np.max(np.abs(g))
        assert np.all(np.abs(fdv - g) <= 1e-6 * np.abs(g) + 1e-7 * sc), comp


def test_directional_derivative_initial_positions():
    mesh = _as64(spring_mesh(6, 5, seed=4, v_sigma=0.8))
    dt, T = 2e-3, 100
    xh = mesh["x"] + 0.01
    yh = mesh["y"] - 0.02
    r = spring_adjoint(mesh, dt, T, every=7, xhat=xh, yhat=yh)
    rng = np.random.default_rng(0)
    dx, dy = rng.standard_normal(mesh["N"]), rng.standard_normal(mesh["N"])
    h = 1e-6
    mp, mm = dict(mesh), dict(mesh)
    mp["x"], mp["y"] = mesh["x"] + h * dx, mesh["y"] + h * dy
    mm["x"], mm["y"] = mesh["x"] - h * dx, mesh["y"] - h * dy
    fd = (_loss(mp, dt, T, xh, yh) - _loss(mm, dt, T, xh, yh)) / (2 * h)
    ad = np.dot(r["gx"], dx) + np.dot(r["gy"], dy)
    assert abs(fd - ad) <= 1e-7 * abs(ad)


@pytest.mark.parametrize("every", [1, 3, 7, 20, 60])
def test_checkpoint_interval_changes_no_bit(every):
    mesh = _as64(spring_mesh(7, 6, seed=9, v_sigma=0.5))
    ref = spring_adjoint(mesh, 1e-3, 60, every=60)
    r = spring_adjoint(mesh, 1e-3, 60, every=every)
    for key in ("gk", "gvx", "gvy", "gx", "gy", "xT", "yT"):
        assert np.array_equal(r[key], ref[key]), key
    assert r["loss"] == ref["loss"]


def test_forward_part_equals_plain_forward():
    mesh = _as64(spring_mesh(9, 4, seed=2, v_sigma=0.5))
    r = spring_adjoint(mesh, 1e-3, 40, every=20)
    f = spring_steps(mesh, 1e-3, 1e30, 40)
    assert np.array_equal(r["xT"], f["x"]) and np.array_equal(r["yT"], f["y"])


def test_single_step_function_composes_to_full_adjoint():
    # the full reverse sweep is the composition of single reverse steps
    from oracle import spring_adjoint_step

    mesh = _as64(spring_mesh(5, 4, seed=12, v_sigma=0.5))
    dt, T = 1e-3, 10
    full = spring_adjoint(mesh, dt, T, every=T)
    xs, ys = [], []
    st = mesh
    for n in range(T):
        xs.append(st["x"].copy())
        ys.append(st["y"].copy())
        st = spring_steps(st, dt, 1e30, 1)
    lx, ly = st["x"] - mesh["x"], st["y"] - mesh["y"]
    lvx, lvy = np.zeros(mesh["N"]), np.zeros(mesh["N"])
    gk = np.zeros(mesh["S"])
    for n in range(T - 1, -1, -1):
        r = spring_adjoint_step(mesh, xs[n], ys[n], dt, lx, ly, lvx, lvy)
        lx, ly, lvx, lvy = r["lx"], r["ly"], r["lvx"], r["lvy"]
        gk += r["gk"]
        # each scale bounds its quantity (triangle inequality over its terms)
        assert np.all(np.abs(r["lx"]) <= r["slx"] * (1 + 1e-12))
        assert np.all(np.abs(r["ly"]) <= r["sly"] * (1 + 1e-12))
        assert np.all(np.abs(r["lvx"]) <= r["slvx"] * (1 + 1e-12))
        assert np.all(np.abs(r["gk"]) <= r["sgk"] * (1 + 1e-12))
    assert np.allclose(gk, full["gk"], rtol=1e-12, atol=0)
    assert np.array_equal(lvx, full["gvx"]) and np.array_equal(lx, full["gx"])


def test_stretch_multiplier_by_hand_and_as_a_bound():
    # single spring, one step (as above): lambda_x1 = (1/4, -1/4), lambda_v1 = 0,
    # mu = dt lambda_x1 = (1/8, -1/8), g = w_a - w_b = 1/4 along u = (1, 0):
    # agk = dt |g| = 1/8, and gk = dt (l - L0) u . g = 1/2 * 1/2 * 1/4
    r = spring_adjoint(line2(), dt=0.5, steps=1, every=1)
    assert r["agk"][0] == 0.125 and r["gk"][0] == 0.0625
    # on a mesh: |dL/dk| <= max over the steps of |l - L0| times agk
    mesh = _as64(spring_mesh(7, 6, seed=9, v_sigma=0.5))
    dt, T = 1e-3, 60
    r = spring_adjoint(mesh, dt, T, every=20)
    st, stretch = mesh, np.zeros(mesh["S"])
    for _ in range(T):
        l = np.hypot(st["x"][mesh["b"]] - st["x"][mesh["a"]], st["y"][mesh["b"]] - st["y"][mesh["a"]])
        stretch = np.maximum(stretch, np.abs(l - mesh["L0"]))
        st = spring_steps(st, dt, 1e30, 1)
    assert np.all(np.abs(r["gk"]) <= stretch * r["agk"] * (1 + 1e-12))
    assert np.all(r["agk"] > 0)


@pytest.mark.slow
def test_directional_derivatives_at_the_100k_node_configuration():
    """The adjoint configuration itself (316 x 317 mesh, 100,172 nodes, dt
    1e-5, 200 steps, checkpoints every 20, L = 1/2 |x_T - x_0|^2): the
    directional derivatives of the oracle's gradients along random
    directions in v0 and in k equal central differences of the float64
    forward, to 1e-6.  The loss is smooth in both (breaking off).  Along v0 a
    relative step of 1e-4 is used.  L depends on k only weakly over 200 steps
    of 1e-5 (it changes by about 1e-9 of itself per unit relative change of
    k), so there a small step would leave the difference to the float64
    rounding of L (the cancellation in x_T - x_0); a relative step of 1e-2
    keeps that noise far below the tolerance, and the truncation error of a
    central difference, second order in the step, stays below it because L
    is close to quadratic in k over that range."""
    mesh = _as64(spring_mesh(316, 317))
    assert mesh["N"] == 100_172
    dt, T = 1e-5, 200
    xh, yh = mesh["x"].copy(), mesh["y"].copy()
    r = spring_adjoint(mesh, dt, T, every=20)
    rng = np.random.default_rng(316)
    # initial velocities: direction d (both components), step h |v0|
    dvx, dvy = rng.standard_normal(mesh["N"]), rng.standard_normal(mesh["N"])
    scale = np.sqrt(np.mean(mesh["vx"] ** 2 + mesh["vy"] ** 2))
    h = 1e-4 * scale
    mp, mm = dict(mesh), dict(mesh)
    mp["vx"], mp["vy"] = mesh["vx"] + h * dvx, mesh["vy"] + h * dvy
    mm["vx"], mm["vy"] = mesh["vx"] - h * dvx, mesh["vy"] - h * dvy
    fd = (_loss(mp, dt, T, xh, yh) - _loss(mm, dt, T, xh, yh)) / (2 * h)
    ad = np.dot(r["gvx"], dvx) + np.dot(r["gvy"], dvy)
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
    # stiffnesses: relative direction k * d
    dk = mesh["k"] * rng.standard_normal(mesh["S"])
    h = 1e-2
    mp, mm = dict(mesh), dict(mesh)
    mp["k"], mm["k"] = mesh["k"] + h * dk, mesh["k"] - h * dk
    fd = (_loss(mp, dt, T, xh, yh) - _loss(mm, dt, T, xh, yh)) / (2 * h)
    ad = np.dot(r["gk"], dk)
    assert abs(fd - ad) <= 1e-6 * abs(ad), (fd, ad)
