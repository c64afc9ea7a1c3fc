"""Pins of the oracle's integer decisions and of the conditioning scales that
set every GPU tolerance (thesis Ch.7 "structure": a spring breaks when it is
stretched past its limit; the force, velocity and position updates of the
compute steps; and the reverse of one step for the differentiable mesh).

Decisions.  The oracle decides in float64 from the state as given: strain
(l - L0)/L0 > threshold for the mesh springs, k (l - L0) > limit for the
"structure" springs.  The pins put springs a few float64 ulps on either side
of the limit, at values where every float32 evaluation of the same state
rounds to the limit itself, so an oracle that copied a float32 order would
fail them.  A float32 implementation can disagree only within its rounding
of the limit (the tie band); the band is pinned against the rounding error
of float32 re-evaluations of the strain.

Scales.  Each scale is the triangle-inequality bound of its quantity: the
sum of the magnitudes of the terms it is computed from.  They are pinned to
hand-computed values on small meshes, checked to bound their quantities,
and checked against float32 re-evaluations of the same step written here
with numpy: the float32 error must stay below 1e-5 of the scale (the scale
covers the rounding) and must reach at least 1e-9 of it somewhere (a scale
inflated by a large factor would widen every tolerance and fails here).
"""

import math

import numpy as np
import pytest

from inputs import spring_mesh
from oracle import (spring_adjoint_step, spring_breaks, spring_steps, spring_tie_band,
                    structure_step, STRUCTURE_TIE_REL)
from test_oracle_spring import line_mesh
from test_oracle_structure import build

E30 = 2.0 ** -30
E40 = 2.0 ** -40
U32 = 2.0 ** -24


# ------------------------------------------------------------ break rule --
def test_break_decided_in_float64_at_exact_strains():
    # 3-4-5 triangle with L0 = 4: strain exactly 0.25
    brk, e = spring_breaks(0, 0, 3, 4, 4.0, 0.25, with_strain=True)
    assert e == 0.25 and not brk                       # strictly greater
    assert spring_breaks(0, 0, 3, 4, 4.0, 0.25 - E40)
    # 3 + 2^-33 rounds to 3 in float32, where the strain is exactly 0.25 and
    # no float32 evaluation breaks; in float64 the spring is longer than 5
    assert np.float32(3 + 2.0 ** -33) == np.float32(3)
    brk, e = spring_breaks(0, 0, 3 + 2.0 ** -33, 4, 4.0, 0.25, with_strain=True)
    assert brk and 0 < e - 0.25 < 1e-9
    brk, e = spring_breaks(0, 0, 3 - 2.0 ** -33, 4, 4.0, 0.25, with_strain=True)
    assert not brk and -1e-9 < e - 0.25 < 0


def test_break_rule_just_inside_and_outside_the_limit():
    # spring 0 at strain 0.25 + 2^-30 breaks, spring 1 at 0.25 - 2^-30 holds
    x1 = 1.25 + E30
    m = line_mesh([0.0, x1, 2.5], [5.0, 5.0], [1.0, 1.0])
    assert m["x"][2] - m["x"][1] == 1.25 - E30
    r = spring_steps(m, dt=1e-3, thresh=0.25)
    assert r["alive"].tolist() == [0, 1] and r["nbroken"] == 1
    assert r["strain"][0] == 0.25 + E30 and r["strain"][1] == 0.25 - E30
    assert r["adj"][0].tolist() == [-1] * 8 and r["adj"][1].tolist() == [-1, 1] + [-1] * 6
    # both decisions flip with the threshold moved across them
    assert spring_steps(m, dt=1e-3, thresh=0.25 + 2 * E30)["alive"].tolist() == [1, 1]
    assert spring_steps(m, dt=1e-3, thresh=0.25 - 2 * E30)["alive"].tolist() == [0, 0]


def test_fixed_tie_decisions_inside_the_band_only():
    x1 = 1.25 + E30
    m = line_mesh([0.0, x1, 2.5], [5.0, 5.0], [1.0, 1.0])
    # both springs are within the band: the other decision is accepted
    r = spring_steps(m, dt=1e-3, thresh=0.25, tie=[0, 1])
    assert r["alive"].tolist() == [1, 0] and r["nbroken"] == 1
    # the kept spring pulls with k (l - L0) = 5 (0.25 + 2^-30)
    assert r["fx"][0] == 5.0 * (0.25 + E30)
    # -1 = decide by the rule
    assert spring_steps(m, dt=1e-3, thresh=0.25, tie=[-1, -1])["alive"].tolist() == [0, 1]
    # a spring far from the limit cannot be fixed
    far = line_mesh([0.0, 1.31, 2.60], [5.0, 5.0], [1.0, 1.0])
    with pytest.raises(RuntimeError):
        spring_steps(far, dt=1e-3, thresh=0.3, tie=[0, -1])
    with pytest.raises(RuntimeError):
        spring_steps(far, dt=1e-3, thresh=0.3, tie=[-1, 1])
    # a fixed decision applies to the first step of a call only
    r2 = spring_steps(m, dt=1e-9, thresh=0.25, steps=2, tie=[0, -1])
    assert r2["alive"].tolist() == [0, 1] and r2["nbroken"] == 2 - 1


def _strain32(xa, ya, xb, yb, L0, order):
    f = np.float32
    dx = f(xb) - f(xa)
    dy = f(yb) - f(ya)
    if order == 0:
        l2 = dx * dx + dy * dy
    else:
        l2 = dy * dy + dx * dx
    l = np.sqrt(l2, dtype=np.float32)
    return (l - f(L0)) / f(L0)


def test_tie_band_covers_float32_rounding_of_the_strain():
    """Springs of the 1000 x 1000 mesh's geometry (unit square, spacing 1e-3)
    stretched to strains near 0.3: every float32 evaluation of the strain from
    the float32 state is within a quarter of the band of the float64 strain
    (the error analysis gives about 4.2 * 2^-24)."""
    band = spring_tie_band()
    assert band == 1e-6
    rng = np.random.default_rng(3)
    n = 200_000
    xa = rng.uniform(-0.5, 0.5, n).astype(np.float32)
    ya = rng.uniform(-0.5, 0.5, n).astype(np.float32)
    th = rng.uniform(0, 2 * np.pi, n)
    L0 = rng.uniform(0.7e-3, 1.7e-3, n).astype(np.float32)
    l = L0.astype(np.float64) * rng.uniform(1.29, 1.31, n)
    xb = (xa + l * np.cos(th)).astype(np.float32)
    yb = (ya + l * np.sin(th)).astype(np.float32)
    dx = xb.astype(np.float64) - xa
    dy = yb.astype(np.float64) - ya
    e64 = (np.sqrt(dx * dx + dy * dy) - L0) / L0
    worst = max(float(np.max(np.abs(_strain32(xa, ya, xb, yb, L0, o) - e64))) for o in (0, 1))
    assert worst <= band / 4, worst
    assert worst >= 2 * U32          # the rounding is real, not zero


def test_structure_break_decided_in_float64_with_ties():
    # k = 2, L0 = 1, l = 1.5: F = 1 exactly; limit 1 holds (strictly greater)
    st = build([0, 2], [[0, 0], [1.5, 0]], [(0, 1)], k=[2.0], L0=[1.0], maxf=[1.0])
    r = structure_step(st, 0.5)
    assert r["nbroken"] == 0 and r["F"][0] == 1.0
    # l = 1.5 + 2^-40: F = 1 + 2^-39 > 1 in float64; every float32 evaluation
    # gives l = 1.5 and F = 1
    assert np.float32(1.5 + E40) == np.float32(1.5)
    st2 = build([0, 2], [[0, 0], [1.5 + E40, 0]], [(0, 1)], k=[2.0], L0=[1.0], maxf=[1.0])
    r2 = structure_step(st2, 0.5)
    assert r2["nbroken"] == 1 and r2["F"][0] == 1.0 + 2 * E40
    # both are ties (|F - limit| <= 1e-6 k (l + L0)): fixed decisions accepted
    assert structure_step(st, 0.5, tie=[1])["nbroken"] == 1
    assert structure_step(st2, 0.5, tie=[0])["nbroken"] == 0
    # far from the limit: refused
    st3 = build([0, 2], [[0, 0], [1.5, 0]], [(0, 1)], k=[2.0], L0=[1.0], maxf=[0.9])
    with pytest.raises(RuntimeError):
        structure_step(st3, 0.5, tie=[0])
    assert STRUCTURE_TIE_REL == 1e-6


def test_structure_tie_band_covers_float32_rounding_of_the_force():
    rng = np.random.default_rng(5)
    n = 100_000
    f = np.float32
    xa = rng.uniform(-0.5, 0.5, n).astype(f)
    ya = rng.uniform(-0.5, 0.5, n).astype(f)
    th = rng.uniform(0, 2 * np.pi, n)
    L0 = rng.uniform(0.7e-3, 1.3e-3, n).astype(f)
    k = (10.0 ** rng.uniform(2, 4, n)).astype(f)
    l = L0.astype(np.float64) * rng.uniform(1.0, 1.1, n)
    xb = (xa + l * np.cos(th)).astype(f)
    yb = (ya + l * np.sin(th)).astype(f)
    dx = xb.astype(np.float64) - xa
    dy = yb.astype(np.float64) - ya
    l64 = np.sqrt(dx * dx + dy * dy)
    F64 = k * (l64 - L0)
    l32 = np.sqrt((xb - xa) * (xb - xa) + (yb - ya) * (yb - ya), dtype=f)
    F32 = k * (l32 - L0)
    rel = np.abs(F32 - F64) / (k.astype(np.float64) * (l64 + L0))
    assert float(np.max(rel)) <= STRUCTURE_TIE_REL / 3, float(np.max(rel))


# --------------------------------------------------------------- scales --
def test_spring_scales_hand_computed():
    # 3-4-5 spring, k = 2, L0 = 4: f = k (l - L0) d / l = (1.2, 1.6); the
    # terms of k (l - L0) are k l = 10 and k L0 = 8, so sf = 18
    m = dict(line_mesh([0.0, 3.0], [2.0], [4.0]))
    m["y"] = np.array([0.0, 4.0])
    r = spring_steps(m, dt=0.5, thresh=1.0)
    assert r["sf"].tolist() == [18.0]
    assert abs(r["fx"][0] - 1.2) < 1e-15 and abs(r["fy"][0] - 1.6) < 1e-15
    # a chain: springs (k 2, L0 1, l 1.5) and (k 3, L0 1.5, l 2); dt 0.5, m 1
    c = line_mesh([0.0, 1.5, 3.5], [2.0, 3.0], [1.0, 1.5], vs=[0.1, -0.2, 0.3])
    r = spring_steps(c, dt=0.5, thresh=1.0)
    assert r["sf"].tolist() == [5.0, 10.5]
    # |v| + dt * sum of the attached sf / m, then |x| + dt * that
    want_svx = [0.1 + 0.5 * 5.0, 0.2 + 0.5 * 15.5, 0.3 + 0.5 * 10.5]
    want_svy = [0.5 * 5.0, 0.5 * 15.5, 0.5 * 10.5]
    want_sx = [0.0 + 0.5 * want_svx[0], 1.5 + 0.5 * want_svx[1], 3.5 + 0.5 * want_svx[2]]
    want_sy = [0.5 * v for v in want_svy]
    for key, want in (("svx", want_svx), ("svy", want_svy), ("sx", want_sx), ("sy", want_sy)):
        assert np.allclose(r[key], want, rtol=1e-15, atol=0), key
    # a slack tension-only spring keeps its scale (k (l + L0) = 2 * 1.5); a
    # broken spring has none
    assert spring_steps(line_mesh([0.0, 0.5], [2.0], [1.0]), dt=0.5, thresh=1.0,
                        tension_only=True)["sf"].tolist() == [3.0]
    assert spring_steps(line_mesh([0.0, 2.5], [2.0], [1.0]), dt=0.5, thresh=1.0)["sf"].tolist() == [0.0]


def _as64(mesh):
    return {k: (v.astype(np.float64) if isinstance(v, np.ndarray) and v.dtype == np.float32 else v)
            for k, v in mesh.items()}


def _spring_step32(m, dt):
    """One step in float32 (numpy), in slot order: the quantities whose
    rounding the scales bound."""
    f = np.float32
    x, y, vx, vy = (np.asarray(m[k], f).copy() for k in ("x", "y", "vx", "vy"))
    a, b = m["a"], m["b"]
    k, L0 = np.asarray(m["k"], f), np.asarray(m["L0"], f)
    dx, dy = x[b] - x[a], y[b] - y[a]
    l = np.sqrt(dx * dx + dy * dy, dtype=f)
    c = k * (l - L0) / l
    fx, fy = c * dx, c * dy
    adj = np.asarray(m["adj"]).reshape(-1, 8)
    sg = np.where(np.asarray(m["adj_is_b"]).reshape(-1, 8) == 1, f(-1), f(1))
    Fx = np.zeros(x.size, f)
    Fy = np.zeros(x.size, f)
    for q in range(8):
        has = adj[:, q] >= 0
        s = np.where(has, adj[:, q], 0)
        Fx = Fx + np.where(has, sg[:, q] * fx[s], f(0))
        Fy = Fy + np.where(has, sg[:, q] * fy[s], f(0))
    mm = np.asarray(m["m"], f)
    vx = vx + Fx / mm * f(dt)
    vy = vy + Fy / mm * f(dt)
    return dict(fx=fx, fy=fy, vx=vx, vy=vy, x=x + vx * f(dt), y=y + vy * f(dt))


@pytest.mark.parametrize("seed,v_sigma,dt", [(1, 0.01, 1e-5), (2, 1.0, 1e-4), (3, 5.0, 1e-3)])
def test_spring_scales_bound_and_are_tight(seed, v_sigma, dt):
    mesh = spring_mesh(40, 30, seed=seed, v_sigma=v_sigma)
    # move the state off rest length so forces are not near zero
    rng = np.random.default_rng(seed)
    mesh["x"] = (mesh["x"] + rng.normal(0, 0.05 * mesh["h"], mesh["N"])).astype(np.float32)
    mesh["y"] = (mesh["y"] + rng.normal(0, 0.05 * mesh["h"], mesh["N"])).astype(np.float32)
    r = spring_steps(mesh, dt, thresh=1e30)
    g = _spring_step32(mesh, dt)
    # triangle bounds hold for the float64 quantities themselves
    assert np.all(np.abs(r["fx"]) <= r["sf"]) and np.all(np.abs(r["fy"]) <= r["sf"])
    v0x = np.asarray(mesh["vx"], float)
    assert np.all(np.abs(r["vx"]) <= r["svx"] * (1 + 1e-12))
    assert np.all(np.abs(r["x"]) <= r["sx"] * (1 + 1e-12))
    assert np.all(r["svx"] >= np.abs(v0x))
    for key, sc in (("fx", "sf"), ("fy", "sf"), ("vx", "svx"), ("vy", "svy"), ("x", "sx"), ("y", "sy")):
        ratio = np.abs(g[key] - r[key]) / r[sc]
        assert float(np.max(ratio)) <= 1e-5, (key, float(np.max(ratio)))
        assert float(np.max(ratio)) >= 1e-9, (key, float(np.max(ratio)))


def test_adjoint_scales_hand_computed():
    """One spring (0,0)-(3,4), k 2, L0 4 (l 5, u (0.6, 0.8)), m 1, dt 0.5,
    incoming adjoints lx = (1, 0), ly = (0, 2), lvx = (0.5, 0), lvy = 0.
    mu = lv + dt lx: a (1, 0), b (0, 1); g = w_a - w_b = (1, -1), u.g = -0.2.
    gk = dt (l - L0) u.g = -0.1; its terms bound it by dt (l + L0) |g|.
    K g = k ((1 - L0/l) g + (L0/l) u (u.g)) = (0.208, -0.656), bounded by
    k (1 + 2 L0/l) |g|; lx_a -= dt K g, lx_b += dt K g."""
    mesh = line_mesh([0.0, 3.0], [2.0], [4.0])
    r = spring_adjoint_step(mesh, [0.0, 3.0], [0.0, 4.0], 0.5, [1.0, 0.0], [0.0, 2.0], [0.5, 0.0], [0.0, 0.0])
    s2 = math.sqrt(2.0)
    assert abs(r["gk"][0] - (-0.1)) < 1e-15
    assert abs(r["sgk"][0] - 0.5 * 9 * s2) < 1e-14
    assert np.allclose([r["lx"][0], r["ly"][0], r["lx"][1], r["ly"][1]], [0.896, 0.328, 0.104, 1.672],
                       rtol=0, atol=1e-15)
    assert np.allclose([r["lvx"][0], r["lvy"][0], r["lvx"][1], r["lvy"][1]], [1, 0, 0, 1], rtol=0, atol=0)
    c = 0.5 * 2 * (1 + 2 * 4 / 5) * s2
    assert np.allclose([r["slx"][0], r["sly"][0], r["slx"][1], r["sly"][1]], [1 + c, c, c, 2 + c],
                       rtol=1e-15, atol=0)
    assert [r["slvx"][0], r["slvy"][0], r["slvx"][1], r["slvy"][1]] == [1.0, 0.0, 0.0, 1.0]


def _adjoint_step32(mesh, px, py, dt, lx, ly, lvx, lvy):
    f = np.float32
    px, py, lx, ly, lvx, lvy = (np.asarray(v, f) for v in (px, py, lx, ly, lvx, lvy))
    m = np.asarray(mesh["m"], f)
    mux, muy = lvx + f(dt) * lx, lvy + f(dt) * ly
    wx, wy = mux / m, muy / m
    a, b = mesh["a"], mesh["b"]
    k, L0 = np.asarray(mesh["k"], f), np.asarray(mesh["L0"], f)
    dx, dy = px[b] - px[a], py[b] - py[a]
    l = np.sqrt(dx * dx + dy * dy, dtype=f)
    ux, uy = dx / l, dy / l
    gx, gy = wx[a] - wx[b], wy[a] - wy[b]
    ug = ux * gx + uy * gy
    r = L0 / l
    kgx = k * ((f(1) - r) * gx + r * ux * ug)
    kgy = k * ((f(1) - r) * gy + r * uy * ug)
    cx, cy = f(dt) * kgx, f(dt) * kgy
    gk = f(dt) * (l - L0) * ug
    adj = np.asarray(mesh["adj"]).reshape(-1, 8)
    isb = np.asarray(mesh["adj_is_b"]).reshape(-1, 8) == 1
    nx, ny = lx.copy(), ly.copy()
    for q in range(8):
        has = adj[:, q] >= 0
        s = np.where(has, adj[:, q], 0)
        sg = np.where(isb[:, q], f(1), f(-1))
        nx = nx + np.where(has, sg * cx[s], f(0))
        ny = ny + np.where(has, sg * cy[s], f(0))
    return dict(lx=nx, ly=ny, lvx=mux, lvy=muy, gk=gk)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_adjoint_scales_bound_and_are_tight(seed):
    mesh = _as64(spring_mesh(30, 20, seed=seed, v_sigma=0.5))
    rng = np.random.default_rng(seed)
    px = (mesh["x"] + rng.normal(0, 0.05 * mesh["h"], mesh["N"])).astype(np.float32).astype(float)
    py = (mesh["y"] + rng.normal(0, 0.05 * mesh["h"], mesh["N"])).astype(np.float32).astype(float)
    seeds = [rng.standard_normal(mesh["N"]).astype(np.float32).astype(float) for _ in range(4)]
    dt = 1e-3
    r = spring_adjoint_step(mesh, px, py, dt, *[s.copy() for s in seeds])
    g = _adjoint_step32(mesh, px, py, dt, *seeds)
    # the scales bound the float64 quantities they belong to
    assert np.all(np.abs(r["gk"]) <= r["sgk"] * (1 + 1e-12))
    assert np.all(np.abs(r["lx"]) <= r["slx"] * (1 + 1e-12)) and np.all(np.abs(r["ly"]) <= r["sly"] * (1 + 1e-12))
    assert np.all(np.abs(r["lvx"]) <= r["slvx"] * (1 + 1e-12))
    for key, sc in (("lx", "slx"), ("ly", "sly"), ("lvx", "slvx"), ("lvy", "slvy"), ("gk", "sgk")):
        ratio = np.abs(g[key] - r[key]) / r[sc]
        assert float(np.max(ratio)) <= 1e-5, (key, float(np.max(ratio)))
        assert float(np.max(ratio)) >= 1e-9, (key, float(np.max(ratio)))
