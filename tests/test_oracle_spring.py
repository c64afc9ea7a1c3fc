"""Pins of the spring-mass oracle (thesis Ch.7 "structure", its compute steps:
Hooke's law F = k dx per spring, then the nbody-style node update; springs
break past a strain limit).

Pinned by: a hand-computed single step; the exact solution of symplectic
Euler on a harmonic oscillator (two nodes, one spring); the exactly
conserved modified energy of symplectic Euler on a linear (collinear) chain;
momentum conservation and bounded energy on a 2-D mesh; the break rule; and
batched runs equal to separate runs.
"""

import math

import numpy as np

from inputs import spring_mesh
from oracle import spring_breaks, spring_steps


def line_mesh(xs, ks, L0s, vs=None):
    """Nodes on the x axis joined in order by springs (node i -> spring i-1, i)."""
    n = len(xs)
    S = n - 1
    adj = -np.ones((n, 8), np.int32)
    adjb = np.zeros((n, 8), np.uint8)
    slot_a = np.zeros(S, np.int32)
    slot_b = np.zeros(S, np.int32)
    fill = [0] * n
    for s in range(S):
        for node, isb in ((s, 0), (s + 1, 1)):
            q = fill[node]
            adj[node, q] = s
            adjb[node, q] = isb
            (slot_b if isb else slot_a)[s] = q
            fill[node] += 1
    return dict(x=np.array(xs, float), y=np.zeros(n), vx=np.zeros(n) if vs is None else np.array(vs, float),
                vy=np.zeros(n), m=np.ones(n), adj=adj, adj_is_b=adjb,
                a=np.arange(S, dtype=np.int32), b=np.arange(1, n, dtype=np.int32),
                k=np.array(ks, float), L0=np.array(L0s, float), slot_a=slot_a, slot_b=slot_b)


def test_hand_computed_step():
    # nodes at 0 and 1.5, k = 2, L0 = 1: force on a = 2 * 0.5 = 1 towards b
    r = spring_steps(line_mesh([0.0, 1.5], [2.0], [1.0]), dt=0.5, thresh=1.0)
    assert r["fx"].tolist() == [1.0] and r["fy"].tolist() == [0.0]
    assert r["vx"].tolist() == [0.5, -0.5]
    assert r["x"].tolist() == [0.25, 1.25]


def test_two_node_oscillator_matches_discrete_closed_form():
    # separation s = L0 + 2u; each node: u'' = -(2k/m) u.  Symplectic Euler on
    # u'' = -w^2 u has the exact solution u_n = A cos(n th) + B sin(n th) with
    # cos th = 1 - w^2 dt^2 / 2.
    k, L0, u0, dt, n = 50.0, 1.0, 0.05, 1e-3, 3000
    w2 = 2 * k
    r = spring_steps(line_mesh([-(L0 / 2 + u0), L0 / 2 + u0], [k], [L0]), dt=dt, thresh=1.0, steps=n)
    # map: v' = v - w2 dt u, u' = u + dt v'.  With u_0 = u0, v_0 = 0:
    th = math.acos(1 - w2 * dt * dt / 2)
    u1 = u0 + dt * (0 - w2 * dt * u0)
    A = u0
    B = (u1 - A * math.cos(th)) / math.sin(th)
    u_n = A * math.cos(n * th) + B * math.sin(n * th)
    assert abs((r["x"][1] - L0 / 2) - u_n) < 1e-12
    assert abs((-r["x"][0] - L0 / 2) - u_n) < 1e-12


def test_linear_chain_conserves_modified_energy():
    # collinear chain, no breaking: forces are linear in the displacements, and
    # symplectic Euler conserves H = 1/2 v.v + 1/2 u.K u - dt/2 v.K u exactly.
    rng = np.random.default_rng(7)
    n = 12
    L0 = 1.0 + 0.2 * rng.random(n - 1)
    ks = 10 + 90 * rng.random(n - 1)
    rest = np.concatenate([[0.0], np.cumsum(L0)])
    u = 0.02 * rng.standard_normal(n)
    v = 0.1 * rng.standard_normal(n)
    K = np.zeros((n, n))
    for s in range(n - 1):
        K[s, s] += ks[s]; K[s + 1, s + 1] += ks[s]
        K[s, s + 1] -= ks[s]; K[s + 1, s] -= ks[s]
    dt = 2e-3

    def H(u, v):
        return 0.5 * v @ v + 0.5 * u @ K @ u - 0.5 * dt * v @ K @ u

    H0 = H(u, v)
    mesh = line_mesh(rest + u, ks, L0, v)
    r = spring_steps(mesh, dt=dt, thresh=1.0, steps=5000)
    H1 = H(r["x"] - rest, r["vx"])
    assert abs(H1 - H0) <= 1e-12 * abs(H0)
    assert r["nbroken"] == 0


def _energy(r):
    alive = r["alive"].astype(bool)
    a, b = r["a"][alive], r["b"][alive]
    l = np.hypot(r["x"][b] - r["x"][a], r["y"][b] - r["y"][a])
    pe = 0.5 * np.sum(r["k"][alive] * (l - r["L0"][alive]) ** 2)
    ke = 0.5 * np.sum(r["m"] * (r["vx"] ** 2 + r["vy"] ** 2))
    return ke + pe


def test_mesh_momentum_conserved_and_energy_bounded():
    mesh = spring_mesh(12, 10, seed=11)
    mesh = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) and v.dtype == np.float32 else v)
            for k, v in mesh.items()}
    p0 = np.array([mesh["vx"].sum(), mesh["vy"].sum()])
    E0 = _energy(dict(mesh, alive=np.ones(mesh["S"], np.uint8)))
    state = mesh
    es = []
    for _ in range(20):
        state = spring_steps(state, dt=1e-5, thresh=1e30, steps=500,
                             alive=state.get("alive"), fx=state.get("fx"), fy=state.get("fy"))
        es.append(_energy(state))
    p1 = np.array([state["vx"].sum(), state["vy"].sum()])
    assert np.all(np.abs(p1 - p0) <= 1e-12 * np.sum(np.abs(state["vx"]) + np.abs(state["vy"])))
    assert max(abs(e - E0) for e in es) <= 1e-3 * E0
    assert state["nbroken"] == 0


def test_initial_strain_is_zero():
    m = spring_mesh(30, 20, seed=5)
    l = np.hypot(m["x"][m["b"]].astype(float) - m["x"][m["a"]], m["y"][m["b"]].astype(float) - m["y"][m["a"]])
    assert np.max(np.abs(l - m["L0"]) / m["L0"]) < 1e-6
    r = spring_steps(m, dt=1e-5, steps=1)
    assert r["nbroken"] == 0


def test_break_rule():
    # strain 0.31 breaks (both slots emptied, no force), 0.29 does not
    m = line_mesh([0.0, 1.31, 2.60], [5.0, 5.0], [1.0, 1.0])
    r = spring_steps(m, dt=1e-3, thresh=0.3)
    assert r["alive"].tolist() == [0, 1]
    assert r["adj"][0].tolist() == [-1] * 8
    assert r["adj"][1].tolist() == [-1, 1] + [-1] * 6
    assert r["nbroken"] == 1
    # node 0 felt nothing; node 2 was pulled towards node 1 by 5 * 0.29
    assert r["vx"][0] == 0.0
    assert abs(r["vx"][2] - (-5 * 0.29 * 1e-3)) < 1e-12
    assert spring_breaks(0, 0, 1.31, 0, 1.0) and not spring_breaks(0, 0, 1.29, 0, 1.0)
    assert spring_breaks(0, 0, 0, 1.31, 1.0) and not spring_breaks(0, 0, 0, 0.5, 1.0)


def test_batched_equals_separate():
    m1 = spring_mesh(9, 7, seed=1)
    m2 = spring_mesh(6, 11, seed=2)
    cat = {}
    for key in ("x", "y", "vx", "vy", "m", "k", "L0", "slot_a", "slot_b", "adj_is_b"):
        cat[key] = np.concatenate([m1[key], m2[key]])
    cat["a"] = np.concatenate([m1["a"], m2["a"] + m1["N"]])
    cat["b"] = np.concatenate([m1["b"], m2["b"] + m1["N"]])
    adj2 = np.where(m2["adj"] >= 0, m2["adj"] + m1["S"], -1)
    cat["adj"] = np.concatenate([m1["adj"], adj2])
    r = spring_steps(cat, dt=1e-4, thresh=0.05, steps=300)
    r1 = spring_steps(m1, dt=1e-4, thresh=0.05, steps=300)
    r2 = spring_steps(m2, dt=1e-4, thresh=0.05, steps=300)
    for key in ("x", "y", "vx", "vy"):
        assert np.array_equal(r[key], np.concatenate([r1[key], r2[key]]))
    assert np.array_equal(r["alive"], np.concatenate([r1["alive"], r2["alive"]]))
    assert r["nbroken"] == r1["nbroken"] + r2["nbroken"]


def test_tension_only_hand_computed():
    # compressed: nodes at 0 and 0.5, k = 2, L0 = 1.  Two-sided: the force on
    # a is k (l - L0) d / l = 2 (-0.5) = -1 (pushed away from b); a
    # tension-only spring is slack and exerts nothing.
    m = line_mesh([0.0, 0.5], [2.0], [1.0])
    two = spring_steps(m, dt=0.5, thresh=1.0)
    assert two["fx"].tolist() == [-1.0] and two["vx"].tolist() == [-0.5, 0.5]
    slack = spring_steps(m, dt=0.5, thresh=1.0, tension_only=True)
    assert slack["fx"].tolist() == [0.0] and slack["vx"].tolist() == [0.0, 0.0]
    assert slack["x"].tolist() == [0.0, 0.5]
    # stretched: the same as the two-sided spring (the hand-computed step above)
    r = spring_steps(line_mesh([0.0, 1.5], [2.0], [1.0]), dt=0.5, thresh=1.0, tension_only=True)
    assert r["fx"].tolist() == [1.0] and r["vx"].tolist() == [0.5, -0.5] and r["x"].tolist() == [0.25, 1.25]


def test_tension_only_oscillator_goes_slack():
    # Two nodes released from a stretch u0 (separation L0 + 2 u0): while the
    # spring is stretched the motion is the harmonic one (the discrete closed
    # form of the two-sided test); after the separation drops below L0 there
    # is no force, so the velocities stay exactly constant and the nodes move
    # in a straight line until they would meet, about 1/(2 u0 w dt) steps on.
    k, L0, u0, dt = 50.0, 1.0, 0.05, 1e-3
    w2 = 2 * k
    mesh = line_mesh([-(L0 / 2 + u0), L0 / 2 + u0], [k], [L0])
    th = math.acos(1 - w2 * dt * dt / 2)
    u1 = u0 + dt * (0 - w2 * dt * u0)
    B = (u1 - u0 * math.cos(th)) / math.sin(th)
    n = 100                                       # u_n > 0: still stretched
    r = spring_steps(mesh, dt=dt, thresh=1.0, steps=n, tension_only=True)
    u_n = u0 * math.cos(n * th) + B * math.sin(n * th)
    assert u_n > 0.02
    assert abs((r["x"][1] - L0 / 2) - u_n) < 1e-12
    # first slack step: u turns negative near n* = pi / (2 th) ~ 157
    r1 = spring_steps(mesh, dt=dt, thresh=1.0, steps=200, tension_only=True)
    r2 = spring_steps(mesh, dt=dt, thresh=1.0, steps=600, tension_only=True)
    assert r1["x"][1] - r1["x"][0] < L0 and r2["x"][1] - r2["x"][0] > 0
    assert r1["vx"].tolist() == r2["vx"].tolist()                  # no force at all
    assert r1["vx"][1] < 0 and r1["vx"][0] == -r1["vx"][1]
    assert abs(r2["x"][1] - (r1["x"][1] + 400 * dt * r1["vx"][1])) < 1e-12
    # the slack speed is the harmonic phase's speed when the spring reached L0
    # (|u'| = u0 w up to O(dt) for the discrete map)
    assert abs(-r1["vx"][1] - u0 * math.sqrt(w2)) < 2e-2 * u0 * math.sqrt(w2)
    # the two-sided spring instead pushes back: at step 600 it is compressed
    # and decelerating, not coasting
    t = spring_steps(mesh, dt=dt, thresh=1.0, steps=600)
    assert t["vx"][1] != r2["vx"][1]


def test_any_degree_oracle_equals_eight_slot_oracle():
    """The variable-degree routine is the 8-slot one on meshes that fit 8
    slots: bit-identical states, forces, topology and scales, with breaking."""
    from oracle import spring_steps_deg
    mesh = spring_mesh(30, 20, seed=4, v_sigma=1.0)
    for steps in (3, 7):
        r8 = spring_steps(mesh, 1e-4, 0.001, steps)
        rd = spring_steps_deg(mesh, 1e-4, 0.001, steps)
        assert r8["nbroken"] == rd["nbroken"] and r8["nbroken"] > 0
        for key in ("x", "y", "vx", "vy", "fx", "fy", "alive", "adj", "sf", "svx", "svy", "sx", "sy"):
            assert np.array_equal(np.asarray(r8[key]).reshape(-1), np.asarray(rd[key]).reshape(-1)), key


def test_hub_mesh_momentum_and_star():
    from inputs import hub_mesh
    from oracle import spring_steps_deg
    mesh = hub_mesh(24, 16, hubs=4, hub_springs=30, v_sigma=0.5)
    assert np.asarray(mesh["adj"]).shape[1] > 8
    p0 = np.array([np.sum(np.asarray(mesh["vx"], float)), np.sum(np.asarray(mesh["vy"], float))])
    r = spring_steps_deg(mesh, 1e-4, 1e9, 50)
    p1 = np.array([np.sum(r["vx"]), np.sum(r["vy"])])
    scale = np.sum(np.abs(r["vx"])) + np.sum(np.abs(r["vy"]))
    assert np.all(np.abs(p1 - p0) <= 1e-12 * scale)
    # a star: a hub with 12 springs (k = 2, L0 = 1) to leaves at distance 1.5
    n = 12
    th = 2 * np.pi * np.arange(n) / n
    x = np.concatenate([[0.0], 1.5 * np.cos(th)])
    y = np.concatenate([[0.0], 1.5 * np.sin(th)])
    adj = -np.ones((n + 1, n), np.int32)
    adjb = np.zeros((n + 1, n), np.uint8)
    adj[0, :] = np.arange(n)
    adj[1:, 0] = np.arange(n)
    adjb[1:, 0] = 1
    star = dict(x=x, y=y, vx=np.zeros(n + 1), vy=np.zeros(n + 1), m=np.ones(n + 1), adj=adj, adj_is_b=adjb,
                a=np.zeros(n, np.int32), b=np.arange(1, n + 1, dtype=np.int32), k=np.full(n, 2.0),
                L0=np.ones(n), slot_a=np.arange(n, dtype=np.int32), slot_b=np.zeros(n, np.int32))
    r = spring_steps_deg(star, 0.5, 1.0, 1)
    # every leaf is pulled 1 towards the hub; the hub's forces cancel
    assert np.allclose(r["vx"][1:], -0.5 * np.cos(th), atol=1e-12)
    assert np.allclose(r["vy"][1:], -0.5 * np.sin(th), atol=1e-12)
    assert abs(r["vx"][0]) < 1e-12 and abs(r["vy"][0]) < 1e-12
