"""Pins of the "structure" oracle (thesis Ch.7 "structure": node subclasses,
tension-only springs that break above a force limit, removal of the nodes no
longer connected to an anchor node by a BFS).

Pinned by: BFS removal against a union-find connectivity computed here and
distances against scipy's unweighted shortest paths on random graphs of
degree <= 3; hand-computed force, slack and break steps (including the
deletion of nodes that lose their last spring); the discrete closed form of
symplectic Euler for a node on a stretched spring to an anchor, then exact
coasting once the spring is slack; a chain cut by a break and cleaned up by
the BFS; and invariants over pulled meshes with breaking.
"""

import math

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

from inputs import structure_mesh
from oracle import (STRUCTURE_MAXDIST, structure_bfs, structure_pull,
                    structure_step)


def build(types, pos, edges, k=None, L0=None, maxf=None, vel=None):
    """State from node types, positions and an edge list (p1, p2)."""
    N = len(types)
    S = len(edges)
    slot = -np.ones((N, 3), np.int32)
    isp2 = np.zeros((N, 3), np.uint8)
    s1 = np.zeros(S, np.int32)
    s2 = np.zeros(S, np.int32)
    fill = [0] * N
    for s, (a, b) in enumerate(edges):
        for node, is2, arr in ((a, 0, s1), (b, 1, s2)):
            q = fill[node]
            slot[node, q] = s
            isp2[node, q] = is2
            arr[s] = q
            fill[node] += 1
    pos = np.asarray(pos, float).reshape(N, 2)
    e = np.asarray(edges, np.int64).reshape(S, 2)
    if L0 is None:
        L0 = np.hypot(*(pos[e[:, 1]] - pos[e[:, 0]]).T) if S else np.zeros(0)
    vel = np.zeros((N, 2)) if vel is None else np.asarray(vel, float)
    return dict(ntype=np.asarray(types, np.int32), nalive=np.ones(N, np.uint8), x=pos[:, 0], y=pos[:, 1],
                vx=vel[:, 0], vy=vel[:, 1], m=np.ones(N), slot=slot.reshape(-1), isp2=isp2.reshape(-1),
                nspr=np.array(fill, np.int32), p1=e[:, 0].astype(np.int32), p2=e[:, 1].astype(np.int32),
                k=np.full(S, 1.0) if k is None else np.asarray(k, float), L0=np.asarray(L0, float),
                maxf=np.full(S, 1e30) if maxf is None else np.asarray(maxf, float), s1=s1, s2=s2,
                salive=np.ones(S, np.uint8))


def random_graph(rng, N, tries):
    deg = np.zeros(N, int)
    edges = set()
    for _ in range(tries):
        a, b = rng.integers(0, N, 2)
        if a == b or deg[a] == 3 or deg[b] == 3 or (min(a, b), max(a, b)) in edges:
            continue
        edges.add((int(min(a, b)), int(max(a, b))))
        deg[a] += 1
        deg[b] += 1
    return sorted(edges), deg


def components(N, edges):
    """Union-find labels (independent of the oracle's BFS)."""
    par = list(range(N))

    def find(v):
        while par[v] != v:
            par[v] = par[par[v]]
            v = par[v]
        return v
    for a, b in edges:
        ra, rb = find(a), find(b)
        if ra != rb:
            par[ra] = rb
    return np.array([find(v) for v in range(N)])


@pytest.mark.parametrize("seed", range(12))
def test_bfs_removal_matches_connectivity(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(1, 60))
    edges, deg = random_graph(rng, N, int(rng.integers(0, 2 * N)))
    types = rng.choice([0, 1, 2], size=N, p=[0.08, 0.12, 0.8])
    st = build(types, rng.random((N, 2)), edges)
    r = structure_bfs(st)
    lab = components(N, edges)
    anchored = set(lab[types == 0].tolist())
    reach = np.array([lab[v] in anchored for v in range(N)])
    want_node = reach | (deg == 0)
    assert np.array_equal(r["nalive"].astype(bool), want_node)
    want_spring = np.array([reach[a] for a, b in edges], bool)
    assert np.array_equal(r["salive"].astype(bool), want_spring)
    assert r["ndeleted"] == int((~want_spring).sum())
    # distances: unweighted shortest paths from the anchors
    if edges:
        e = np.array(edges)
        g = csr_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(N, N))
    else:
        g = csr_matrix((N, N))
    anchors = np.flatnonzero(types == 0)
    if anchors.size:
        d = shortest_path(g, directed=False, unweighted=True, indices=anchors).min(axis=0)
        fin = np.isfinite(d)
        assert np.array_equal(r["dist"][fin], d[fin].astype(int))
        assert np.all(r["dist"][~fin] == STRUCTURE_MAXDIST)
        assert r["levels"] == int(d[fin].max()) + 2
    else:
        assert r["levels"] == 1 and np.all(r["dist"] == STRUCTURE_MAXDIST)
    # slots of the survivors are consistent
    slot = r["slot"].reshape(N, 3)
    for v in np.flatnonzero(r["nalive"]):
        occ = slot[v][slot[v] >= 0]
        assert r["nspr"][v] == occ.size and all(r["salive"][s] for s in occ)


def test_hand_computed_force_slack_and_break():
    # anchor at 0, node at 1.5; k = 2, L0 = 1: pull 1 on the node towards the anchor
    st = build([0, 2], [[0, 0], [1.5, 0]], [(0, 1)], k=[2.0], L0=[1.0], maxf=[10.0])
    r = structure_step(st, 0.5)
    assert r["fx"].tolist() == [1.0] and r["fy"].tolist() == [0.0]
    assert r["vx"].tolist() == [0.0, -0.5] and r["x"].tolist() == [0.0, 1.25]
    # compressed: slack, nothing moves
    st = build([0, 2], [[0, 0], [0.5, 0]], [(0, 1)], k=[2.0], L0=[1.0], maxf=[10.0])
    r = structure_step(st, 0.5)
    assert r["fx"].tolist() == [0.0] and r["vx"].tolist() == [0.0, 0.0] and r["x"].tolist() == [0.0, 0.5]
    # limit 0.9 < 1: the spring breaks, and both endpoints lose their last spring
    st = build([0, 2], [[0, 0], [1.5, 0]], [(0, 1)], k=[2.0], L0=[1.0], maxf=[0.9])
    r = structure_step(st, 0.5)
    assert r["nbroken"] == 1 and r["salive"].tolist() == [0] and r["nalive"].tolist() == [0, 0]
    # exactly at the limit: no break (strictly greater)
    st = build([0, 2], [[0, 0], [1.5, 0]], [(0, 1)], k=[2.0], L0=[1.0], maxf=[1.0])
    assert structure_step(st, 0.5)["nbroken"] == 0


def test_pull_nodes_move_exactly():
    st = build([1, 2, 0], [[0.25, 0.5], [0, 0], [1, 1]], [], vel=[[2.0, -1.0], [3.0, 3.0], [5.0, 5.0]])
    r = structure_pull(st, 0.125)
    assert r["x"].tolist() == [0.5, 0.0, 1.0] and r["y"].tolist() == [0.375, 0.0, 1.0]


def test_anchored_oscillator_then_coasting():
    # a node on a spring to an anchor: w^2 = k / m while stretched; the
    # discrete map u' = u + dt v', v' = v - w^2 dt u has u_n = A cos(n th) +
    # B sin(n th), cos th = 1 - w^2 dt^2 / 2.  Once slack it coasts exactly.
    k, L0, u0, dt = 100.0, 1.0, 0.05, 1e-3
    st = build([0, 2], [[0, 0], [L0 + u0, 0]], [(0, 1)], k=[k], L0=[L0])
    th = math.acos(1 - k * dt * dt / 2)
    u1 = u0 - k * dt * dt * u0
    B = (u1 - u0 * math.cos(th)) / math.sin(th)
    for n in range(100):
        st = structure_step(st, dt)
    u_n = u0 * math.cos(100 * th) + B * math.sin(100 * th)
    assert u_n > 0.02 and abs((st["x"][1] - L0) - u_n) < 1e-12
    for n in range(100, 400):
        st = structure_step(st, dt)
    v400, x400 = st["vx"][1], st["x"][1]
    assert x400 < L0 and v400 < 0
    for n in range(400, 600):
        st = structure_step(st, dt)
    assert st["vx"][1] == v400
    assert abs(st["x"][1] - (x400 + 200 * dt * v400)) < 1e-12


def test_chain_cut_and_cleaned_up():
    # anchor 0 - 1 - 2 - 3 on a line, all stretched by 10 %; spring 1-2 has a
    # low limit and breaks; 2 and 3 keep their spring until the BFS
    pos = [[0, 0], [1.1, 0], [2.2, 0], [3.3, 0]]
    st = build([0, 2, 2, 2], pos, [(0, 1), (1, 2), (2, 3)], k=[1.0, 1.0, 1.0], L0=[1.0, 1.0, 1.0],
               maxf=[1.0, 0.05, 1.0])
    r = structure_step(st, 1e-3)
    assert r["nbroken"] == 1 and r["salive"].tolist() == [1, 0, 1] and r["nalive"].tolist() == [1, 1, 1, 1]
    assert r["nspr"].tolist() == [1, 1, 1, 1]
    b = structure_bfs(r)
    assert b["dist"][:2].tolist() == [0, 1] and b["levels"] == 3
    assert b["nalive"].tolist() == [1, 1, 0, 0] and b["salive"].tolist() == [1, 0, 0] and b["ndeleted"] == 1


@pytest.mark.parametrize("seed", [1, 2])
def test_pulled_mesh_invariants(seed):
    """Pull, 20 compute steps and the BFS removal, 12 times, on a 24 x 10
    mesh pulled fast enough to break: afterwards every live spring joins two
    live nodes that name it in the recorded slots, spring counts match the
    slots, and every live node with springs is connected to an anchor node
    (union-find over the live springs)."""
    st = structure_mesh(24, 10, seed=seed, pull_speed=2.0, break_strain=0.02)
    broken = removed = 0
    for it in range(12):
        st = structure_pull(st, 20 * 1e-4)
        for _ in range(20):
            st = structure_step(st, 1e-4)
            broken += st["nbroken"]
        st = structure_bfs(st)
        removed += st["ndeleted"]
        N, S = st["x"].size, st["p1"].size
        slot = st["slot"].reshape(N, 3)
        isp2 = st["isp2"].reshape(N, 3)
        for s in np.flatnonzero(st["salive"]):
            a, b = st["p1"][s], st["p2"][s]
            assert st["nalive"][a] and st["nalive"][b]
            assert slot[a, st["s1"][s]] == s and isp2[a, st["s1"][s]] == 0
            assert slot[b, st["s2"][s]] == s and isp2[b, st["s2"][s]] == 1
        live_edges = [(int(st["p1"][s]), int(st["p2"][s])) for s in np.flatnonzero(st["salive"])]
        lab = components(N, live_edges)
        anchored = set(lab[(st["ntype"] == 0) & (st["nalive"] == 1)].tolist())
        for v in np.flatnonzero(st["nalive"]):
            assert st["nspr"][v] == int((slot[v] >= 0).sum())
            if st["nspr"][v]:
                assert lab[v] in anchored
    assert broken > 0 and removed > 0, (broken, removed)
