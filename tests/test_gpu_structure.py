"""GPU parity of "structure" (thesis Ch.7: node subclasses under an abstract
NodeBase, tension-only springs that break above a force limit, BFS removal of
the nodes no longer connected to an anchor node) against the float64 oracle.

Every phase is checked from the GPU's own state: the oracle takes the state
read back before the phase and runs that phase once.  Integer results must
match exactly: which nodes and springs are alive, every spring slot of every
node, the spring counts, the BFS distances and the number of BFS levels.  The
oracle decides breaks in float64 and the kernel in float32: a spring decided
differently must be a tie (its float64 force within float32 rounding of the
limit; counted and reported), and the oracle's step is then rerun with the
GPU's decision for it.  Floats must match within 1e-5 of their conditioning scale
(spring force: k (l + L0); node velocity and position: |v| + dt S_F / m and
|x| + dt S_v).
"""

import numpy as np
import pytest

from inputs import structure_mesh
from oracle import STRUCTURE_MAXDIST, structure_bfs, structure_pull
from paper_1908_05845_amd import smmo
from paper_1908_05845_amd.sims import StructureSim
from spring_parity import structure_compute_step

pytestmark = pytest.mark.gpu

TOL = 1e-5
TOPO = ("p1", "p2", "k", "L0", "maxf", "s1", "s2", "m")


def state(mesh, st):
    d = {k: mesh[k] for k in TOPO}
    for k in ("ntype", "nalive", "x", "y", "vx", "vy", "slot", "isp2", "nspr", "dist", "salive", "fx", "fy",
              "sdel"):
        d[k] = st[k]
    return d


def check_topology(s1, ref):
    assert np.array_equal(s1["nalive"], ref["nalive"]), np.flatnonzero(s1["nalive"] != ref["nalive"])[:10]
    assert np.array_equal(s1["salive"], ref["salive"]), np.flatnonzero(s1["salive"] != ref["salive"])[:10]
    al = ref["nalive"].astype(bool)
    assert np.array_equal(s1["nspr"][al], ref["nspr"][al])
    sl = s1["slot"].reshape(-1, 3)[al]
    assert np.array_equal(sl, ref["slot"].reshape(-1, 3)[al])
    assert np.array_equal(s1["isp2"].reshape(-1, 3)[al][sl >= 0], ref["isp2"].reshape(-1, 3)[al][sl >= 0])


def check_step(sim, mesh):
    st = sim.read()
    assert (st["slot"] != -2).all(), "a slot names a dead spring"
    sim.compute_step()
    s1 = sim.read()
    ref, _, _ = structure_compute_step(state(mesh, st), sim.dt, s1["salive"])
    check_topology(s1, ref)
    sal = ref["salive"].astype(bool)
    for key in ("fx", "fy"):
        err = np.abs(s1[key][sal] - ref[key][sal])
        assert np.all(err <= TOL * ref["sf"][sal]), (key, float(np.max(err / np.maximum(ref["sf"][sal], 1e-30))))
    mov = ref["nalive"].astype(bool) & (ref["ntype"] == 2)
    for key, sc in (("vx", "svx"), ("vy", "svy"), ("x", "sx"), ("y", "sy")):
        err = np.abs(s1[key][mov] - ref[key][mov])
        assert np.all(err <= TOL * ref[sc][mov]), (key, float(np.max(err / ref[sc][mov])))
    fixed = ref["nalive"].astype(bool) & (ref["ntype"] != 2)
    assert np.array_equal(s1["x"][fixed], st["x"][fixed]) and np.array_equal(s1["y"][fixed], st["y"][fixed])
    return ref["nbroken"]


def check_pull(sim, mesh, dt):
    st = sim.read()
    ref = structure_pull(state(mesh, st), dt)
    sim.pull(dt)
    s1 = sim.read()
    al = ref["nalive"].astype(bool)
    for key, v in (("x", "vx"), ("y", "vy")):
        sc = np.abs(st[key][al]) + dt * np.abs(st[v][al])
        assert np.all(np.abs(s1[key][al] - ref[key][al]) <= TOL * np.maximum(sc, 1e-30))


def check_bfs(sim, mesh):
    st = sim.read()
    ref = structure_bfs(state(mesh, st))
    levels = sim.remove_disconnected()
    s1 = sim.read()
    check_topology(s1, ref)
    al = ref["nalive"].astype(bool)
    assert np.array_equal(s1["dist"][al], ref["dist"][al])
    assert levels == ref["levels"], (levels, ref["levels"])
    return ref["ndeleted"], int(np.sum(st["nalive"]) - np.sum(ref["nalive"]))


@pytest.mark.parametrize("W,H,seed,batch", [(24, 10, 1, 8), (17, 9, 2, 1), (40, 16, 3, 3)])
def test_iterations_phase_by_phase(dev, W, H, seed, batch):
    print("structure %dx%d seed %d bfs batch %d" % (W, H, seed, batch), flush=True)
    mesh = structure_mesh(W, H, seed=seed, pull_speed=2.0, break_strain=0.02, v_sigma=0.05)
    sim = StructureSim(mesh, 1e-4, bfs_batch=batch)
    broken = springs_removed = nodes_removed = 0
    for it in range(8):
        check_pull(sim, mesh, 10 * sim.dt)
        for _ in range(10):
            broken += check_step(sim, mesh)
        ds, dn = check_bfs(sim, mesh)
        springs_removed += ds
        nodes_removed += dn
    assert broken > 0 and nodes_removed > 0, (broken, springs_removed, nodes_removed)
    inv = sim.heap.invariants()
    assert inv.hierarchy_violations == 0 and inv.state_violations == 0 and inv.active_violations == 0
    assert inv.type_violations == 0 and inv.empty_allocated == 0
    st = sim.heap.stats()
    c = sim.heap.cls
    s = sim.read()
    assert st.live_objects[c["Spring"]] == int(s["salive"].sum())
    assert sum(st.live_objects[c[n]] for n in ("AnchorNode", "AnchorPullNode", "Node")) == int(s["nalive"].sum())


@pytest.mark.parametrize("W,H", [(1, 3), (2, 5), (3, 1), (5, 2)])
def test_small_meshes(dev, W, H):
    """Meshes without free nodes, without pull nodes or with one row."""
    print("structure %dx%d" % (W, H), flush=True)
    mesh = structure_mesh(W, H, seed=W * 10 + H, pull_speed=5.0, break_strain=0.01)
    sim = StructureSim(mesh, 1e-4)
    for it in range(3):
        check_pull(sim, mesh, 5 * sim.dt)
        for _ in range(5):
            check_step(sim, mesh)
        check_bfs(sim, mesh)


def test_no_anchor_removes_everything(dev):
    """Without anchor nodes the BFS visits nothing: every node with springs
    and every spring is deleted (a node loses its last spring and goes with
    it); the level count is 1."""
    mesh = structure_mesh(6, 4, seed=5)
    mesh["ntype"] = np.where(mesh["ntype"] == 0, 2, mesh["ntype"]).astype(np.int32)
    sim = StructureSim(mesh, 1e-4)
    ref = check_bfs(sim, mesh)
    s = sim.read()
    assert s["nalive"].sum() == 0 and s["salive"].sum() == 0 and sim.levels == 1, ref


def test_abstract_class_and_family_dispatch(dev):
    import torch

    mesh = structure_mesh(4, 3, seed=9)
    sim = StructureSim(mesh, 1e-4)
    with pytest.raises(smmo.SmmoError) as e:
        sim.heap.new("NodeBase", 1, x=torch.zeros(1, device=dev))
    assert e.value.status == smmo.SMMO_EINVAL
    # bfs_init on NodeBase reaches every node class; on AnchorNode only anchors
    sim.do("NodeBase", "bfs_init")
    d = sim.read()["dist"]
    assert np.array_equal(d == 0, mesh["ntype"] == 0) and np.all(d[mesh["ntype"] != 0] == STRUCTURE_MAXDIST)
    # a node method on the spring class is refused
    with pytest.raises(smmo.SmmoError):
        sim.do("Spring", "bfs_init")


@pytest.mark.parametrize("wg,waves", [(64, 1), (64, 3), (128, 2)])
def test_bfs_walks_with_small_grids(dev, wg, waves):
    """The family walk with fewer wavefronts than blocks: each wavefront steps
    through several blocks and across the three node classes' lists, and the
    distances, levels and deletions still equal the oracle's."""
    from paper_1908_05845_amd import smmo

    print("structure bfs grid wg %d waves %d" % (wg, waves), flush=True)
    mesh = structure_mesh(40, 16, seed=3, pull_speed=2.0, break_strain=0.02, v_sigma=0.05)
    sim = StructureSim(mesh, 1e-4, bfs_batch=4)
    nb = sim.heap.cls["NodeBase"]
    for name in ("structure.bfs_init", "structure.bfs_visit", "structure.bfs_mark"):
        smmo.smmo_set_launch(sim.heap.h, smmo.smmo_method_id(name), nb, wg, waves, 0)
    removed = 0
    for _ in range(8):
        sim.pull(10 * sim.dt)
        for _ in range(10):
            sim.compute_step()
        removed += check_bfs(sim, mesh)[1]
    assert removed > 0
    st = sim.heap.stats()
    assert st.device_error == 0
