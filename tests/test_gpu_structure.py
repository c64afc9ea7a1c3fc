"""GPU parity of "structure" (thesis Ch.7: node subclasses under an abstract
NodeBase, tension-only springs that break above a force limit, BFS removal of
the nodes no longer connected to an anchor node) against the float64 oracle,
with no GPU value given to the oracle.

The oracle runs its own trajectory (pull, compute steps, BFS removal) from
the mesh.  Every phase is checked by a restart: the oracle's state before
the phase, rounded to float32, is loaded into a fresh heap, the GPU runs the
phase, and the result is compared with the oracle's phase from the same
rounded state.  Beside it the GPU runs the whole trajectory on one heap, and
every phase of that run must give bit for bit what a fresh heap loaded with
its state gives (same-heap check).  Integer results must match exactly:
which nodes and springs are alive, every spring slot of every node, the
spring counts, the BFS distances and the number of BFS levels.  The oracle
decides breaks in float64 and the kernel in float32: a spring decided
otherwise must be a tie (its float64 force within float32 rounding of the
limit; counted and reported), and it and its two end nodes are then left
out of the comparison.  Floats must match within 1e-5 of their conditioning
scale (spring force: k (l + L0); node velocity and position: |v| + dt S_F / m
and |x| + dt S_v).
"""

import numpy as np
import pytest

from inputs import structure_mesh
from oracle import STRUCTURE_MAXDIST, structure_bfs, structure_pull, structure_step
from paper_1908_05845_amd import smmo
from paper_1908_05845_amd.sims import StructureSim
from spring_parity import round32, structure_compare

pytestmark = pytest.mark.gpu

TOL = 1e-5
TOPO = ("p1", "p2", "k", "L0", "maxf", "s1", "s2", "m")
STATE = ("ntype", "nalive", "x", "y", "vx", "vy", "slot", "isp2", "nspr", "dist", "salive", "fx", "fy", "sdel")
DT = 1e-4


def state(mesh, st):
    """A GPU read-back as a structure state (constants from the mesh)."""
    d = {k: mesh[k] for k in TOPO}
    for k in STATE:
        d[k] = st[k]
    return d


def check_topology(s1, ref, node_ok=None, sdiff=None):
    N = ref["nalive"].size
    node_ok = np.ones(N, bool) if node_ok is None else node_ok
    sok = np.ones(ref["salive"].size, bool) if sdiff is None else ~sdiff
    assert np.array_equal(s1["nalive"][node_ok], ref["nalive"][node_ok]), \
        np.flatnonzero((s1["nalive"] != ref["nalive"]) & node_ok)[:10]
    assert np.array_equal(s1["salive"][sok], ref["salive"][sok]), \
        np.flatnonzero((s1["salive"] != ref["salive"]) & sok)[:10]
    al = ref["nalive"].astype(bool) & node_ok
    assert np.array_equal(s1["nspr"][al], ref["nspr"][al])
    sl = s1["slot"].reshape(-1, 3)[al]
    assert (s1["slot"] != -2).all(), "a slot names a dead spring"
    assert np.array_equal(sl, ref["slot"].reshape(-1, 3)[al])
    assert np.array_equal(s1["isp2"].reshape(-1, 3)[al][sl >= 0], ref["isp2"].reshape(-1, 3)[al][sl >= 0])


# the BFS forms: the one-call queue BFS with its visited set in LDS, in device
# memory, with a 64-node LDS frontier (the rest queued in device memory), both
# of the latter; and the thesis's level passes
BFS_FORMS = {"queue": ("queue", 0),
             "queue-device-visited": ("queue", smmo.SMMO_BFS_DEVICE_VISITED),
             "queue-small-frontier": ("queue", smmo.SMMO_BFS_SMALL_FRONTIER),
             "queue-device-both": ("queue", smmo.SMMO_BFS_DEVICE_VISITED | smmo.SMMO_BFS_SMALL_FRONTIER),
             "levels": ("levels", 0)}


def make_sim(batch=8, shapes=None, bfs="queue", class_shapes=None):
    """A maker of fresh simulations: `shapes` are launch shapes of methods on
    NodeBase (the BFS family walks), `class_shapes` of (method, class)
    pairs."""
    mode, options = BFS_FORMS[bfs]

    def make(st):
        sim = StructureSim(st, DT, bfs_batch=batch, bfs=mode, bfs_options=options)
        for name, shape in (shapes or {}).items():
            smmo.smmo_set_launch(sim.heap.h, smmo.smmo_method_id(name), sim.heap.cls["NodeBase"], *shape)
        for (name, cname), shape in (class_shapes or {}).items():
            smmo.smmo_set_launch(sim.heap.h, smmo.smmo_method_id(name), sim.heap.cls[cname], *shape)
        return sim
    return make


def restart_pull(cur, dt, make):
    s32 = round32(cur)
    sim = make(s32)
    sim.pull(dt)
    s1 = sim.read()
    ref = structure_pull(s32, dt)
    al = ref["nalive"].astype(bool)
    for key, v in (("x", "vx"), ("y", "vy")):
        sc = np.abs(s32[key][al]) + dt * np.abs(s32[v][al])
        assert np.all(np.abs(s1[key][al] - ref[key][al]) <= TOL * np.maximum(sc, 1e-30))


def restart_step(cur, make):
    s32 = round32(cur)
    sim = make(s32)
    sim.compute_step()
    s1 = sim.read()
    ref = structure_step(s32, DT)
    _, _, node_ok, sdiff = structure_compare(s1, ref, s32)
    check_topology(s1, ref, node_ok, sdiff)
    sal = ref["salive"].astype(bool) & ~sdiff
    for key in ("fx", "fy"):
        err = np.abs(s1[key][sal] - ref[key][sal])
        assert np.all(err <= TOL * ref["sf"][sal]), (key, float(np.max(err / np.maximum(ref["sf"][sal], 1e-30))))
    mov = ref["nalive"].astype(bool) & (ref["ntype"] == 2) & node_ok
    for key, sc in (("vx", "svx"), ("vy", "svy"), ("x", "sx"), ("y", "sy")):
        err = np.abs(s1[key][mov] - ref[key][mov])
        assert np.all(err <= TOL * ref[sc][mov]), (key, float(np.max(err / ref[sc][mov])))
    fixed = ref["nalive"].astype(bool) & (ref["ntype"] != 2) & node_ok
    assert np.array_equal(s1["x"][fixed], s32["x"][fixed]) and np.array_equal(s1["y"][fixed], s32["y"][fixed])


def restart_bfs(cur, make):
    s32 = round32(cur)
    sim = make(s32)
    levels = sim.remove_disconnected()
    s1 = sim.read()
    ref = structure_bfs(s32)
    check_topology(s1, ref)
    al = ref["nalive"].astype(bool)
    assert np.array_equal(s1["dist"][al], ref["dist"][al])
    assert levels == ref["levels"], (levels, ref["levels"])


def same_heap(sim, mesh, make, phase):
    """`phase` on the GPU's own heap and on a fresh heap loaded with its
    state: bit for bit the same result.  Returns the state after it."""
    fresh = make(state(mesh, sim.read()))
    ra = phase(sim)
    rb = phase(fresh)
    assert ra == rb
    a, b = sim.read(), fresh.read()
    for key in ("nalive", "salive", "slot", "isp2", "nspr", "dist", "x", "y", "vx", "vy"):
        assert np.array_equal(a[key], b[key]), key
    sal = a["salive"].astype(bool)
    for key in ("fx", "fy"):
        assert np.array_equal(a[key][sal], b[key][sal]), key
    return a


def run_checked(mesh, iters, substeps, pull_mult, make):
    """The oracle trajectory and the GPU's own run, iteration by iteration;
    every phase restarted and same-heap checked.  Returns the oracle's
    (springs broken, nodes removed by BFS) and the GPU run's sim."""
    sim = make(mesh)
    cur = structure_bfs_ready(mesh)
    broken = removed = 0
    for _ in range(iters):
        dt_pull = pull_mult * DT
        restart_pull(cur, dt_pull, make)
        same_heap(sim, mesh, make, lambda s: s.pull(dt_pull))
        cur = structure_pull(cur, dt_pull)
        for _ in range(substeps):
            restart_step(cur, make)
            same_heap(sim, mesh, make, lambda s: s.compute_step())
            cur = structure_step(cur, DT)
            broken += cur["nbroken"]
        restart_bfs(cur, make)
        same_heap(sim, mesh, make, lambda s: s.remove_disconnected())
        before = int(cur["nalive"].sum())
        cur = structure_bfs(cur)
        removed += before - int(cur["nalive"].sum())
    return broken, removed, sim


def structure_bfs_ready(mesh):
    """The mesh as an oracle state (every object alive, no forces yet)."""
    d = dict(mesh)
    S = np.asarray(mesh["p1"]).size
    d.setdefault("fx", np.zeros(S))
    d.setdefault("fy", np.zeros(S))
    d.setdefault("sdel", np.zeros(S, np.uint8))
    return d


@pytest.mark.parametrize("W,H,seed,batch,bfs", [(24, 10, 1, 8, "levels"), (17, 9, 2, 1, "levels"),
                                                (40, 16, 3, 3, "levels"), (24, 10, 1, 0, "queue"),
                                                (40, 16, 3, 0, "queue"), (40, 16, 3, 0, "queue-device-both")])
def test_iterations_phase_by_phase(dev, W, H, seed, batch, bfs):
    print("structure %dx%d seed %d bfs %s batch %d" % (W, H, seed, bfs, batch), flush=True)
    mesh = structure_mesh(W, H, seed=seed, pull_speed=2.0, break_strain=0.02, v_sigma=0.05)
    broken, removed, sim = run_checked(mesh, 8, 10, 10, make_sim(max(batch, 1), bfs=bfs))
    assert broken > 0 and removed > 0, (broken, removed)
    inv = sim.heap.invariants()
    assert inv.hierarchy_violations == 0 and inv.state_violations == 0 and inv.active_violations == 0
    assert inv.type_violations == 0 and inv.empty_allocated == 0
    st = sim.heap.stats()
    c = sim.heap.cls
    s = sim.read()
    assert st.live_objects[c["Spring"]] == int(s["salive"].sum())
    assert sum(st.live_objects[c[n]] for n in ("AnchorNode", "AnchorPullNode", "Node")) == int(s["nalive"].sum())
    assert int(s["nalive"].sum()) < mesh["ntype"].size        # the GPU's own run removed nodes too


@pytest.mark.parametrize("group,wg", [(2, 1024), (4, 64), (2, 64)])
def test_iterations_with_grouped_force_and_node_passes(dev, group, wg):
    """The force and node passes taking 2 or 4 blocks per wavefront iteration,
    in work-groups of 64 or 1,024 threads: every phase restarted against the
    oracle and same-heap checked, with springs breaking and nodes removed."""
    print("structure 40x16 force/node group %d wg %d" % (group, wg), flush=True)
    mesh = structure_mesh(40, 16, seed=3, pull_speed=2.0, break_strain=0.02, v_sigma=0.05)
    cs = {("structure.force", "Spring"): (wg, 0, group), ("structure.node_update", "Node"): (wg, 0, group)}
    broken, removed, _ = run_checked(mesh, 6, 10, 10, make_sim(8, class_shapes=cs))
    assert broken > 0 and removed > 0, (broken, removed)


@pytest.mark.parametrize("bfs", ["queue", "queue-device-visited", "levels"])
@pytest.mark.parametrize("W,H", [(1, 3), (2, 5), (3, 1), (5, 2)])
def test_small_meshes(dev, W, H, bfs):
    """Meshes without free nodes, without pull nodes or with one row."""
    print("structure %dx%d bfs %s" % (W, H, bfs), flush=True)
    mesh = structure_mesh(W, H, seed=W * 10 + H, pull_speed=5.0, break_strain=0.01)
    run_checked(mesh, 3, 5, 5, make_sim(bfs=bfs))


@pytest.mark.parametrize("bfs", sorted(BFS_FORMS))
def test_no_anchor_removes_everything(dev, bfs):
    """Without anchor nodes the BFS visits nothing: every node with springs
    and every spring is deleted (a node loses its last spring and goes with
    it); the level count is 1."""
    mesh = structure_mesh(6, 4, seed=5)
    mesh["ntype"] = np.where(mesh["ntype"] == 0, 2, mesh["ntype"]).astype(np.int32)
    make = make_sim(bfs=bfs)
    restart_bfs(structure_bfs_ready(mesh), make)
    sim = make(mesh)
    sim.remove_disconnected()
    s = sim.read()
    assert s["nalive"].sum() == 0 and s["salive"].sum() == 0 and sim.levels == 1


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
    distances, levels and deletions still equal the oracle's (restarts from
    the oracle trajectory after each iteration's compute steps)."""
    print("structure bfs grid wg %d waves %d" % (wg, waves), flush=True)
    mesh = structure_mesh(40, 16, seed=3, pull_speed=2.0, break_strain=0.02, v_sigma=0.05)
    shapes = {n: (wg, waves, 0) for n in ("structure.bfs_init", "structure.bfs_visit", "structure.bfs_mark")}
    make = make_sim(4, shapes, bfs="levels")
    cur = structure_bfs_ready(mesh)
    removed = 0
    for _ in range(8):
        cur = structure_pull(cur, 10 * DT)
        for _ in range(10):
            cur = structure_step(cur, DT)
        restart_bfs(cur, make)
        before = int(cur["nalive"].sum())
        cur = structure_bfs(cur)
        removed += before - int(cur["nalive"].sum())
    assert removed > 0


def test_queue_bfs_on_a_larger_broken_mesh(dev):
    """The queue BFS at a size where levels hold hundreds of nodes and the
    frontier outgrows the work-group (and the small LDS frontier): a 300 x 200
    mesh that the oracle has pulled apart for a few iterations, restarted on
    the GPU with every BFS form; distances, levels and deletions equal the
    oracle's."""
    print("structure 300x200 queue BFS", flush=True)
    mesh = structure_mesh(300, 200, seed=11, pull_speed=5.0, break_strain=0.05, v_sigma=0.05)
    cur = structure_bfs_ready(mesh)
    for it in range(4):
        cur = structure_pull(cur, 20 * DT)
        for _ in range(20):
            cur = structure_step(cur, DT)
        for bfs in sorted(BFS_FORMS):
            restart_bfs(cur, make_sim(8, bfs=bfs))
        before = int(cur["nalive"].sum())
        cur = structure_bfs(cur)
        print("  iteration %d: %d levels, %d nodes removed" % (it, cur["levels"], before - int(cur["nalive"].sum())),
              flush=True)


def test_queue_bfs_workspace_checks(dev):
    import torch

    mesh = structure_mesh(6, 4, seed=5)
    sim = StructureSim(mesh, DT)
    small = torch.empty(64 + 10, dtype=torch.int32, device=dev)
    with pytest.raises(smmo.SmmoError) as e:
        smmo.smmo_structure_remove_disconnected(sim.heap.h, sim.args, small, sim.bfs_levels)
    assert e.value.status == smmo.SMMO_EINVAL
    bad = smmo.smmo_structure_args.from_buffer_copy(sim.args)
    bad.anchor_class = sim.heap.cls["Spring"]
    with pytest.raises(smmo.SmmoError):
        smmo.smmo_structure_remove_disconnected(sim.heap.h, bad, sim.bfs_work, sim.bfs_levels)
    bad = smmo.smmo_structure_args.from_buffer_copy(sim.args)
    bad.bfs_options = 4
    with pytest.raises(smmo.SmmoError) as e:
        smmo.smmo_structure_remove_disconnected(sim.heap.h, bad, sim.bfs_work, sim.bfs_levels)
    assert e.value.status == smmo.SMMO_EINVAL
    assert sim.remove_disconnected() >= 1
