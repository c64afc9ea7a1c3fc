"""GPU parity of batched execution: many independent spring meshes of uneven
size in one heap, stepped by the same do-alls (one launch per phase for all
meshes), the step loop captured in a HIP graph.  The oracle result of the
batch is the concatenation of the separate meshes' results (pinned on the
CPU); here checked steps restart from the oracle's own trajectory of the
concatenated mesh and the GPU's own run passes the same-heap check, as for
a single mesh (spring_parity).  Graph replays are compared with the same
number of launched steps on a second heap built from the same meshes, bit
for bit: the kernels are deterministic (no float atomics, slot-order sums),
so a replay that does other work than the launched steps shows."""

import numpy as np
import pytest

from inputs import batched_meshes, concat_meshes, spring_mesh
from oracle import spring_steps
from paper_1908_05845_amd.sims import SpringSim
from spring_parity import mesh_restart, same_heap

pytestmark = pytest.mark.gpu
STATE = ("x", "y", "vx", "vy", "alive", "fx", "fy", "adj")


def same_state(a, b):
    sa, sb = a.read(), b.read()
    for k in STATE:
        assert np.array_equal(sa[k], sb[k]), k


def test_small_batch_every_step(dev):
    rng = np.random.default_rng(4)
    meshes = [spring_mesh(int(rng.integers(2, 30)), int(rng.integers(2, 20)), seed=100 + i, v_sigma=1.0)
              for i in range(12)]
    mesh = concat_meshes(meshes)
    dt, limit = 1e-4, 0.3
    make = lambda state: SpringSim(state, dt, limit)
    sim = make(mesh)
    cur = dict(mesh, alive=np.ones(mesh["S"], np.uint8))
    broken = 0
    for _ in range(60):
        mesh_restart(cur, dt, limit, make)
        same_heap(sim, mesh, make)
        cur = spring_steps(cur, dt, limit, 1, alive=cur["alive"])
        broken += cur["nbroken"]
    assert broken > 0 and int(sim.read()["alive"].sum()) < mesh["S"]


def test_batched_config_graph_captured(dev):
    """The 256-mesh configuration: a graph of 10 steps replayed on one heap;
    the same steps launched on a twin heap; restarts from the oracle
    trajectory and same-heap checks of the twin among those steps; after
    each of 22 replays the two heaps hold the same state bit for bit, and
    the replayed heap passes the same-heap check at the end."""
    import torch

    print("batched 256 meshes", flush=True)
    meshes = batched_meshes(256)
    mesh = concat_meshes(meshes)
    assert 3_000_000 < mesh["N"] < 5_000_000
    dt, limit = 1e-5, 0.3
    make = lambda state: SpringSim(state, dt, limit)
    sim = make(mesh)
    twin = make(mesh)
    cur = dict(mesh, alive=np.ones(mesh["S"], np.uint8))
    sim.step(2)
    twin.step(2)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s = torch.cuda.current_stream()
        for _ in range(10):
            sim.step(1, stream=s)
    sim.step(1)
    twin.step(1)
    cur = spring_steps(cur, dt, limit, 3, alive=cur["alive"])
    torch.cuda.synchronize()
    g.replay()
    torch.cuda.synchronize()
    for i in range(10):
        if i in (0, 9):
            print("  restart at step %d" % (3 + i), flush=True)
            mesh_restart(cur, dt, limit, make)
        if i in (0, 5, 9):
            print("  same-heap check of the launched run at step %d" % (3 + i), flush=True)
            same_heap(twin, mesh, make)
        else:
            twin.step(1)
        cur = spring_steps(cur, dt, limit, 1, alive=cur["alive"])
    same_state(sim, twin)
    # 21 more replays, each against ten launched steps, eager reads between
    for r in range(21):
        g.replay()
        twin.step(10)
        torch.cuda.synchronize()
        if r % 5 == 4 or r == 20:
            print("  replay %d compared" % (r + 2), flush=True)
            same_state(sim, twin)
    same_heap(sim, mesh, make)
    assert sim.heap.stats().device_error == 0 and twin.heap.stats().device_error == 0
