"""GPU parity of batched execution: many independent spring meshes of uneven
size in one heap, stepped by the same do-alls (one launch per phase for all
meshes), the step loop captured in a HIP graph.  The oracle result of the
batch is the concatenation of the separate meshes' results (pinned on the
CPU); here each checked step is compared object by object from the GPU's own
state, as for a single mesh (break decisions that differ from the float64
rule only at ties, see spring_parity).  Graph replays are compared with the
same number of launched steps on a second heap built from the same meshes,
bit for bit: the kernels are deterministic (no float atomics, slot-order
sums), so a replay that does other work than the launched steps shows."""

import numpy as np
import pytest

from inputs import batched_meshes, concat_meshes, spring_mesh
from paper_1908_05845_amd.sims import SpringSim
from spring_parity import mesh_step

pytestmark = pytest.mark.gpu
TOL = 1e-5
TOPO = ("a", "b", "k", "L0", "slot_a", "slot_b")
STATE = ("x", "y", "vx", "vy", "alive", "fx", "fy", "adj")


def check_step(sim, mesh, dt, limit, step_fn):
    st = sim.read()
    d = {k: mesh[k] for k in TOPO}
    for k in ("x", "y", "vx", "vy", "m", "adj", "adj_is_b"):
        d[k] = st[k]
    step_fn()
    s1 = sim.read()
    ref, near, flipped = mesh_step(d, dt, limit, st["alive"], st["fx"], st["fy"], s1["alive"])
    assert np.array_equal(s1["alive"], ref["alive"])
    assert np.array_equal(s1["adj"], ref["adj"])
    for key, sc in (("vx", "svx"), ("vy", "svy"), ("x", "sx"), ("y", "sy")):
        assert np.all(np.abs(s1[key] - ref[key]) <= TOL * ref[sc]), key
    al = ref["alive"].astype(bool)
    for key in ("fx", "fy"):
        assert np.all(np.abs(s1[key][al] - ref[key][al]) <= TOL * ref["sf"][al]), key
    return ref["nbroken"], near, flipped


def same_state(a, b):
    sa, sb = a.read(), b.read()
    for k in STATE:
        assert np.array_equal(sa[k], sb[k]), k


def test_small_batch_every_step(dev):
    rng = np.random.default_rng(4)
    meshes = [spring_mesh(int(rng.integers(2, 30)), int(rng.integers(2, 20)), seed=100 + i, v_sigma=1.0)
              for i in range(12)]
    mesh = concat_meshes(meshes)
    sim = SpringSim(mesh, 1e-4, 0.3)
    broken = sum(check_step(sim, mesh, 1e-4, 0.3, lambda: sim.step(1))[0] for _ in range(60))
    assert broken > 0


def test_batched_config_graph_captured(dev):
    """The 256-mesh configuration: a graph of 10 steps replayed on one heap;
    the same steps launched on a twin heap, each checked against the oracle;
    after each of 22 replays the two heaps hold the same state bit for bit."""
    import torch

    print("batched 256 meshes", flush=True)
    meshes = batched_meshes(256)
    mesh = concat_meshes(meshes)
    assert 3_000_000 < mesh["N"] < 5_000_000
    dt, limit = 1e-5, 0.3
    sim = SpringSim(mesh, dt, limit)
    twin = SpringSim(mesh, dt, limit)
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
    torch.cuda.synchronize()
    # first replay: the twin's ten launched steps are each checked strictly
    g.replay()
    torch.cuda.synchronize()
    near = flipped = 0
    for i in range(10):
        print("  launched step %d checked" % i, flush=True)
        _, n, f = check_step(twin, mesh, dt, limit, lambda: twin.step(1))
        near += n
        flipped += f
    same_state(sim, twin)
    # 21 more replays, each against ten launched steps, eager reads between
    for r in range(21):
        g.replay()
        twin.step(10)
        torch.cuda.synchronize()
        if r % 5 == 4 or r == 20:
            print("  replay %d compared" % (r + 2), flush=True)
            same_state(sim, twin)
    # one more step, checked object by object from the GPU state
    _, n, f = check_step(sim, mesh, dt, limit, lambda: sim.step(1))
    print("  ties within the band: %d, decided otherwise: %d" % (near + n, flipped + f), flush=True)
    assert sim.heap.stats().device_error == 0 and twin.heap.stats().device_error == 0
