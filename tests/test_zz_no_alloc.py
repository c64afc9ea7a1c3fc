"""The allocation-free BFS removal (smmo_structure_remove_disconnected_noalloc,
the workspace being the library's own device array) against the entry point
with a caller workspace, on the same states: every node's and spring's
liveness, every slot, spring count and distance, and the level count, bit
for bit; and against the oracle.  Two calls in a row, the second on a smaller
mesh (the array keeps the first call's contents), and the size limit."""

import numpy as np
import pytest

from inputs import structure_mesh
from oracle import structure_bfs, structure_pull, structure_step
from paper_1908_05845_amd import smmo
from paper_1908_05845_amd.sims import StructureSim
from spring_parity import round32

pytestmark = pytest.mark.gpu
DT = 1e-4


def broken_state(W, H, seed):
    """An oracle state of a W x H mesh pulled until parts come loose."""
    mesh = structure_mesh(W, H, seed=seed, pull_speed=5.0, break_strain=0.05, v_sigma=0.05)
    S = np.asarray(mesh["p1"]).size
    cur = dict(mesh, fx=np.zeros(S), fy=np.zeros(S), sdel=np.zeros(S, np.uint8))
    for _ in range(2):
        cur = structure_pull(cur, 20 * DT)
        for _ in range(20):
            cur = structure_step(cur, DT)
    return round32(cur)


def run_both(state):
    import torch

    a = StructureSim(state, DT)
    b = StructureSim(state, DT)
    smmo.smmo_structure_remove_disconnected(a.heap.h, a.args, a.bfs_work, a.bfs_levels)
    lv = torch.full((1,), -7, dtype=torch.int32, device=b.heap.dev)
    smmo.smmo_structure_remove_disconnected_noalloc(b.heap.h, b.args, lv)
    a.heap.sync()
    b.heap.sync()
    ra, rb = a.read(), b.read()
    for key in ("nalive", "salive", "slot", "isp2", "nspr", "dist"):
        assert np.array_equal(ra[key], rb[key]), key
    la, lb = int(a.bfs_levels.cpu().item()), int(lv.cpu().item())
    assert la == lb, (la, lb)
    ref = structure_bfs(state)
    al = ref["nalive"].astype(bool)
    assert np.array_equal(rb["nalive"], ref["nalive"]) and np.array_equal(rb["salive"], ref["salive"])
    assert np.array_equal(rb["dist"][al], ref["dist"][al]) and lb == ref["levels"]
    return lb, int(state["nalive"].sum()) - int(al.sum())


def test_no_alloc_bfs_matches_the_workspace_entry_point(dev):
    print("no-alloc BFS: 160x120 then 40x16", flush=True)
    big = run_both(broken_state(160, 120, 3))
    small = run_both(broken_state(40, 16, 4))
    print("  levels and removed nodes: %s then %s" % (big, small), flush=True)
    assert big[0] > small[0] > 1 and big[1] > 0


def test_no_alloc_bfs_refuses_a_heap_beyond_its_array(dev):
    import torch

    mesh = structure_mesh(6, 4, seed=5)
    sim = StructureSim(mesh, DT, extra_blocks=16400)
    lv = torch.zeros(1, dtype=torch.int32, device=sim.heap.dev)
    with pytest.raises(smmo.SmmoError) as e:
        smmo.smmo_structure_remove_disconnected_noalloc(sim.heap.h, sim.args, lv)
    assert e.value.status == smmo.SMMO_EINVAL
    assert "16,384" in str(e.value)
