"""GPU parity of the spring-mass mesh with partially inlined adjacency
(thesis Ch.4 sec.4.3.1 "SOA with Partial Inlining": K slots inline, the rest
outside the heap) on meshes with high-degree hub nodes, against the
any-degree float64 oracle.  As for the plain mesh (spring_parity): restarts
from the oracle's own trajectory (live springs and every adjacency slot
exact, ties aside; forces and node states within 1e-5 of their conditioning
scale) and the same-heap check of the GPU's unrestarted run."""

import numpy as np
import pytest

from inputs import hub_mesh
from oracle import spring_steps_deg
from paper_1908_05845_amd import smmo
from paper_1908_05845_amd.sims import SpringPiSim
from spring_parity import mesh_restart, same_heap

pytestmark = pytest.mark.gpu


def run_checked(mesh, dt, limit, K, steps):
    """Oracle trajectory and the GPU's own run side by side, restart and
    same-heap checks every step.  Returns (oracle breaks, GPU breaks, sim)."""
    make = lambda state: SpringPiSim(state, dt, K, strain_limit=limit)
    sim = make(mesh)
    cur = dict(mesh, alive=np.ones(np.asarray(mesh["a"]).size, np.uint8))
    broken = 0
    for _ in range(steps):
        mesh_restart(cur, dt, limit, make, any_degree=True)
        same_heap(sim, mesh, make)
        cur = spring_steps_deg(cur, dt, limit, 1, alive=cur["alive"])
        broken += cur["nbroken"]
    gpu_broken = int(np.asarray(mesh["a"]).size - sim.read()["alive"].sum())
    return broken, gpu_broken, sim


@pytest.mark.parametrize("K", [1, 2, 4, 8])
def test_hub_mesh_with_breaking(dev, K):
    print("spring_pi hub mesh K %d" % K, flush=True)
    mesh = hub_mesh(40, 24, hubs=6, hub_springs=36, v_sigma=1.0)
    assert np.asarray(mesh["adj"]).shape[1] > 8
    broken, gpu_broken, sim = run_checked(mesh, 1e-4, 0.01, K, 60)
    assert broken > 10 and gpu_broken > 10, (broken, gpu_broken)
    inv = sim.heap.invariants()
    assert inv.hierarchy_violations == 0 and inv.state_violations == 0 and inv.type_violations == 0


def test_all_slots_inline(dev):
    """K = the largest degree: no slot lives outside the heap."""
    mesh = hub_mesh(20, 12, hubs=3, hub_springs=12, v_sigma=1.0)
    D = np.asarray(mesh["adj"]).shape[1]
    if D > 32 - 8:
        pytest.skip("degree too high to inline")
    assert SpringPiSim(mesh, 1e-4, D, strain_limit=0.01).args.overflow_len == 0
    run_checked(mesh, 1e-4, 0.01, D, 20)


def test_bad_overflow_length_is_a_device_error(dev):
    """An overflow array shorter than the slots need: the kernels stay in
    bounds and report SMMO_EDEVICE."""
    mesh = hub_mesh(12, 8, hubs=2, hub_springs=16)
    sim = SpringPiSim(mesh, 1e-4, 2)
    bad = smmo.smmo_spring_pi_args.from_buffer_copy(sim.args)
    bad.overflow_len = 1
    smmo.smmo_parallel_do(sim.heap.h, sim.heap.cls["Node"], sim.m_node, bad)
    with pytest.raises(smmo.SmmoError) as e:
        sim.heap.sync()
    assert e.value.status == smmo.SMMO_EDEVICE
