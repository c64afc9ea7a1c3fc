"""GPU parity of the spring-mass mesh with partially inlined adjacency
(thesis Ch.4 sec.4.3.1 "SOA with Partial Inlining": K slots inline, the rest
outside the heap) on meshes with high-degree hub nodes, against the
any-degree float64 oracle: live springs and every adjacency slot exact
(break decisions that differ from the float64 rule only at ties, see
spring_parity), forces and node states within 1e-5 of their conditioning
scale."""

import numpy as np
import pytest

from inputs import hub_mesh
from paper_1908_05845_amd import smmo
from paper_1908_05845_amd.sims import SpringPiSim
from spring_parity import mesh_step

pytestmark = pytest.mark.gpu

TOL = 1e-5
TOPO = ("a", "b", "k", "L0", "slot_a", "slot_b")


def check_step(sim, mesh, dt, limit):
    st = sim.read()
    assert (st["adj"] != -2).all(), "a slot names a dead spring"
    d = {k: mesh[k] for k in TOPO}
    for k in ("x", "y", "vx", "vy", "m", "adj", "adj_is_b"):
        d[k] = st[k]
    sim.step(1)
    s1 = sim.read()
    ref, _, _ = mesh_step(d, dt, limit, st["alive"], st["fx"], st["fy"], s1["alive"], any_degree=True)
    assert np.array_equal(s1["alive"], ref["alive"])
    assert np.array_equal(s1["adj"], ref["adj"])
    al = ref["alive"].astype(bool)
    for key in ("fx", "fy"):
        err = np.abs(s1[key][al] - ref[key][al])
        assert np.all(err <= TOL * ref["sf"][al]), key
    for key, sc in (("vx", "svx"), ("vy", "svy"), ("x", "sx"), ("y", "sy")):
        assert np.all(np.abs(s1[key] - ref[key]) <= TOL * ref[sc]), key
    return ref["nbroken"]


@pytest.mark.parametrize("K", [1, 2, 4, 8])
def test_hub_mesh_with_breaking(dev, K):
    print("spring_pi hub mesh K %d" % K, flush=True)
    mesh = hub_mesh(40, 24, hubs=6, hub_springs=36, v_sigma=1.0)
    assert np.asarray(mesh["adj"]).shape[1] > 8
    sim = SpringPiSim(mesh, 1e-4, K, strain_limit=0.01)
    broken = 0
    for _ in range(60):
        broken += check_step(sim, mesh, 1e-4, 0.01)
    assert broken > 10, broken
    inv = sim.heap.invariants()
    assert inv.hierarchy_violations == 0 and inv.state_violations == 0 and inv.type_violations == 0


def test_all_slots_inline(dev):
    """K = the largest degree: no slot lives outside the heap."""
    mesh = hub_mesh(20, 12, hubs=3, hub_springs=12, v_sigma=1.0)
    D = np.asarray(mesh["adj"]).shape[1]
    if D > 32 - 8:
        pytest.skip("degree too high to inline")
    sim = SpringPiSim(mesh, 1e-4, D, strain_limit=0.01)
    assert sim.args.overflow_len == 0
    for _ in range(20):
        check_step(sim, mesh, 1e-4, 0.01)


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
