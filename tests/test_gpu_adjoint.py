"""GPU parity of the reverse sweep through the spring-mesh step.

Per reverse step (the gate): from a GPU state (positions x_n in float32 and
adjoints at step n+1), one GPU reverse step is compared with one float64
oracle step from exactly those values, within 1e-5 of each quantity's
conditioning scale.  End to end on a well-conditioned mesh: GPU gradients
dL/dk and dL/dv0 against the float64 oracle adjoint, normwise within 1e-4.
Checkpointing must not change a bit, and the autograd wrapper must return
the same gradients.
"""

import numpy as np
import pytest

from inputs import spring_mesh
from oracle import spring_adjoint, spring_adjoint_step
from paper_1908_05845_amd.adjoint import DiffSpringSim, spring_rollout

pytestmark = pytest.mark.gpu
TOL = 1e-5


def one_reverse_step(sim, seeds):
    """GPU: positions of the current state into tape slot 0, then one reverse
    step from the seeded adjoints.  Returns (px, py, lx, ly, lvx, lvy, gk) as numpy."""
    sim._do(sim.cn, "adjoint.seed", sim._aargs(sim.tape, seeds=seeds, count=sim.N))
    sim._do(sim.cs, "adjoint.zero", sim._aargs(sim.tape))
    sim._do(sim.cn, "adjoint.record", sim._aargs(sim.tape, slot=0))
    sim._do(sim.cn, "adjoint.node", sim._aargs(sim.tape, mode=2))
    sim._do(sim.cs, "adjoint.spring", sim._aargs(sim.tape, slot=0))
    sim._do(sim.cn, "adjoint.node", sim._aargs(sim.tape, mode=1))
    sim.heap.sync()
    pos = sim.positions().cpu().numpy()
    gk, gv, gx = (t.cpu().numpy() for t in sim.gradients())
    return pos[:, 0], pos[:, 1], gx[:, 0], gx[:, 1], gv[:, 0], gv[:, 1], gk


@pytest.mark.parametrize("W,H,steps", [(20, 15, 0), (20, 15, 37), (65, 3, 5), (316, 317, 3)])
def test_reverse_step_matches_oracle(dev, W, H, steps):
    import torch

    print("adjoint step %dx%d after %d steps" % (W, H, steps), flush=True)
    mesh = spring_mesh(W, H, seed=W + H, v_sigma=0.5)
    dt = 1e-3 if W < 100 else 1e-5
    sim = DiffSpringSim(mesh, dt, steps=max(steps, 1), every=20)
    for _ in range(steps):
        sim.step()
    rng = np.random.default_rng(steps)
    seeds_np = [rng.standard_normal(mesh["N"]).astype(np.float32) for _ in range(4)]
    seeds = [torch.from_numpy(s).to(dev) for s in seeds_np]
    px, py, lx, ly, lvx, lvy, gk = one_reverse_step(sim, seeds)
    ref = spring_adjoint_step(mesh, px, py, dt, *seeds_np)
    for got, key, sc in ((lx, "lx", "slx"), (ly, "ly", "sly"), (lvx, "lvx", "slvx"), (lvy, "lvy", "slvy")):
        err = np.abs(got - ref[key])
        assert np.all(err <= TOL * ref[sc]), (key, float(np.max(err / ref[sc])))
    err = np.abs(gk - ref["gk"])
    assert np.all(err <= TOL * ref["sgk"] + 1e-30), float(np.max(err / np.maximum(ref["sgk"], 1e-30)))


def _gpu_adjoint(mesh, dt, T, every):
    import torch

    sim = DiffSpringSim(mesh, dt, T, every)
    xT = sim.forward()
    x0 = torch.from_numpy(np.stack([mesh["x"], mesh["y"]], 1).astype(np.float32)).to(xT.device)
    g = xT - x0
    gk, gv, gx = sim.backward(g[:, 0], g[:, 1])
    return gk.cpu().numpy(), gv.cpu().numpy(), gx.cpu().numpy(), xT.cpu().numpy()


def test_end_to_end_against_float64_adjoint(dev):
    mesh = spring_mesh(20, 16, seed=5, v_sigma=0.5)
    dt, T = 1e-3, 200
    gk, gv, gx, xT = _gpu_adjoint(mesh, dt, T, 20)
    ref = spring_adjoint(mesh, dt, T, every=20)
    assert np.linalg.norm(xT[:, 0] - ref["xT"]) <= 1e-5 * np.linalg.norm(ref["xT"])
    for got, want in ((gk, ref["gk"]), (gv[:, 0], ref["gvx"]), (gv[:, 1], ref["gvy"]),
                      (gx[:, 0], ref["gx"]), (gx[:, 1], ref["gy"])):
        rel = np.linalg.norm(got - want) / np.linalg.norm(want)
        assert rel <= 1e-4, rel


def test_checkpointing_changes_no_bit(dev):
    mesh = spring_mesh(12, 9, seed=8, v_sigma=0.5)
    a = _gpu_adjoint(mesh, 1e-3, 60, 20)
    b = _gpu_adjoint(mesh, 1e-3, 60, 60)
    c = _gpu_adjoint(mesh, 1e-3, 60, 7)
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, y) and np.array_equal(x, z)


def test_autograd_wrapper(dev):
    import torch

    mesh = spring_mesh(10, 8, seed=3, v_sigma=0.5)
    dt, T = 1e-3, 50
    k = torch.from_numpy(mesh["k"]).to(dev).requires_grad_(True)
    v0 = torch.from_numpy(np.stack([mesh["vx"], mesh["vy"]], 1)).to(dev).requires_grad_(True)
    xT = spring_rollout(k, v0, mesh, dt, T, 10)
    x0 = torch.from_numpy(np.stack([mesh["x"], mesh["y"]], 1)).to(dev)
    loss = 0.5 * ((xT - x0) ** 2).sum()
    loss.backward()
    ref = spring_adjoint(mesh, dt, T, every=10)
    assert abs(loss.item() - ref["loss"]) <= 1e-4 * ref["loss"]
    gk = k.grad.cpu().numpy()
    assert np.linalg.norm(gk - ref["gk"]) <= 1e-4 * np.linalg.norm(ref["gk"])
    gv = v0.grad.cpu().numpy()
    want = np.stack([ref["gvx"], ref["gvy"]], 1)
    assert np.linalg.norm(gv - want) <= 1e-4 * np.linalg.norm(want)


def test_graph_replay_matches_eager(dev):
    """Forward (from the step-0 checkpoint) and reverse sweep captured in one
    HIP graph: every replay, with eager work and synchronizations between
    replays, gives the eager run's positions and gradients bit for bit."""
    import torch

    print("adjoint graph replay 20x15", flush=True)
    mesh = spring_mesh(20, 15, seed=12, v_sigma=0.5)
    dt, T, every = 1e-3, 60, 20
    sim = DiffSpringSim(mesh, dt, T, every)
    xT = sim.forward()
    x0 = torch.from_numpy(np.stack([mesh["x"], mesh["y"]], 1).astype(np.float32)).to(dev)
    g = (xT - x0).contiguous()
    sx, sy = g[:, 0].contiguous(), g[:, 1].contiguous()
    want = [t.cpu().numpy() for t in sim.backward(sx, sy)] + [xT.cpu().numpy()]
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        st = torch.cuda.current_stream().cuda_stream
        sim.restart(st)
        sim.run_forward(st)
        sim.run_backward(sx, sy, stream=st)
    torch.cuda.synchronize()
    for rep in range(3):
        sim.step()                      # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = [t.cpu().numpy() for t in sim.gradients()]
        for a, b in zip(got, want[:3]):
            assert np.array_equal(a, b), rep
    sim.restart()
    assert np.array_equal(sim.forward().cpu().numpy(), want[3])


def test_step_node_tape_and_forward_step(dev):
    """adjoint.step_node writes to tape plane pair `slot` exactly the positions
    it leaves in the heap, moves the mesh as spring.node_update does (1e-6),
    and refuses a slot beyond the tape."""
    import torch

    from paper_1908_05845_amd import smmo

    print("adjoint step_node tape 33x21", flush=True)
    mesh = spring_mesh(33, 21, seed=21, v_sigma=0.5)
    a = DiffSpringSim(mesh, 1e-3, steps=4, every=4)
    b = DiffSpringSim(mesh, 1e-3, steps=4, every=4)
    mid_node = smmo.smmo_method_id("spring.node_update")
    for t in range(3):
        a.L_force(a._stream())
        a._do(a.cn, "adjoint.step_node", a._aargs(a.tape, slot=t + 1))
        b.L_force(b._stream())
        smmo.smmo_parallel_do(b.heap.h, b.cn, mid_node, b.fargs)
        a.heap.sync()
        b.heap.sync()
        pa, pb = a.positions().cpu().numpy(), b.positions().cpu().numpy()
        np.testing.assert_allclose(pa, pb, rtol=1e-6, atol=0)
        h = a.node_h.long()
        tx = a.tape[(2 * (t + 1)) * a.plane + h].cpu().numpy()
        ty = a.tape[(2 * (t + 1) + 1) * a.plane + h].cpu().numpy()
        assert np.array_equal(tx, pa[:, 0]) and np.array_equal(ty, pa[:, 1]), t
    with pytest.raises(smmo.SmmoError):
        a._do(a.cn, "adjoint.step_node", a._aargs(a.tape, slot=4))
    torch.cuda.synchronize()


@pytest.mark.parametrize("group", [2, 4])
def test_step_node_groups_change_no_bit(dev, group):
    """The node pass's blocks per wavefront iteration (1, 2 or 4) leave the
    positions and gradients of a checkpointed sweep unchanged bit for bit."""
    from paper_1908_05845_amd import smmo

    print("adjoint step_node group %d" % group, flush=True)
    mesh = spring_mesh(40, 30, seed=4, v_sigma=0.5)
    want = _gpu_adjoint(mesh, 1e-3, 30, 7)
    import torch

    sim = DiffSpringSim(mesh, 1e-3, 30, 7)
    smmo.smmo_set_launch(sim.heap.h, smmo.smmo_method_id("adjoint.step_node"), sim.cn, 0, 0, group)
    xT = sim.forward()
    x0 = torch.from_numpy(np.stack([mesh["x"], mesh["y"]], 1).astype(np.float32)).to(xT.device)
    g = xT - x0
    got = [t.cpu().numpy() for t in sim.backward(g[:, 0], g[:, 1])] + [xT.cpu().numpy()]
    for x, y in zip(got, want):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("T,every", [(60, 7), (41, 20), (40, 20)])
def test_overlapped_sweep_equals_single_stream(dev, T, every):
    """The reverse sweep with each segment's recompute on a second stream
    gives the single-stream sweep's gradients bit for bit, run twice in a row."""
    import torch

    print("adjoint overlap T=%d every=%d" % (T, every), flush=True)
    mesh = spring_mesh(30, 22, seed=T + every, v_sigma=0.5)
    x0 = torch.from_numpy(np.stack([mesh["x"], mesh["y"]], 1).astype(np.float32)).to(dev)
    ref = DiffSpringSim(mesh, 1e-3, T, every)
    xT = ref.forward()
    g = (xT - x0).contiguous()
    sx, sy = g[:, 0].contiguous(), g[:, 1].contiguous()
    ref.run_backward(sx, sy, overlap=False)
    ref.heap.sync()
    want = [t.cpu().numpy() for t in ref.gradients()]
    # a fresh sim on a created stream: its first sweep already overlaps
    ms = torch.cuda.Stream()
    with torch.cuda.stream(ms):
        sim = DiffSpringSim(mesh, 1e-3, T, every)
        assert sim.overlap
        assert np.array_equal(sim.forward().cpu().numpy(), xT.cpu().numpy())
        for rep in range(2):
            sim.run_backward(sx, sy)
            sim.heap.sync()
            torch.cuda.synchronize()
            got = [t.cpu().numpy() for t in sim.gradients()]
            for a, b in zip(got, want):
                assert np.array_equal(a, b), rep
