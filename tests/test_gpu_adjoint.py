"""GPU parity of the reverse sweep through the spring-mesh step, with no GPU
value given to the oracle.

Per reverse step (the gate): the oracle's own forward trajectory (breaking
off) gives the positions x_n; rounded to float32 they are loaded into a fresh
heap, and one GPU reverse step from oracle-made adjoint seeds is compared
with one float64 oracle step from the same values, within 1e-5 of each
quantity's conditioning scale.

End to end, GPU forward and sweep against the float64 oracle adjoint from the
same initial state:
  * a well-conditioned mesh (dt 1e-3): dL/dk, dL/dv0, dL/dx0 normwise 1e-4;
  * the 316 x 317 configuration (dt 1e-5, 200 steps, checkpoints every 20)
    with an oracle-made seed dL/dx_T: dL/dv0 and dL/dx0 normwise 1e-3, and
    dL/dk per spring within the bound the float32 rounding of the positions
    allows (below);
  * the configuration's own loss L = 1/2 |x_T - x_0|^2, whose seed x_T - x_0
    (about 2e-5 against coordinates up to 1.5) is itself dominated by that
    rounding: gradients within the bound it implies, and the directional
    derivative along v0 against a central difference of the float64 forward.
Position rounding bound: each float32 step rounds x + v dt once, so after n
steps a coordinate is off by at most eps_n = n u max|x| (u = 2^-24) plus the
far smaller force and velocity terms.  A term dt (l - L0) (u . g) of dL/dk
then moves by at most dt |g| times: the stretch's error 2 eps_n + (n + 4) u
(l + L0), plus the stretch times the relative error of u . g (the direction
u off by 2 eps_n / l, the float32 sweep's g by 1e-4).  Summed over the steps
with the oracle's agk = sum of dt |g|.
Checkpointing must not change a bit, and the autograd wrapper must return
the same gradients.
"""

import numpy as np
import pytest

from inputs import spring_mesh
from oracle import spring_adjoint, spring_adjoint_step, spring_steps
from paper_1908_05845_amd.adjoint import DiffSpringSim, spring_rollout
from spring_parity import round32

pytestmark = pytest.mark.gpu
TOL = 1e-5
U32 = 2.0 ** -24


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


def reverse_step_restart(mesh, state, dt, seed):
    """One reverse step from the oracle's forward state `state` (float64),
    rounded to float32, with adjoint seeds drawn from `seed`."""
    import torch

    s32 = round32(state)
    rng = np.random.default_rng(seed)
    seeds_np = [rng.standard_normal(mesh["N"]).astype(np.float32) for _ in range(4)]
    seeds = [torch.from_numpy(s).cuda() for s in seeds_np]
    sim = DiffSpringSim(dict(mesh, x=s32["x"], y=s32["y"], vx=s32["vx"], vy=s32["vy"]), dt, steps=1, every=20)
    px, py, lx, ly, lvx, lvy, gk = one_reverse_step(sim, seeds)
    assert np.array_equal(px, s32["x"]) and np.array_equal(py, s32["y"])   # the tape holds the loaded state
    ref = spring_adjoint_step(mesh, s32["x"], s32["y"], dt, *seeds_np)
    for got, key, sc in ((lx, "lx", "slx"), (ly, "ly", "sly"), (lvx, "lvx", "slvx"), (lvy, "lvy", "slvy")):
        err = np.abs(got - ref[key])
        assert np.all(err <= TOL * ref[sc]), (key, float(np.max(err / ref[sc])))
    err = np.abs(gk - ref["gk"])
    assert np.all(err <= TOL * ref["sgk"] + 1e-30), float(np.max(err / np.maximum(ref["sgk"], 1e-30)))


@pytest.mark.parametrize("W,H,steps", [(20, 15, 0), (20, 15, 37), (65, 3, 5), (9, 1, 2)])
def test_reverse_step_matches_oracle(dev, W, H, steps):
    print("adjoint step %dx%d after %d steps" % (W, H, steps), flush=True)
    mesh = spring_mesh(W, H, seed=W + H, v_sigma=0.5)
    dt = 1e-3
    state = spring_steps(mesh, dt, np.inf, steps) if steps else mesh
    reverse_step_restart(mesh, state, dt, steps)


def _gpu_adjoint(mesh, dt, T, every, seed=None):
    """GPU forward and sweep.  Seed dL/dx_T: x_T - x_0 (the loss of the
    configuration), or the given float32 arrays (sx, sy)."""
    import torch

    sim = DiffSpringSim(mesh, dt, T, every)
    xT = sim.forward()
    if seed is None:
        x0 = torch.from_numpy(np.stack([mesh["x"], mesh["y"]], 1).astype(np.float32)).to(xT.device)
        g = xT - x0
        gx_, gy_ = g[:, 0], g[:, 1]
    else:
        gx_, gy_ = (torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(xT.device) for v in seed)
    gk, gv, gx = sim.backward(gx_, gy_)
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


# ------------------------------------------------ the 316 x 317 configuration --
C5 = dict(W=316, H=317, dt=1e-5, T=200, every=20)


@pytest.fixture(scope="module")
def config5():
    mesh = spring_mesh(C5["W"], C5["H"])
    assert mesh["N"] == 100_172
    return mesh


def _stretch_bound(mesh, T, ref):
    """Per spring, the bound on the float32 error of one step's term of dL/dk
    per unit dt |g| (see the module text); ref = the oracle's adjoint (its
    final positions give the stretch, doubled as a bound of all steps')."""
    xmax = float(max(np.max(np.abs(mesh["x"])), np.max(np.abs(mesh["y"])))) * 1.01
    eps = T * U32 * xmax
    L0 = np.asarray(mesh["L0"], np.float64)
    a, b = mesh["a"], mesh["b"]
    l = np.hypot(ref["xT"][b] - ref["xT"][a], ref["yT"][b] - ref["yT"][a])
    stretch = 2 * np.abs(l - L0) + 2 * eps
    return 2 * eps + (T + 4) * U32 * 2.02 * L0 + stretch * (2 * eps / (0.5 * L0) + 1e-4)


def test_config5_reverse_steps_along_the_oracle_trajectory(dev, config5):
    mesh = config5
    dt = C5["dt"]
    state, n = mesh, 0
    for k in (0, 1, 20, 100, 199):
        if k > n:
            state = spring_steps(state, dt, np.inf, k - n)
            n = k
        print("  config 5 reverse step at n = %d" % k, flush=True)
        reverse_step_restart(mesh, state, dt, 1000 + k)


def test_config5_sweep_with_an_oracle_seed(dev, config5):
    """The whole checkpointed sweep from a seed dL/dx_T drawn by the test:
    only the Jacobians' dependence on the float32 positions separates the
    GPU's gradients from the float64 oracle's.  dL/dv0 and dL/dx0 see it
    through the stretch part of K, a few times u max|x| T / l relative;
    dL/dk directly (bound above)."""
    mesh = config5
    dt, T, every = C5["dt"], C5["T"], C5["every"]
    rng = np.random.default_rng(5)
    sx = rng.standard_normal(mesh["N"]).astype(np.float32)
    sy = rng.standard_normal(mesh["N"]).astype(np.float32)
    print("  config 5 sweep, oracle seed", flush=True)
    gk, gv, gx, _ = _gpu_adjoint(mesh, dt, T, every, seed=(sx, sy))
    r0 = spring_adjoint(mesh, dt, T, every=every)
    ref = spring_adjoint(mesh, dt, T, every=every, xhat=r0["xT"] - sx, yhat=r0["yT"] - sy)
    for got, want in ((gv[:, 0], ref["gvx"]), (gv[:, 1], ref["gvy"]), (gx[:, 0], ref["gx"]),
                      (gx[:, 1], ref["gy"])):
        rel = np.linalg.norm(got - want) / np.linalg.norm(want)
        assert rel <= 1e-3, rel
    bound = _stretch_bound(mesh, T, r0) * ref["agk"] + TOL * np.abs(ref["gk"])
    err = np.abs(gk - ref["gk"])
    assert np.all(err <= bound), float(np.max(err / bound))
    print("  dL/dk relative error %.3g (normwise), at most %.3g of its bound"
          % (np.linalg.norm(gk - ref["gk"]) / np.linalg.norm(ref["gk"]), float(np.max(err / bound))), flush=True)


def test_config5_own_loss(dev, config5):
    """L = 1/2 |x_T - x_0|^2 at the configuration: the GPU's seed x_T - x_0
    differs from the float64 one by at most eps_T per coordinate, so the
    gradients may differ by that error carried through the (linear) sweep:
    |dL/dv0 error| <= (|eps_T| / |x_T - x_0|) |dL/dv0| with a factor 2 for the
    sweep's amplification; dL/dk as above plus the same relative term.  The
    directional derivative along a random v0 direction is checked against a
    central difference of the float64 forward under the same bound."""
    mesh = config5
    dt, T, every = C5["dt"], C5["T"], C5["every"]
    print("  config 5 own loss", flush=True)
    gk, gv, gx, xT = _gpu_adjoint(mesh, dt, T, every)
    ref = spring_adjoint(mesh, dt, T, every=every)
    lam = np.concatenate([ref["xT"] - mesh["x"], ref["yT"] - mesh["y"]])
    xabs = np.concatenate([np.abs(mesh["x"]), np.abs(mesh["y"])]).astype(np.float64) * 1.01
    rel_seed = 2 * np.linalg.norm(T * U32 * xabs) / np.linalg.norm(lam)
    gvr = np.concatenate([ref["gvx"], ref["gvy"]])
    ev = np.linalg.norm(np.concatenate([gv[:, 0], gv[:, 1]]) - gvr) / np.linalg.norm(gvr)
    assert ev <= rel_seed, (ev, rel_seed)
    bound = _stretch_bound(mesh, T, ref) * ref["agk"]
    ek = np.linalg.norm(gk - ref["gk"])
    assert ek <= np.linalg.norm(bound) + rel_seed * np.linalg.norm(ref["gk"]), ek
    # directional derivative along v0 against the float64 forward's central difference
    rng = np.random.default_rng(317)
    dvx, dvy = rng.standard_normal(mesh["N"]), rng.standard_normal(mesh["N"])
    h = 1e-4 * float(np.sqrt(np.mean(mesh["vx"].astype(np.float64) ** 2 + mesh["vy"].astype(np.float64) ** 2)))

    def loss(vx, vy):
        r = spring_steps(dict(mesh, vx=vx, vy=vy), dt, np.inf, T)
        return 0.5 * np.sum((r["x"] - mesh["x"]) ** 2 + (r["y"] - mesh["y"]) ** 2)

    vx, vy = mesh["vx"].astype(np.float64), mesh["vy"].astype(np.float64)
    fd = (loss(vx + h * dvx, vy + h * dvy) - loss(vx - h * dvx, vy - h * dvy)) / (2 * h)
    ad = float(np.dot(gv[:, 0], dvx) + np.dot(gv[:, 1], dvy))
    assert abs(ad - fd) <= rel_seed * np.linalg.norm(gvr) * np.linalg.norm(np.concatenate([dvx, dvy])), (ad, fd)
    print("  dL/dv0 relative error %.3g (bound %.3g); directional derivative %.6g vs float64 difference %.6g"
          % (ev, rel_seed, ad, fd), flush=True)


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
