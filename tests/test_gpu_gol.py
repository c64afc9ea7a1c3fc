"""GPU parity of Game of Life in SMMO form against the oracle: bit-exact cell
states, neighbour counts and the canonical Alive set after every generation
(objects are created on birth and deleted on death by the device allocator)."""

import numpy as np
import pytest

from inputs import gol_init
from oracle import GolWorld
from paper_1908_05845_amd import smmo
from paper_1908_05845_amd.sims import GolSim

pytestmark = pytest.mark.gpu


def compare_run(W, H, init, steps, cfg=None, every=1, concurrent=False, fused=False):
    sim = GolSim(W, H, init, cfg=cfg, concurrent=concurrent, fused=fused)
    ref = GolWorld(W, H, init)
    for s in range(1, steps + 1):
        sim.step(1)
        ref.step(1)
        if s % every == 0 or s == steps:
            gs, gc, ga = sim.read()
            rs, rc, ra = ref.read()
            assert np.array_equal(gs, rs), ("state", s)
            assert np.array_equal(gc, rc), ("count", s)
            assert np.array_equal(ga, ra), ("alive set", s)
    inv = sim.heap.invariants()
    assert inv.hierarchy_violations == 0 and inv.state_violations == 0
    assert inv.active_violations == 0 and inv.type_violations == 0 and inv.empty_allocated == 0
    st = sim.heap.stats()
    assert st.live_objects[sim.heap.cls["Alive"]] == ref.read()[2].size
    return sim


def test_config_256_torus_100_steps_bit_exact(dev):
    print("gol 256x256 x 100", flush=True)
    compare_run(256, 256, gol_init(256, 256), 100)


@pytest.mark.parametrize("W,H", [(37, 23), (8, 8), (1, 1), (3, 70), (64, 1), (100, 65)])
def test_ragged_tori(dev, W, H):
    print("gol %dx%d" % (W, H), flush=True)
    rng = np.random.default_rng(W * 1000 + H)
    compare_run(W, H, (rng.random(W * H) < 0.3).astype(np.uint8), 30)


@pytest.mark.parametrize("concurrent", [False, True])
def test_three_bitmap_levels(dev, concurrent):
    """512 x 512 (12,304 blocks, three bitmap levels): births start their
    active-block search from the prefetched middle level and load the level
    below it; bit-exact with the oracle."""
    print("gol 512x512 three levels, concurrent", concurrent, flush=True)
    sim = compare_run(512, 512, gol_init(512, 512, seed=5), 12, every=4, concurrent=concurrent)
    # more than 64 * 64 blocks: the level above the blocks' containers has
    # more than one container, so the hierarchy has three levels
    assert 64 * 64 < sim.heap.blocks <= 64 ** 3


def test_glider_on_torus(dev):
    g = np.zeros((16, 16), np.uint8)
    for (x, y) in [(1, 0), (2, 1), (0, 2), (1, 2), (2, 2)]:
        g[y, x] = 1
    sim = compare_run(16, 16, g.reshape(-1), 64, every=4)
    st, _, _ = sim.read()
    assert np.array_equal(st.reshape(16, 16), g)


def test_empty_and_full_boards(dev):
    compare_run(20, 20, np.zeros(400, np.uint8), 3)
    compare_run(20, 20, np.ones(400, np.uint8), 3)


@pytest.mark.parametrize("variant", [dict(rotation=0), dict(coalescing=0), dict(lookup_retries=1),
                                     dict(bulk_ordered=0), dict(sparse_packing=2),
                                     dict(sparse_packing=1, grid_waves=8)])
def test_allocator_variants_same_result(dev, variant):
    print("gol variant", variant, flush=True)
    c = smmo.smmo_config_default()
    for k, v in variant.items():
        setattr(c, k, v)
    compare_run(128, 96, gol_init(128, 96, seed=77), 40, cfg=c, every=5)


def test_graph_replays_match_the_oracle(dev):
    """Ten generations captured in one HIP graph (the bench's launch form),
    replayed four times with eager reads between the replays: every replay
    matches the oracle bit for bit (enumerations, births and deaths included)."""
    import torch

    W = H = 96
    init = gol_init(W, H, seed=31)
    sim = GolSim(W, H, init)
    ref = GolWorld(W, H, init)
    sim.step(2)
    ref.step(2)
    sim.heap.sync()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sim.step(10, stream=torch.cuda.current_stream())
    # capture records the launches without running them
    assert np.array_equal(sim.read()[0], ref.read()[0])
    for r in range(4):
        g.replay()
        torch.cuda.synchronize()
        ref.step(10)
        gs, gc, ga = sim.read()
        rs, rc, ra = ref.read()
        assert np.array_equal(gs, rs) and np.array_equal(gc, rc) and np.array_equal(ga, ra), r


@pytest.mark.parametrize("W,H,steps,variant", [(256, 256, 100, {}), (37, 23, 30, {}), (1, 1, 5, {}),
                                               (100, 65, 30, {}), (128, 96, 40, dict(sparse_packing=2)),
                                               (128, 96, 40, dict(sparse_packing=1, grid_waves=8)),
                                               (128, 96, 40, dict(rotation=0))])
def test_death_beside_birth_on_two_streams(dev, W, H, steps, variant):
    """Alive::death on a second stream, running at the same time as
    Cell::birth, with the Alive snapshot taken on that stream while
    Cell::count runs: bit-exact with the oracle after every generation, and
    the heap's block states stay consistent under the concurrent births and
    deaths."""
    print("gol concurrent %dx%d" % (W, H), variant, flush=True)
    c = smmo.smmo_config_default()
    for k, v in variant.items():
        setattr(c, k, v)
    init = gol_init(W, H, seed=W + H) if W * H >= 64 else np.ones(W * H, np.uint8)
    compare_run(W, H, init, steps, cfg=c, every=1 if steps <= 40 else 5, concurrent=True)


def test_two_stream_graph_replays_match_the_oracle(dev):
    """The two-stream generation captured in one HIP graph (fork and join
    through events, so death and birth are concurrent branches), replayed
    four times with eager reads between the replays."""
    import torch

    W = H = 96
    init = gol_init(W, H, seed=32)
    sim = GolSim(W, H, init, concurrent=True)
    ref = GolWorld(W, H, init)
    sim.step(2)
    ref.step(2)
    sim.heap.sync()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sim.step(10, stream=torch.cuda.current_stream())
    assert np.array_equal(sim.read()[0], ref.read()[0])
    for r in range(4):
        g.replay()
        torch.cuda.synchronize()
        ref.step(10)
        gs, gc, ga = sim.read()
        rs, rc, ra = ref.read()
        assert np.array_equal(gs, rs) and np.array_equal(gc, rc) and np.array_equal(ga, ra), r
    inv = sim.heap.invariants()
    assert inv.hierarchy_violations == 0 and inv.state_violations == 0 and inv.empty_allocated == 0


@pytest.mark.parametrize("W,H,steps,variant", [(256, 256, 100, {}), (37, 23, 30, {}), (1, 1, 5, {}),
                                               (100, 65, 30, {}), (128, 96, 40, dict(rotation=0)),
                                               (128, 96, 40, dict(coalescing=0)),
                                               (128, 96, 40, dict(lookup_retries=1)),
                                               (128, 96, 40, dict(sparse_packing=2)),
                                               (128, 96, 40, dict(grid_waves=8)), (512, 512, 12, {})])
def test_fused_generation(dev, W, H, steps, variant):
    """gol.generation: the count with the Alive snapshot, then death and
    birth in one launch (the direct walk's heaps), or the three do-alls
    (512 x 512: 12,304 blocks): bit-exact with the oracle, block states
    consistent."""
    print("gol fused %dx%d" % (W, H), variant, flush=True)
    c = smmo.smmo_config_default()
    for k, v in variant.items():
        setattr(c, k, v)
    init = gol_init(W, H, seed=W * 7 + H) if W * H >= 64 else np.ones(W * H, np.uint8)
    compare_run(W, H, init, steps, cfg=c, every=1 if steps <= 40 else 5, fused=True)


def test_fused_generation_graph_replays(dev):
    """Ten fused generations in one HIP graph, replayed four times with
    eager reads between the replays."""
    import torch

    W = H = 96
    init = gol_init(W, H, seed=33)
    sim = GolSim(W, H, init, fused=True)
    ref = GolWorld(W, H, init)
    sim.step(2)
    ref.step(2)
    sim.heap.sync()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sim.step(10, stream=torch.cuda.current_stream())
    assert np.array_equal(sim.read()[0], ref.read()[0])
    for r in range(4):
        g.replay()
        torch.cuda.synchronize()
        ref.step(10)
        gs, gc, ga = sim.read()
        rs, rc, ra = ref.read()
        assert np.array_equal(gs, rs) and np.array_equal(gc, rc) and np.array_equal(ga, ra), r
    inv = sim.heap.invariants()
    assert inv.hierarchy_violations == 0 and inv.state_violations == 0 and inv.empty_allocated == 0


def test_cell_ids_outside_the_grid_are_a_device_error(dev):
    """A Cell whose id lies outside the W x H grid (a caller's mistake) is
    reported as SMMO_EDEVICE; the kernels do not read past the grid array."""
    import torch

    W = H = 8
    sim = GolSim(W, H, gol_init(W, H, seed=3))
    bad = torch.tensor([W * H + 5], dtype=torch.int32, device=dev)
    sim.heap.new("Cell", 1, cell_id=bad)
    smmo.smmo_parallel_do(sim.heap.h, sim.heap.cls["Cell"], sim.m_count, sim.args)
    with pytest.raises(smmo.SmmoError) as e:
        sim.heap.sync()
    assert e.value.status == smmo.SMMO_EDEVICE
