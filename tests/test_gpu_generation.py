"""GPU parity of "generation" (thesis Ch.7: Game of Life with dying cells,
rule Burst) against the oracle: bit-exact cell states and dying counters
every generation (integer work), one Alive object per live or dying cell."""

import numpy as np
import pytest

from inputs import gol_init
from oracle import generation_steps
from paper_1908_05845_amd import smmo
from paper_1908_05845_amd.sims import GenerationSim

pytestmark = pytest.mark.gpu


def run(W, H, steps, dying, cfg=None, every=1, seed=None, density=0.25):
    init = gol_init(W, H, seed=seed, density=density)
    sim = GenerationSim(W, H, init, dying=dying, cfg=cfg)
    state = init.copy()
    left = np.zeros(W * H, np.int32)
    for g in range(0, steps, every):
        k = min(every, steps - g)
        sim.step(k)
        state, left = generation_steps(W, H, state, left, k, dying=dying)
        s, lf, na = sim.read()
        assert np.array_equal(s, state), (g + k, np.flatnonzero(s != state)[:10])
        assert np.array_equal(lf, left), (g + k, np.flatnonzero(lf != left)[:10])
        assert na == int(np.count_nonzero(state))
    inv = sim.heap.invariants()
    assert inv.hierarchy_violations == 0 and inv.state_violations == 0 and inv.active_violations == 0
    assert inv.type_violations == 0 and inv.empty_allocated == 0
    return sim, state


@pytest.mark.parametrize("W,H,dying", [(64, 64, 4), (37, 23, 2), (1, 1, 3), (3, 70, 5), (100, 65, 1)])
def test_every_generation(dev, W, H, dying):
    print("generation %dx%d dying %d" % (W, H, dying), flush=True)
    run(W, H, 40, dying)


def test_burst_256_torus_past_the_dying_period(dev):
    """The thesis's rule with dying 255 on 96 x 96 for 300 generations: cells
    that died early come free again."""
    print("generation 96x96 burst 300", flush=True)
    sim, state = run(96, 96, 300, 255, every=25, seed=11)
    assert (state == 2).any() and (state == 1).any()


@pytest.mark.parametrize("variant", [dict(rotation=0), dict(coalescing=0), dict(sparse_packing=2),
                                     dict(sparse_packing=1, grid_waves=8), dict(block_group=1),
                                     dict(block_group=4)])
def test_configurations(dev, variant):
    print("generation variant", variant, flush=True)
    c = smmo.smmo_config_default()
    for k, v in variant.items():
        setattr(c, k, v)
    run(80, 48, 30, 3, cfg=c, every=3, seed=5)


def test_rule_masks_validated(dev):
    sim = GenerationSim(8, 8, np.zeros(64, np.uint8))
    for field, value in (("survive", 1 << 9), ("birth", 1 << 10), ("dying", 0)):
        bad = smmo.smmo_generation_args.from_buffer_copy(sim.args)
        setattr(bad, field, value)
        with pytest.raises(smmo.SmmoError):
            smmo.smmo_parallel_do(sim.heap.h, sim.heap.cls["Cell"], sim.m_count, bad)


def test_graph_replays_match_the_oracle(dev):
    """Twelve generations in one HIP graph (the bench's launch form), replayed
    five times with eager reads in between; dying 7 so that cells expire
    within the replays."""
    import torch

    W, H, D = 80, 64, 7
    init = gol_init(W, H, seed=13)
    sim = GenerationSim(W, H, init, dying=D)
    state, left = init.copy(), np.zeros(W * H, np.int32)
    sim.step(2)
    state, left = generation_steps(W, H, state, left, 2, dying=D)
    sim.heap.sync()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        sim.step(12, stream=torch.cuda.current_stream())
    for r in range(5):
        g.replay()
        torch.cuda.synchronize()
        state, left = generation_steps(W, H, state, left, 12, dying=D)
        s, lf, na = sim.read()
        assert np.array_equal(s, state) and np.array_equal(lf, left), r
        assert na == int(np.count_nonzero(state))
