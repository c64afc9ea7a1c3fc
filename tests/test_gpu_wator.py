"""GPU parity of wa-tor (thesis Ch.7 "wa-tor") against the oracle.

Everything in wa-tor is integer work (agent kinds, spawn timers, energies,
random picks from a counter-based generator keyed by iteration, phase and
cell), so the GPU state must equal the oracle's bit for bit, cell by cell,
after every checked iteration.  Fish and sharks are created and deleted
inside the update do-alls through the device allocator; the block-state
invariants must hold at the end, under every allocator configuration.
"""

import numpy as np
import pytest

from inputs import config_seed, wator_init
from oracle import WatorWorld
from paper_1908_05845_amd import smmo
from paper_1908_05845_amd.sims import WatorSim

pytestmark = pytest.mark.gpu


def clean(heap):
    inv = heap.invariants()
    bad = {f: getattr(inv, f) for f in ("hierarchy_violations", "state_violations", "active_violations",
                                        "type_violations", "empty_allocated")}
    assert all(v == 0 for v in bad.values()), bad


def run_pair(W, H, prm, seed, iters, check_every=1, cfg=None, p_fish=0.3, p_shark=0.05):
    init = wator_init(W, H, seed=seed, p_fish=p_fish, p_shark=p_shark, fish_spawn=prm[0],
                      shark_spawn=prm[1], energy0=prm[2])
    ref = WatorWorld(W, H, seed, prm, init)
    sim = WatorSim(W, H, seed, prm, init, cfg=cfg)
    k, tm, en, c = sim.read()
    assert np.array_equal(k, init["kind"]) and np.array_equal(tm, init["timer"])
    done = 0
    events = 0
    last = c
    while done < iters:
        n = min(check_every, iters - done)
        ref.step(n)
        sim.step(n)
        done += n
        kr, tr, er, cr = ref.read()
        kg, tg, eg, cg = sim.read()
        assert cg == cr, (done, cg, cr)
        assert np.array_equal(kg, kr), (done, int(np.sum(kg != kr)))
        assert np.array_equal(tg, tr), done
        assert np.array_equal(eg, er), done
        events += abs(cr[0] - last[0]) + abs(cr[1] - last[1])
        last = cr
    sim.heap.sync()
    clean(sim.heap)
    return sim, events


@pytest.mark.parametrize("W,H,prm", [(16, 16, (2, 5, 4, 3)), (37, 23, (4, 12, 8, 4)), (64, 1, (1, 3, 3, 2)),
                                     (5, 70, (3, 6, 5, 2))])
def test_every_iteration(dev, W, H, prm):
    print("wator %dx%d %s" % (W, H, prm), flush=True)
    sim, events = run_pair(W, H, prm, seed=W * 31 + H, iters=80, p_fish=0.35, p_shark=0.1)
    assert events > 0


@pytest.mark.parametrize("config", ["no_rotation", "no_coalescing", "retries_1", "packed", "packed_short_grid"])
def test_allocator_configurations(dev, config):
    """Allocator variants, and packed do-alls for the agent classes (always,
    and in mode 1 with a grid shorter than the agent lists): the same
    world as the oracle's."""
    print("wator 40x40 %s" % config, flush=True)
    kw = {"no_rotation": {"rotation": 0}, "no_coalescing": {"coalescing": 0},
          "retries_1": {"lookup_retries": 1}, "packed": {"sparse_packing": 2},
          "packed_short_grid": {"sparse_packing": 1, "grid_waves": 6}}[config]
    cfg = smmo.smmo_config_default()
    for k, v in kw.items():
        setattr(cfg, k, v)
    run_pair(40, 40, (3, 8, 5, 3), seed=77, iters=60, cfg=cfg, p_fish=0.35, p_shark=0.1)


def test_256_torus_checked(dev):
    """256 x 256 with the default parameters: allocation waves (fish
    population boom, shark boom, collapse) over 300 iterations, checked every
    10 iterations."""
    print("wator 256x256", flush=True)
    sim, events = run_pair(256, 256, (4, 12, 8, 4), seed=config_seed(7), iters=300, check_every=10)
    st = sim.heap.stats()
    print("  news %d deletes %d fragmentation %.3f" % (st.device_news, st.device_deletes, st.fragmentation),
          flush=True)
    assert st.device_news > 10000 and st.device_deletes > 10000


def test_defragmented_between_iterations(dev):
    """Fish and Shark blocks merged (CompactGpu, n = 1) every 5 iterations:
    Cell::agent handles are rewritten with the shark tag kept, and the state
    stays equal to the oracle's bit for bit."""
    print("wator 48x48 with defragmentation", flush=True)
    W = H = 48
    prm = (3, 8, 5, 3)
    init = wator_init(W, H, seed=5, p_fish=0.35, p_shark=0.1, fish_spawn=prm[0], shark_spawn=prm[1],
                      energy0=prm[2])
    ref = WatorWorld(W, H, 5, prm, init)
    sim = WatorSim(W, H, 5, prm, init)
    moved = 0
    for it in range(60):
        ref.step(1)
        sim.step(1)
        if it % 5 == 4:
            for cls in ("Fish", "Shark"):
                moved += sim.heap.defragment(cls, n=1)[1]
            clean(sim.heap)
        kr, tr, er, cr = ref.read()
        kg, tg, eg, cg = sim.read()
        assert cg == cr and np.array_equal(kg, kr) and np.array_equal(tg, tr) and np.array_equal(eg, er), it
    assert moved > 0
