"""The autotuner on the GPU: tune() times the spring kernels' launch shapes
on a small mesh and keeps one; the mesh then runs under that shape, and
under the corner shapes the tuner may pick (work-groups of 64 and 1,024
threads, 1 and 128 wavefronts per CU, 1, 2 and 4 blocks per wavefront
iteration), with the restart and same-heap parity checks of the spring
tests at every step.  The knobs: work-group size, the wavefronts of the
launch (so the objects a lane serves over the launch: one per block it
walks) and the group (blocks a wavefront holds at once: the objects a lane
has in flight)."""

import pytest

from inputs import spring_mesh
from paper_1908_05845_amd import autotune, smmo
from paper_1908_05845_amd.sims import SpringSim
from test_gpu_spring import run_checked

pytestmark = pytest.mark.gpu


def test_tuned_shapes_keep_parity(dev, tmp_path):
    print("autotune spring 60x40", flush=True)
    mesh = spring_mesh(60, 40, seed=31, v_sigma=1.0)
    dt, limit = 1e-4, 0.3
    sim = SpringSim(mesh, dt, limit)
    frozen = smmo.smmo_spring_args(sim.args.node_class, sim.args.spring_class, 0.0, limit, 0)
    cache = str(tmp_path / "shapes.json")
    picked = {}
    for name, cls, args in (("spring.force", "Spring", sim.args), ("spring.node_update", "Node", frozen)):
        r = autotune.tune(sim.heap, name, cls, args, repeat=5, groups=(1, 2, 4), cache_path=cache)
        assert r["wg"] in autotune.DEFAULT_WG and r["group"] in (1, 2, 4) and r["us"] > 0
        assert r["us"] == min(t["us"] for t in r["tried"])
        picked[name] = (r["wg"], r["waves"], r["group"])
        # the cache gives the same shape back to another heap of the same layout and size bucket
        other = SpringSim(mesh, dt, limit)
        assert autotune.apply_cached(other.heap, name, cls, cache)["wg"] == r["wg"]
    sim.heap.sync()
    broken, gpu_broken, _, _ = run_checked(mesh, dt, limit, 60, shapes=picked)
    assert broken > 0 and gpu_broken > 0


CORNERS = [(64, 1, 1), (64, 128, 4), (1024, 1, 4), (1024, 128, 2), (256, 1, 2)]


@pytest.mark.parametrize("wg,per_cu,group", CORNERS)
def test_corner_shapes_keep_parity(dev, wg, per_cu, group):
    print("spring 60x40 shape wg %d, %d wavefronts per CU, group %d" % (wg, per_cu, group), flush=True)
    mesh = spring_mesh(60, 40, seed=32, v_sigma=1.0)
    import torch

    waves = per_cu * torch.cuda.get_device_properties(0).multi_processor_count
    shapes = {"spring.force": (wg, waves, group), "spring.node_update": (wg, waves, group)}
    broken, gpu_broken, _, _ = run_checked(mesh, 1e-4, 0.3, 40, shapes=shapes)
    assert broken > 0 and gpu_broken > 0
