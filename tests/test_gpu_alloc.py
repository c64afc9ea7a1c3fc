"""GPU tests of the allocator under the Linux Scalability pattern (Ch.8 "Raw
Allocation Performance", in SMMO form): every Worker object allocates n
objects of class Obj with the device allocator, then frees them.  Checked
against the plain live-set model: every handle names a distinct live Obj,
the live count is workers * n after the allocation and zero after the free,
every block returns to the free state, and the block-state invariants hold
under every allocator configuration."""

import numpy as np
import pytest

from paper_1908_05845_amd import smmo

pytestmark = pytest.mark.gpu

CLASSES = {
    "Worker": [("id", "i32", 1)],
    "Obj": [("payload", "u32", 16)],          # 64-byte objects
}


def cfg(**kw):
    c = smmo.smmo_config_default()
    for k, v in kw.items():
        setattr(c, k, v)
    return c


def clean(heap):
    inv = heap.invariants()
    bad = {f: getattr(inv, f) for f in ("hierarchy_violations", "state_violations", "active_violations",
                                        "type_violations", "empty_allocated")}
    assert all(v == 0 for v in bad.values()), bad


def run_ls(dev, workers, n, blocks, config=None):
    import torch

    heap = smmo.Heap(CLASSES, blocks=blocks, cfg=config)
    heap.new("Worker", workers, id=torch.arange(workers, dtype=torch.int32, device=dev))
    handles = torch.full((n * workers,), -1, dtype=torch.int32, device=dev)
    args = smmo.smmo_ls_args(heap.cls["Obj"], n, workers, 0, handles.data_ptr())
    heap.do("Worker", "alloc.ls_alloc", args)
    return heap, handles, args


@pytest.mark.parametrize("workers,n", [(1, 1), (63, 3), (1000, 5), (16384, 2)])
@pytest.mark.parametrize("config", ["default", "no_rotation", "no_coalescing", "retries_1"])
def test_linux_scalability_pattern(dev, workers, n, config):
    print("ls workers %d n %d %s" % (workers, n, config), flush=True)
    kw = {"default": {}, "no_rotation": {"rotation": 0}, "no_coalescing": {"coalescing": 0},
          "retries_1": {"lookup_retries": 1}}[config]
    need = (workers * n + 63) // 64
    blocks = (workers + 63) // 64 + 2 * need + 8
    heap, handles, args = run_ls(dev, workers, n, blocks, cfg(**kw))
    heap.sync()
    h = handles.cpu().numpy().view(np.uint32)
    assert np.all(h != 0xFFFFFFFF)
    assert np.unique(h).size == h.size                       # all distinct
    st = heap.stats()
    obj = heap.cls["Obj"]
    assert st.live_objects[obj] == workers * n
    assert st.device_news >= workers * n
    g = heap.gather("Obj", [])
    assert np.array_equal(np.sort(g["_handle"].cpu().numpy().view(np.uint32)), np.sort(h))
    clean(heap)
    heap.do("Worker", "alloc.ls_free", args)
    heap.sync()
    st = heap.stats()
    assert st.live_objects[obj] == 0 and st.blocks[obj] == 0
    assert st.free_blocks == st.total_blocks - st.blocks[heap.cls["Worker"]]
    clean(heap)


def test_exhaustion_is_reported(dev):
    """A heap too small for workers * n objects: the device error is ENOMEM,
    the handles that were stored are distinct and live, the rest are null,
    and freeing them (after clearing the error) empties the heap."""
    workers, n = 640, 8
    heap, handles, args = run_ls(dev, workers, n, blocks=10 + 40)
    with pytest.raises(smmo.SmmoError) as e:
        heap.sync()
    assert e.value.status == smmo.SMMO_ENOMEM
    smmo.smmo_clear_error(heap.h)
    h = handles.cpu().numpy().view(np.uint32)
    got = h[h != 0xFFFFFFFF]
    assert 0 < got.size <= 40 * 64 and np.unique(got).size == got.size
    assert heap.stats().live_objects[heap.cls["Obj"]] == got.size
    clean(heap)
    heap.do("Worker", "alloc.ls_free", args)
    heap.sync()
    assert heap.stats().live_objects[heap.cls["Obj"]] == 0
    clean(heap)


def test_bad_arguments(dev):
    import torch

    heap = smmo.Heap(CLASSES, blocks=16)
    heap.new("Worker", 10, id=torch.arange(10, dtype=torch.int32, device=dev))
    buf = torch.empty(100, dtype=torch.int32, device=dev)
    for bad in (smmo.smmo_ls_args(heap.cls["Obj"], 0, 10, 0, buf.data_ptr()),
                smmo.smmo_ls_args(heap.cls["Obj"], 10, 10, 0, None),
                smmo.smmo_ls_args(heap.cls["Worker"], 10, 10, 0, buf.data_ptr())):
        with pytest.raises(smmo.SmmoError) as e:
            heap.do("Worker", "alloc.ls_alloc", bad)
        assert e.value.status == smmo.SMMO_EINVAL
    # an id outside [0, workers) is a device error; nothing is allocated for it
    heap.do("Worker", "alloc.ls_alloc", smmo.smmo_ls_args(heap.cls["Obj"], 10, 5, 0, buf.data_ptr()))
    with pytest.raises(smmo.SmmoError) as e:
        heap.sync()
    assert e.value.status == smmo.SMMO_EDEVICE
