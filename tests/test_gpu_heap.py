"""GPU tests of the heap itself: creation, gather, do-all, self-deletion,
host destroy, device allocation (coalesced or not, rotated or not), the
iteration snapshot, heap exhaustion, and the block-state invariants after
every operation.  Results are checked against a plain Python model of the
live set (the SMMO semantics), never against the GPU itself."""

import numpy as np
import pytest

from paper_1908_05845_amd import smmo

pytestmark = pytest.mark.gpu

ALL = {
    "A": [("x", "f32", 1), ("key", "i32", 1), ("tag", "u8", 1), ("h", "handle", 1), ("arr", "u32", 3)],
    "B": [("key", "i32", 1), ("x", "f32", 1)],
}


def clean(heap):
    inv = heap.invariants()
    bad = {f: getattr(inv, f) for f in ("hierarchy_violations", "state_violations", "active_violations",
                                        "type_violations", "empty_allocated")}
    assert all(v == 0 for v in bad.values()), bad


def keys_of(heap, cls="A"):
    g = heap.gather(cls, ["key"])
    return np.sort(g["key"].cpu().numpy())


def cfg(**kw):
    c = smmo.smmo_config_default()
    for k, v in kw.items():
        setattr(c, k, v)
    return c


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 1000, 4097])
def test_new_gather_roundtrip(dev, n):
    import torch

    print("roundtrip n=%d" % n, flush=True)
    heap = smmo.Heap(ALL, blocks=200)
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n).astype(np.float32)
    key = np.arange(n, dtype=np.int32)
    tag = rng.integers(0, 256, n).astype(np.uint8)
    hh = rng.integers(0, 2 ** 31, n).astype(np.int64).astype(np.int32)
    arr = rng.integers(0, 2 ** 31, 3 * n).astype(np.int32)
    t = lambda a: torch.from_numpy(a).to(dev)
    hd = heap.new("A", n, x=t(x), key=t(key), tag=t(tag), h=t(hh), arr=t(arr))
    g = heap.gather("A")
    assert g["_count"] == n
    o = np.argsort(g["key"].cpu().numpy())
    assert np.array_equal(g["key"].cpu().numpy()[o], key)
    assert np.array_equal(g["x"].cpu().numpy()[o], x)
    assert np.array_equal(g["tag"].cpu().numpy()[o], tag)
    assert np.array_equal(g["h"].cpu().numpy()[o], hh)
    assert np.array_equal(g["arr"].cpu().numpy()[o].reshape(-1), arr)
    hs = hd.cpu().numpy()
    assert len(set(hs.tolist())) == n
    assert set(hs.tolist()) == set(g["_handle"].cpu().numpy().tolist())
    # handle of object i is the one reported for key i
    assert np.array_equal(g["_handle"].cpu().numpy()[o], hs)
    st = heap.stats()
    assert st.live_objects[0] == n and st.blocks[0] == (n + 63) // 64
    clean(heap)
    heap.close()


def test_axpy_visits_every_live_object_once(dev):
    import torch

    heap = smmo.Heap(ALL, blocks=64)
    n = 1500
    x = torch.arange(n, dtype=torch.float32, device=dev)
    heap.new("A", n, x=x, key=torch.arange(n, dtype=torch.int32, device=dev))
    heap.do("A", "test.axpy", smmo.smmo_axpy_args(2.0, 1.0))
    heap.do("A", "test.axpy", smmo.smmo_axpy_args(1.0, -3.0))
    g = heap.gather("A", ["x", "key"])
    o = np.argsort(g["key"].cpu().numpy())
    assert np.array_equal(g["x"].cpu().numpy()[o], 2.0 * np.arange(n, dtype=np.float32) - 2.0)
    # a class with no objects: the do-all is a no-op
    heap.do("B", "test.axpy", smmo.smmo_axpy_args(2.0, 1.0))
    heap.sync()
    clean(heap)


def test_self_deletion_frees_empty_blocks(dev):
    import torch

    heap = smmo.Heap(ALL, blocks=64)
    n = 2048
    heap.new("A", n, key=torch.arange(n, dtype=torch.int32, device=dev))
    model = np.arange(n)
    for mod, rem in ((3, 1), (5, 0), (2, 0), (7, 3)):
        heap.do("A", "test.destroy_if", smmo.smmo_destroy_if_args(mod, rem))
        model = model[model % mod != rem]
        assert np.array_equal(keys_of(heap), model)
        clean(heap)
    st = heap.stats()
    assert st.live_objects[0] == model.size
    # delete everything: all blocks return to the free state
    heap.do("A", "test.destroy_if", smmo.smmo_destroy_if_args(1, 0))
    st = heap.stats()
    assert st.live_objects[0] == 0 and st.blocks[0] == 0 and st.free_blocks == heap.blocks
    clean(heap)
    heap.do("A", "test.axpy", smmo.smmo_axpy_args(1.0, 1.0))   # stale block list, nothing to visit
    heap.sync()


def test_host_destroy_and_bad_handles(dev):
    import torch

    heap = smmo.Heap(ALL, blocks=64)
    n = 1000
    hd = heap.new("A", n, key=torch.arange(n, dtype=torch.int32, device=dev))
    rng = np.random.default_rng(1)
    pick = rng.choice(n, 600, replace=False)
    heap.destroy("A", hd[torch.from_numpy(pick).to(dev)])
    model = np.setdiff1d(np.arange(n), pick)
    assert np.array_equal(keys_of(heap), model)
    clean(heap)
    # destroying one of them again is an error reported by the next sync
    heap.destroy("A", hd[torch.from_numpy(pick[:1]).to(dev)])
    with pytest.raises(smmo.SmmoError) as e:
        heap.sync()
    assert e.value.status == smmo.SMMO_EDEVICE
    smmo.smmo_clear_error(heap.h)
    heap.sync()
    # one object named twice in one call: released once, reported
    live = np.setdiff1d(model, [])
    dup = hd[torch.from_numpy(np.array([model[0], model[0]])).to(dev)]
    heap.destroy("A", dup)
    with pytest.raises(smmo.SmmoError) as e:
        heap.sync()
    assert e.value.status == smmo.SMMO_EDEVICE
    smmo.smmo_clear_error(heap.h)
    model = live[1:]
    assert np.array_equal(keys_of(heap), model)
    clean(heap)
    # a handle of the wrong class is rejected too
    hb = heap.new("B", 10, key=torch.arange(10, dtype=torch.int32, device=dev))
    heap.destroy("A", hb[:1])
    with pytest.raises(smmo.SmmoError):
        heap.sync()
    smmo.smmo_clear_error(heap.h)
    assert np.array_equal(keys_of(heap), model)
    assert keys_of(heap, "B").size == 10
    clean(heap)


@pytest.mark.parametrize("variant", [
    dict(),
    dict(rotation=0),
    dict(coalescing=0),
    dict(lookup_retries=1, rotation=0),
])
def test_device_allocator_parallel_new(dev, variant):
    import torch

    print("device new", variant, flush=True)
    heap = smmo.Heap(ALL, blocks=2500, cfg=cfg(bulk_ordered=0, **variant))
    n = 100_000
    hd = heap.new("A", n, key=torch.arange(n, dtype=torch.int32, device=dev))
    heap.sync()
    hs = hd.cpu().numpy()
    assert (hs != -1).all() and len(set(hs.tolist())) == n
    assert np.array_equal(keys_of(heap), np.arange(n))
    st = heap.stats()
    assert st.live_objects[0] == n
    assert st.blocks[0] >= (n + 63) // 64
    clean(heap)


def test_spawn_into_own_class_is_not_visited(dev):
    import torch

    heap = smmo.Heap(ALL, blocks=256)
    n = 1000
    heap.new("A", n, key=torch.arange(n, dtype=torch.int32, device=dev))
    # keys 3k spawn two objects with keys 3*key + c, c = 0, 1; key 3*key is
    # again divisible by 3, so a visit of a new object would spawn more
    heap.do("A", "test.spawn", smmo.smmo_spawn_args(heap.cls["A"], 3, 0, 2, 3, 0))
    base = np.arange(n)
    sel = base[base % 3 == 0]
    model = np.sort(np.concatenate([base, 3 * sel, 3 * sel + 1]))
    assert np.array_equal(keys_of(heap), model)
    clean(heap)


@pytest.mark.parametrize("packing", [0, 2])
def test_snapshot_ahead_of_the_do_all(dev, packing):
    """smmo_snapshot takes the iteration snapshot before the do-all: objects
    created in between (by parallel_new, into the holes of the snapshot's
    blocks as well as into new blocks) are not visited; the snapshot serves
    one do-all; a gather or a host destroy in between drops it, and the
    do-all then visits every object alive at its start."""
    import torch

    print("snapshot packing %d" % packing, flush=True)
    heap = smmo.Heap(ALL, blocks=256, cfg=cfg(sparse_packing=packing, bulk_ordered=0))
    n0, n1 = 1000, 700
    ar = lambda a, b: torch.arange(a, b, dtype=torch.int32, device=dev)
    hd = heap.new("A", n0, x=torch.ones(n0, device=dev), key=ar(0, n0))
    gone = np.flatnonzero(np.arange(n0) % 5 == 0)
    heap.destroy("A", hd[torch.from_numpy(gone).to(dev)])
    old = np.setdiff1d(np.arange(n0), gone)
    heap.snapshot("A")
    heap.new("A", n1, x=torch.ones(n1, device=dev), key=ar(n0, n0 + n1))
    heap.do("A", "test.axpy", smmo.smmo_axpy_args(2.0, 0.0))

    def xs():
        g = heap.gather("A", ["x", "key"])
        k = g["key"].cpu().numpy()
        o = np.argsort(k)
        return k[o], g["x"].cpu().numpy()[o]

    keys, x = xs()
    assert np.array_equal(keys, np.concatenate([old, np.arange(n0, n0 + n1)]))
    assert np.array_equal(x, np.where(keys < n0, 2.0, 1.0).astype(np.float32))
    # used up: the next do-all visits every object
    heap.do("A", "test.axpy", smmo.smmo_axpy_args(1.0, 1.0))
    keys, x = xs()
    assert np.array_equal(x, np.where(keys < n0, 3.0, 2.0).astype(np.float32))
    # dropped by a gather, then by a host destroy
    for drop in ("gather", "destroy"):
        heap.snapshot("A")
        if drop == "gather":
            heap.gather("A", ["key"])
        else:
            e = heap.new("A", 1, x=torch.ones(1, device=dev), key=ar(10 ** 6, 10 ** 6 + 1))
            heap.destroy("A", e)
        before = xs()[1]
        heap.new("A", 10, x=torch.zeros(10, device=dev), key=ar(2 * n0 + 10 * len(drop), 2 * n0 + 10 * len(drop) + 10))
        heap.do("A", "test.axpy", smmo.smmo_axpy_args(1.0, 1.0))
        keys, x = xs()
        assert np.array_equal(x, np.concatenate([before + 1.0, np.ones(10, np.float32)])), drop
    clean(heap)


def test_snapshot_of_a_class_family_and_its_drop_by_defragmentation(dev):
    """A snapshot of an abstract base class covers its concrete classes and
    is used by the next do-all on the base (one launch per concrete class);
    a defragmentation of a class in between drops that class's snapshot, so
    the do-all visits every object alive at its start."""
    import torch

    fam = {"Base": {"parent": None, "abstract": True, "fields": [("x", "f32", 1), ("key", "i32", 1)]},
           "C1": {"parent": "Base"}, "C2": {"parent": "Base", "fields": [("y", "f32", 1)]}}
    heap = smmo.Heap(fam, blocks=128, cfg=cfg(bulk_ordered=0))
    ar = lambda a, b: torch.arange(a, b, dtype=torch.int32, device=dev)
    heap.new("C1", 500, x=torch.ones(500, device=dev), key=ar(0, 500))
    heap.new("C2", 300, x=torch.ones(300, device=dev), key=ar(500, 800))
    heap.snapshot("Base")
    heap.new("C1", 100, x=torch.ones(100, device=dev), key=ar(800, 900))
    heap.new("C2", 50, x=torch.ones(50, device=dev), key=ar(900, 950))
    heap.do("Base", "test.axpy", smmo.smmo_axpy_args(2.0, 0.0))

    def xs(c):
        g = heap.gather(c, ["x", "key"])
        k = g["key"].cpu().numpy()
        o = np.argsort(k)
        return k[o], g["x"].cpu().numpy()[o]

    for c in ("C1", "C2"):
        keys, x = xs(c)
        assert np.array_equal(x, np.where(keys < 800, 2.0, 1.0).astype(np.float32)), c
    # C1 loses two thirds of its objects (sparse blocks to compact), then: a
    # snapshot, a defragmentation of C1, new objects of both classes, a
    # do-all on the base: C1's snapshot is gone (all C1 objects visited),
    # C2's holds (its new objects are not)
    g = heap.gather("C1", ["key"])
    h1 = g["_handle"][: int(g["_count"])]
    drop = h1[torch.from_numpy(g["key"].cpu().numpy() % 3 != 0).to(dev)]
    heap.destroy("C1", drop)
    b1, b2 = xs("C1")[1], xs("C2")[1]     # (a gather would drop a snapshot: read first)
    heap.snapshot("Base")
    passes, moved = heap.defragment("C1", n=1)
    assert moved > 0
    heap.new("C1", 10, x=torch.zeros(10, device=dev), key=ar(2000, 2010))
    heap.new("C2", 10, x=torch.zeros(10, device=dev), key=ar(3000, 3010))
    heap.do("Base", "test.axpy", smmo.smmo_axpy_args(1.0, 1.0))
    x1 = xs("C1")[1]
    x2 = xs("C2")[1]
    assert np.array_equal(x1, np.concatenate([b1 + 1.0, np.ones(10, np.float32)]))
    assert np.array_equal(x2, np.concatenate([b2 + 1.0, np.zeros(10, np.float32)]))
    heap.sync()
    clean(heap)


def test_churn_against_live_set_model(dev):
    import torch

    for variant in (dict(), dict(rotation=0, lookup_retries=1), dict(coalescing=0)):
        print("churn", variant, flush=True)
        # headroom: without rotation, concurrent leaders that miss the active
        # bitmap each start a block, so fragmentation can reach one partly
        # filled block per allocating wavefront (Ch.5 sec.5.6.3)
        heap = smmo.Heap(ALL, blocks=2400, cfg=cfg(**variant))
        n = 3000
        heap.new("A", n, key=torch.arange(n, dtype=torch.int32, device=dev))
        model = np.arange(n, dtype=np.int64)
        rng = np.random.default_rng(2)
        for rnd in range(12):
            mod = int(rng.integers(2, 6))
            rem = int(rng.integers(0, mod))
            heap.do("A", "test.destroy_if", smmo.smmo_destroy_if_args(mod, rem))
            model = model[model % mod != rem]
            mod2 = int(rng.integers(2, 5))
            rem2 = int(rng.integers(0, mod2))
            copies = int(rng.integers(1, 3))
            add = int(rng.integers(0, 1000))
            sel = model[model % mod2 == rem2]
            if model.size + copies * sel.size < 20000:    # stay well inside the heap
                heap.do("A", "test.spawn", smmo.smmo_spawn_args(heap.cls["A"], mod2, rem2, copies, 1, add))
                new = [sel + add + c for c in range(copies)]
                model = np.sort(np.concatenate([model] + new))
            st = heap.stats()
            print("  round %d live %d blocks %d F %.3f slow %d retries %d" % (
                rnd, st.live_objects[0], st.blocks[0], st.fragmentation, st.slow_paths,
                st.alloc_retries), flush=True)
            assert np.array_equal(keys_of(heap), model), (variant, rnd)
            clean(heap)
        heap.close()


def test_cross_class_allocation(dev):
    import torch

    heap = smmo.Heap(ALL, blocks=256)
    n = 640
    heap.new("A", n, key=torch.arange(n, dtype=torch.int32, device=dev))
    heap.do("A", "test.spawn", smmo.smmo_spawn_args(heap.cls["B"], 1, 0, 3, 10, 0))
    kb = keys_of(heap, "B")
    assert np.array_equal(kb, np.sort(np.concatenate([10 * np.arange(n) + c for c in range(3)])))
    assert keys_of(heap, "A").size == n
    clean(heap)


def test_bulk_oom_creates_nothing(dev):
    import torch

    heap = smmo.Heap(ALL, blocks=10)
    heap.new("B", 5 * 64, key=torch.arange(320, dtype=torch.int32, device=dev))
    # 6 blocks needed, 5 free: the device finds too few free blocks
    n = 6 * 64
    heap.new("A", n, key=torch.arange(n, dtype=torch.int32, device=dev))
    with pytest.raises(smmo.SmmoError) as e:
        heap.sync()
    assert e.value.status == smmo.SMMO_ENOMEM
    smmo.smmo_clear_error(heap.h)
    assert heap.stats().live_objects[0] == 0
    clean(heap)
    # exactly full is fine
    heap.new("A", 5 * 64, key=torch.arange(320, dtype=torch.int32, device=dev))
    heap.sync()
    assert heap.stats().free_blocks == 0
    clean(heap)
    # the host rejects more objects than slots outright
    with pytest.raises(smmo.SmmoError) as e:
        heap.new("A", 10 * 64 + 1)
    assert e.value.status == smmo.SMMO_ENOMEM


def test_device_oom_is_reported_not_hung(dev):
    import torch

    heap = smmo.Heap(ALL, blocks=20)
    n = 64 * 10
    heap.new("A", n, key=torch.arange(n, dtype=torch.int32, device=dev))
    heap.do("A", "test.spawn", smmo.smmo_spawn_args(heap.cls["B"], 1, 0, 4, 1, 0))
    with pytest.raises(smmo.SmmoError) as e:
        heap.sync()
    assert e.value.status in (smmo.SMMO_ENOMEM, smmo.SMMO_EDEVICE)
    smmo.smmo_clear_error(heap.h)
    st = heap.stats()
    assert st.free_blocks == 0 and 0 < st.live_objects[1] <= 64 * 10
    assert st.live_objects[0] == n
    clean(heap)


def test_gather_capacity_and_bad_method_binding(dev):
    import torch

    heap = smmo.Heap(ALL, blocks=64)
    heap.new("A", 300, key=torch.arange(300, dtype=torch.int32, device=dev))
    g = heap.gather("A", ["key"], capacity=100)
    assert g["_count"] == 300 and g["key"].numel() == 100
    assert len(set(g["key"].cpu().numpy().tolist())) == 100
    # class B has no "key"-less problem but lacks the spring fields
    with pytest.raises(smmo.SmmoError) as e:
        heap.do("B", "spring.force", smmo.smmo_spring_args(0, 1, 1e-3, 0.3))
    assert e.value.status == smmo.SMMO_EINVAL
    with pytest.raises(smmo.SmmoError):
        smmo.smmo_parallel_do(heap.h, heap.cls["A"], smmo.smmo_method_id("test.axpy"),
                              smmo.smmo_spawn_args(0, 1, 0, 1, 1, 0))   # wrong argument struct size


def test_launch_shape_validation(dev):
    """smmo_set_launch and the heap configuration reject shapes outside the
    documented sets; a method without block groups ignores the group knob."""
    import torch

    with pytest.raises(smmo.SmmoError) as e:
        smmo.Heap(ALL, blocks=16, cfg=cfg(block_group=3))
    with pytest.raises(smmo.SmmoError):
        smmo.Heap(ALL, blocks=16, cfg=cfg(sparse_packing=3))
    assert e.value.status == smmo.SMMO_EINVAL
    heap = smmo.Heap(ALL, blocks=64)
    mid = smmo.smmo_method_id("test.axpy")
    a = heap.cls["A"]
    for bad in ((96, 0, 0), (0, 0, 3), (2048, 0, 0)):
        with pytest.raises(smmo.SmmoError) as e:
            smmo.smmo_set_launch(heap.h, mid, a, *bad)
        assert e.value.status == smmo.SMMO_EINVAL
    heap.new("A", 1000, x=torch.ones(1000, device=dev), key=torch.arange(1000, dtype=torch.int32, device=dev))
    smmo.smmo_set_launch(heap.h, mid, a, 64, 3, 4)
    heap.do("A", "test.axpy", smmo.smmo_axpy_args(2.0, 1.0))
    g = heap.gather("A", ["x"])
    assert torch.all(g["x"] == 3.0)
    clean(heap)


@pytest.mark.parametrize("C", [1, 2, 64])
def test_coalescing_probe_touches_every_element_once(dev, C):
    import torch

    data = torch.zeros(64 * 64 * 10, dtype=torch.float32, device=dev)
    smmo.smmo_coalescing_probe(data, C, grid=3)
    torch.cuda.synchronize()
    assert torch.all(data == 8.0)
    with pytest.raises(smmo.SmmoError):
        smmo.smmo_coalescing_probe(data, 3)
    with pytest.raises(smmo.SmmoError):
        smmo.smmo_coalescing_probe(data[:100], 1)


@pytest.mark.parametrize("packing,waves", [(2, 0), (1, 4), (2, 3), (0, 0), (1, 0)])
@pytest.mark.parametrize("keep_frac,seed", [(0.2, 1), (0.5, 2), (0.03, 3), (0.51, 4)])
def test_packed_do_all_on_sparse_blocks(dev, keep_frac, seed, packing, waves):
    """test.axpy and test.destroy_if run packed (a wavefront takes one block
    with more than 32 live objects, or two with at most 32): after random
    deletions every live object is visited exactly once, and self-deletion
    from two blocks per wavefront keeps the live set and the block states
    right.  Packing always on (also with a 3-wavefront grid), on in mode 1
    once the list (38 blocks) is longer than the grid (4 wavefronts, so that
    wavefronts loop), off (the default), and off in mode 1 with a grid as
    long as the list."""
    import torch

    print("packed keep %.2f packing %d waves %d" % (keep_frac, packing, waves), flush=True)
    rng = np.random.default_rng(seed)
    n = 64 * 37 + 11
    heap = smmo.Heap(ALL, blocks=128, cfg=cfg(sparse_packing=packing, grid_waves=waves))
    hd = heap.new("A", n, x=torch.arange(n, dtype=torch.float32, device=dev),
                  key=torch.arange(n, dtype=torch.int32, device=dev))
    # blocks 0 and 1 keep exactly 32 and 33 objects; the rest a random share
    keep = rng.random(n) < keep_frac
    keep[:64] = np.arange(64) < 32
    keep[64:128] = np.arange(64) < 33
    dead = np.flatnonzero(~keep)
    heap.destroy("A", hd[torch.from_numpy(dead).to(dev)])
    model = np.flatnonzero(keep)
    heap.do("A", "test.axpy", smmo.smmo_axpy_args(2.0, 1.0))
    g = heap.gather("A", ["x", "key"])
    o = np.argsort(g["key"].cpu().numpy())
    assert np.array_equal(g["key"].cpu().numpy()[o], model)
    assert np.array_equal(g["x"].cpu().numpy()[o], 2.0 * model.astype(np.float32) + 1.0)
    clean(heap)
    heap.do("A", "test.destroy_if", smmo.smmo_destroy_if_args(3, 1))
    heap.sync()
    model = model[model % 3 != 1]
    assert np.array_equal(keys_of(heap), model)
    clean(heap)


def test_maximum_heap_size(dev):
    """A heap of the largest block count (2^25 - 2 blocks, 2,147,483,520
    slots): an ordered bulk allocation of every slot gives the handles 0 ..
    n-1 (bit 31 stays clear), one more object is out of memory, a do-all over
    all of them and a self-deleting do-all keep counts and invariants, and a
    sampled gather reads the do-all's result."""
    import torch

    M = (1 << 25) - 2
    n = 64 * M
    print("max heap: %d blocks, %d objects" % (M, n), flush=True)
    heap = smmo.Heap({"A": [("x", "f32", 1), ("key", "i32", 1)]}, blocks=M)
    assert heap.blocks == M
    key = torch.arange(n, dtype=torch.int32, device=dev)
    hd = heap.new("A", n, x=key.float(), key=key)
    assert torch.equal(hd, key) and int(hd.max().item()) < (1 << 31)
    del hd
    assert heap.stats().free_blocks == 0
    # no free block left: the device reports the allocation at the next sync
    heap.new("A", 1, key=torch.zeros(1, dtype=torch.int32, device=dev))
    with pytest.raises(smmo.SmmoError) as e:
        heap.sync()
    assert e.value.status == smmo.SMMO_ENOMEM
    smmo.smmo_clear_error(heap.h)
    assert heap.stats().live_objects[heap.cls["A"]] == n
    heap.do("A", "test.axpy", smmo.smmo_axpy_args(2.0, 1.0))
    g = heap.gather("A", ["x", "key"], capacity=1 << 20)
    assert g["_count"] == n
    k = g["key"].double()
    assert torch.equal(g["x"].double(), (2.0 * k.float().double() + 1.0).float().double())
    heap.do("A", "test.destroy_if", smmo.smmo_destroy_if_args(3, 1))
    st = heap.stats()
    want = n - len(range(1, n, 3))
    assert st.live_objects[heap.cls["A"]] == want and st.device_error == 0
    clean(heap)
    heap.close()
    del heap, key, g, k
    torch.cuda.empty_cache()


@pytest.mark.parametrize("variant", [dict(), dict(rotation=0, lookup_retries=1), dict(coalescing=0),
                                     dict(lookup_retries=1)])
def test_blocks_change_class_within_a_launch(dev, variant):
    """test.transmute moves selected objects between two classes in one
    launch (create the replacement, then delete this), so blocks emptied by
    self-deletions are invalidated and taken by the other class's
    allocations while the launch still runs: the enumerated races of a block
    replaced by another type, delete-last against allocate and re-activation.
    The key sets of both classes must follow a model exactly, round after
    round, with clean bitmaps; contention variants included."""
    import torch

    print("transmute", variant, flush=True)
    # a small heap (100 blocks in use of 400) makes the classes take each
    # other's freed blocks; the peak of a full transfer (the new class's
    # blocks before the old ones are freed, plus a partly filled block per
    # allocating wavefront) still fits.  Without rotation that fragmentation
    # is larger, so that variant gets more headroom
    blocks = 800 if variant.get("rotation", 1) == 0 else 400
    heap = smmo.Heap(ALL, blocks=blocks, cfg=cfg(**variant))
    n = 6400
    heap.new("A", n, key=torch.arange(n, dtype=torch.int32, device=dev))
    model = {"A": np.arange(n, dtype=np.int64), "B": np.zeros(0, np.int64)}
    rng = np.random.default_rng(17)
    for rnd in range(16):
        src, dst = ("A", "B") if rnd % 2 == 0 else ("B", "A")
        mod = int(rng.integers(1, 4))
        rem = int(rng.integers(0, mod))
        heap.do(src, "test.transmute", smmo.smmo_spawn_args(heap.cls[dst], mod, rem, 1, 1, 0))
        sel = model[src] % mod == rem
        model[dst] = np.sort(np.concatenate([model[dst], model[src][sel]]))
        model[src] = model[src][~sel]
        for c in ("A", "B"):
            assert np.array_equal(keys_of(heap, c), model[c]), (variant, rnd, c)
        clean(heap)
    st = heap.stats()
    if blocks == 400:
        # more block initializations than blocks that were never used: freed
        # blocks were taken again, by either class
        assert st.slow_paths > blocks - n // 64, st.slow_paths
    with pytest.raises(smmo.SmmoError):
        heap.do("A", "test.transmute", smmo.smmo_spawn_args(heap.cls["A"], 1, 0, 1, 1, 0))
    heap.close()


def test_heap_from_an_allocator_callback(dev):
    """A heap created without a buffer takes it from the allocator set by
    smmo_set_allocator (here torch's caching allocator) and gives it back when
    it is freed; objects created in it round-trip, and a heap in a caller's
    buffer does not touch the allocator."""
    import torch

    ta = smmo.TorchDeviceAllocator()
    smmo.smmo_set_allocator(ta.alloc, ta.release)
    try:
        heap = smmo.Heap({"B": ALL["B"]}, blocks=64, from_allocator=True)
        assert (ta.allocs, ta.releases, len(ta.live)) == (1, 0, 1)
        n = 1000
        heap.new("B", n, key=torch.arange(n, dtype=torch.int32, device=dev),
                 x=torch.arange(n, dtype=torch.float32, device=dev) * 0.5)
        g = heap.gather("B")
        assert g["_count"] == n
        k, x = g["key"].cpu().numpy(), g["x"].cpu().numpy()
        order = np.argsort(k)
        assert np.array_equal(k[order], np.arange(n)) and np.array_equal(x[order], np.arange(n) * 0.5)
        clean(heap)
        heap.close()
        assert (ta.allocs, ta.releases, len(ta.live)) == (1, 1, 0)
        other = smmo.Heap({"B": ALL["B"]}, blocks=8)
        other.close()
        assert (ta.allocs, ta.releases) == (1, 1)
    finally:
        smmo.smmo_set_allocator(None)
