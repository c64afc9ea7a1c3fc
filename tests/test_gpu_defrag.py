"""GPU tests of memory defragmentation (CompactGpu, thesis Ch.6).

Defragmentation changes where objects live, never what they hold: the live
set of every class (by key), every field value, and every reference (HANDLE
fields of all classes, external handle arrays, flag bit 31 included) must
name the same objects afterwards.  Fragmentation of the class must fall to
the thesis's bound 1/(n+1) when all candidates are merged, and the
block-state invariants must hold.  Simulations that defragment between steps
must keep their parity with the oracle.
"""

import numpy as np
import pytest

from inputs import spring_mesh
from paper_1908_05845_amd import smmo
from paper_1908_05845_amd.sims import SpringSim

pytestmark = pytest.mark.gpu

CLASSES = {
    "A": [("key", "i32", 1), ("x", "f32", 1), ("tag", "u8", 3), ("ref", "handle", 1)],
    "B": [("key", "i32", 1), ("a", "handle", 2)],
}
NULL = 0xFFFFFFFF


def clean(heap):
    inv = heap.invariants()
    bad = {f: getattr(inv, f) for f in ("hierarchy_violations", "state_violations", "active_violations",
                                        "type_violations", "empty_allocated")}
    assert all(v == 0 for v in bad.values()), bad


def u32(t):
    return t.cpu().numpy().view(np.uint32)


def key_of(heap, cls="A"):
    g = heap.gather(cls, ["key"])
    return dict(zip(u32(g["_handle"]).tolist(), g["key"].cpu().numpy().tolist()))


def frag(heap, cls):
    st = heap.stats()
    c = heap.cls[cls]
    return 1.0 - st.live_objects[c] / (64.0 * st.blocks[c]), st.blocks[c]


@pytest.mark.parametrize("n", [1, 2, 3])
def test_defragment_keeps_objects_and_references(dev, n):
    import torch

    print("defrag n=%d" % n, flush=True)
    rng = np.random.default_rng(n)
    N = 8000
    heap = smmo.Heap(CLASSES, blocks=400)
    keys = np.arange(N, dtype=np.int32)
    hA = heap.new("A", N, key=torch.from_numpy(keys).to(dev), x=torch.from_numpy(keys * 0.5).float().to(dev),
                  tag=torch.from_numpy(np.stack([keys % 251, keys % 13, keys % 7], 1).astype(np.uint8)).to(dev),
                  ref=torch.full((N,), -1, dtype=torch.int32, device=dev))
    hA_np = u32(hA).copy()
    # delete a random 70 %, keep the rest; references only to survivors
    keep = np.sort(rng.choice(N, N * 3 // 10, replace=False))
    dead = np.setdiff1d(np.arange(N), keep)
    heap.destroy("A", hA[torch.from_numpy(dead).to(dev)])
    heap.sync()
    # an external array: each survivor's entry names the next survivor (bit
    # 31 set on odd keys)
    nxt = np.roll(keep, -1)
    ref = hA_np[nxt] | np.where(keep % 2 == 1, 0x80000000, 0).astype(np.uint32)
    assert len(key_of(heap)) == keep.size
    # class B names two survivors per object (some flagged, some null)
    M = 500
    bsel = rng.choice(keep, (M, 2))
    bref = hA_np[bsel].astype(np.uint32)
    bref[::7, 1] = NULL
    bref[::3, 0] |= np.uint32(0x80000000)
    heap.new("B", M, key=torch.arange(M, dtype=torch.int32, device=dev),
             a=torch.from_numpy(bref.reshape(-1).view(np.int32)).to(dev))
    ext = torch.from_numpy(ref.view(np.int32).copy()).to(dev)
    ext_null = torch.full((17,), -1, dtype=torch.int32, device=dev)
    f0, b0 = frag(heap, "A")
    before = heap.gather("A", ["key", "x", "tag"])
    order = np.argsort(before["key"].cpu().numpy())
    passes, moved = heap.defragment("A", n=n, k1=0, max_passes=64, external=[ext, ext_null])
    heap.sync()
    f1, b1 = frag(heap, "A")
    print("  fragmentation %.3f -> %.3f, blocks %d -> %d, passes %d, moved %d" % (f0, f1, b0, b1, passes, moved),
          flush=True)
    assert passes >= 1 and moved > 0 and b1 < b0
    assert f1 <= 1.0 / (n + 1) + 64.0 * (n + 1) / (64.0 * b1)   # up to n candidates may be left over
    clean(heap)
    after = heap.gather("A", ["key", "x", "tag"])
    o2 = np.argsort(after["key"].cpu().numpy())
    for f in ("key", "x", "tag"):
        assert np.array_equal(before[f].cpu().numpy()[order], after[f].cpu().numpy()[o2]), f
    kmap = key_of(heap)
    # external references: same keys, same flag bits
    e = u32(ext)
    assert np.array_equal(np.array([kmap[v & 0x7FFFFFFF] for v in e]), nxt)
    assert np.array_equal(e >> 31, (keep % 2 == 1).astype(np.uint32))
    assert np.all(u32(ext_null) == NULL)
    # B's HANDLE fields
    gb = heap.gather("B", ["key", "a"])
    bk = gb["key"].cpu().numpy()
    ba = u32(gb["a"]).reshape(-1, 2)
    for i, k in enumerate(bk):
        for j in range(2):
            want = bref[k, j]
            if want == NULL:
                assert ba[i, j] == NULL
                continue
            assert kmap[ba[i, j] & 0x7FFFFFFF] == keys[bsel[k, j]]
            assert (ba[i, j] >> 31) == (want >> 31)


def test_defragment_arguments(dev):
    heap = smmo.Heap(CLASSES, blocks=16)
    for bad in (0, 9):
        with pytest.raises(smmo.SmmoError) as e:
            heap.defragment("A", n=bad)
        assert e.value.status == smmo.SMMO_EINVAL
    # nothing to do on an empty class
    assert heap.defragment("A") == (0, 0)


def test_spring_mesh_defragmented_between_steps(dev):
    """Breaking spring mesh with the Spring class defragmented every 10
    steps: every defragmentation leaves the read-back state unchanged bit for
    bit, the defragmented heap steps exactly as a fresh heap loaded with its
    state (same-heap check, every step), and restarts from the oracle's
    trajectory hold as without defragmentation."""
    from oracle import spring_steps
    from spring_parity import mesh_restart, same_heap

    print("spring 40x30 breaking with defragmentation", flush=True)
    mesh = spring_mesh(40, 30, seed=21, v_sigma=1.0)
    dt, limit = 1e-4, 0.3
    make = lambda state: SpringSim(state, dt, limit)
    sim = make(mesh)
    cur = dict(mesh, alive=np.ones(mesh["S"], np.uint8))
    broken = 0
    moved = 0
    for step in range(150):
        if step % 10 == 0:
            mesh_restart(cur, dt, limit, make)
        same_heap(sim, mesh, make)
        cur = spring_steps(cur, dt, limit, 1, alive=cur["alive"])
        broken += cur["nbroken"]
        if step % 10 == 9:
            before = sim.read()
            moved += sim.heap.defragment("Spring", n=1)[1]
            after = sim.read()
            for key in ("alive", "adj", "adj_is_b", "x", "y", "vx", "vy", "fx", "fy"):
                assert np.array_equal(before[key], after[key]), key
            clean(sim.heap)
    gpu_broken = mesh["S"] - int(sim.read()["alive"].sum())
    assert broken > 20 and gpu_broken > 20 and moved > 0, (broken, gpu_broken, moved)
