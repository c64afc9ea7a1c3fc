"""C-ABI checks that need no GPU: the library loads, exports every function
that include/*.h declares, and validates schema arguments on the host."""

import ctypes as C
import os
import re

import pytest

from paper_1908_05845_amd import smmo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:smmo_status|void|const char)\s+\**\s*(smmo_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(smmo.LIB_PATH):
        from paper_1908_05845_amd import build

        build.build()
    return smmo.load_library()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    assert names == set(smmo.EXPORTS)
    for n in names:
        assert getattr(lib, n) is not None, n


def test_config_defaults(lib):
    cfg = smmo.smmo_config_default()
    assert cfg.lookup_retries == 5 and cfg.rotation == 1 and cfg.coalescing == 1
    assert cfg.bulk_ordered == 1 and cfg.spin_limit >= 1024
    assert cfg.grid_waves == 0 and cfg.block_group == 0 and cfg.sparse_packing == 0


def test_schema_and_layout(lib):
    s = smmo.smmo_schema_create()
    node = smmo.smmo_define_class(s, "Node", [("x", "f32", 1), ("adj", "handle", 8), ("tag", "u8", 1)])
    spr = smmo.smmo_define_class(s, "Spring", [("a", "handle", 1), ("k", "f32", 1)])
    assert (node, spr) == (0, 1)
    assert smmo.smmo_field_id(s, node, "adj") == 1
    # Node: x 256 B, adj 8 x 256 B, tag 64 B -> 2368 -> rounded to 2560
    assert smmo.smmo_block_bytes(s) == 2560
    b1 = smmo.smmo_heap_bytes(s, 1000)
    b2 = smmo.smmo_heap_bytes(s, 2000)
    assert b2 - b1 >= 1000 * 2560
    smmo.smmo_schema_free(s)


def test_subclass_schema(lib):
    """Single inheritance: a subclass's field list is its parent's (same ids)
    followed by its own; is_a follows the parent chain; bad parents, flags,
    redefined inherited fields are refused."""
    s = smmo.smmo_schema_create()
    base = smmo.smmo_define_subclass(s, "NodeBase", smmo.SMMO_NO_PARENT,
                                     [("x", "f32", 1), ("springs", "handle", 3), ("n", "i32", 1)], abstract=True)
    anchor = smmo.smmo_define_subclass(s, "AnchorNode", base)
    node = smmo.smmo_define_subclass(s, "Node", base, [("vx", "f32", 1)])
    leaf = smmo.smmo_define_subclass(s, "HeavyNode", node, [("m", "f32", 1)])
    other = smmo.smmo_define_class(s, "Spring", [("a", "handle", 1)])
    assert (base, anchor, node, leaf, other) == (0, 1, 2, 3, 4)
    assert smmo.smmo_field_id(s, anchor, "springs") == 1 and smmo.smmo_field_id(s, node, "vx") == 3
    assert smmo.smmo_field_id(s, leaf, "n") == 2 and smmo.smmo_field_id(s, leaf, "m") == 4
    # largest class: HeavyNode = x, 3 springs, n, vx, m = 7 arrays of 256 B
    assert smmo.smmo_block_bytes(s) == 7 * 256
    isa = lambda c, a: smmo.smmo_class_is_a(s, c, a)
    assert isa(leaf, node) and isa(leaf, base) and isa(anchor, base) and isa(base, base)
    assert not isa(node, leaf) and not isa(anchor, node) and not isa(other, base) and not isa(base, anchor)
    with pytest.raises(smmo.SmmoError):
        smmo.smmo_define_subclass(s, "Bad", 17)
    with pytest.raises(smmo.SmmoError) as e:
        smmo.smmo_define_subclass(s, "Dup", node, [("x", "f32", 1)])
    assert "duplicate field" in str(e.value)
    with pytest.raises(smmo.SmmoError):
        smmo.smmo_define_subclass(s, "Empty", smmo.SMMO_NO_PARENT, [])
    lib_ = smmo.load_library()
    cid = smmo.C.c_uint32()
    assert lib_.smmo_define_subclass(s, b"Flags", base, 2, None, 0, smmo.C.byref(cid)) == smmo.SMMO_EINVAL
    smmo.smmo_schema_free(s)


@pytest.mark.parametrize("fields,msg", [
    ([], "bad field count"),
    ([("x", "f32", 0)], "count 0"),
    ([("x", 99, 1)], "bad dtype"),
    ([("x", "f32", 1), ("x", "i32", 1)], "duplicate field"),
    ([("", "f32", 1)], "1..31"),
    ([("arr", "f32", 33)], "too many field arrays"),
])
def test_define_class_rejects_bad_fields(lib, fields, msg):
    s = smmo.smmo_schema_create()
    with pytest.raises(smmo.SmmoError) as e:
        smmo.smmo_define_class(s, "C", fields)
    assert e.value.status == smmo.SMMO_EINVAL and msg in str(e.value)
    smmo.smmo_schema_free(s)


def test_too_many_classes_and_duplicates(lib):
    s = smmo.smmo_schema_create()
    for i in range(16):
        smmo.smmo_define_class(s, "C%d" % i, [("x", "f32", 1)])
    with pytest.raises(smmo.SmmoError) as e:
        smmo.smmo_define_class(s, "C16", [("x", "f32", 1)])
    assert e.value.status == smmo.SMMO_ENOMEM
    s2 = smmo.smmo_schema_create()
    smmo.smmo_define_class(s2, "A", [("x", "f32", 1)])
    with pytest.raises(smmo.SmmoError):
        smmo.smmo_define_class(s2, "A", [("y", "f32", 1)])
    smmo.smmo_schema_free(s)
    smmo.smmo_schema_free(s2)


def test_method_ids(lib):
    names = ["gol.cell_count", "gol.alive_death", "gol.cell_birth", "nbody.force", "nbody.update",
             "spring.force", "spring.node_update", "spring.link", "adjoint.record", "adjoint.save",
             "adjoint.load", "adjoint.seed", "adjoint.zero", "adjoint.node", "adjoint.spring", "adjoint.step_node", "test.axpy",
             "test.destroy_if", "test.spawn", "test.transmute", "alloc.ls_alloc", "alloc.ls_free", "wator.cell_prepare",
             "wator.fish_prepare", "wator.shark_prepare", "wator.cell_decide", "wator.fish_update",
             "wator.shark_update", "wator.cell_link", "wator.link", "spring_pi.force", "spring_pi.node_update",
             "spring_pi.link", "generation.cell_count",
             "generation.cell_birth", "generation.alive_update", "structure.pull", "structure.force",
             "structure.node_update", "structure.bfs_init", "structure.bfs_visit", "structure.bfs_mark",
             "structure.bfs_delete", "structure.link", "gol.generation"]
    ids = [smmo.smmo_method_id(n) for n in names]
    assert len(set(ids)) == len(ids)
    with pytest.raises(smmo.SmmoError) as e:
        smmo.smmo_method_id("no.such")
    assert "unknown method" in str(e.value)


def test_null_and_state_errors(lib):
    assert lib.smmo_define_class(None, b"x", None, 0, None) == smmo.SMMO_EINVAL
    assert lib.smmo_sync(None) == smmo.SMMO_EINVAL
    assert lib.smmo_parallel_do(None, 0, 0, None, 0, None) == smmo.SMMO_EINVAL
    assert lib.smmo_snapshot(None, 0, None) == smmo.SMMO_EINVAL
    s = smmo.smmo_schema_create()
    out = C.c_uint64()
    assert lib.smmo_heap_bytes(s, 10, C.byref(out)) == smmo.SMMO_ESTATE   # no classes yet
    buf = C.create_string_buffer(128)
    lib.smmo_last_error(buf, 128)
    assert b"no classes" in buf.value
    smmo.smmo_schema_free(s)


def test_struct_sizes_match_header(lib):
    # sizes of the argument structs the methods check against
    assert C.sizeof(smmo.smmo_gol_args) == 24
    assert C.sizeof(smmo.smmo_nbody_args) == 16
    assert C.sizeof(smmo.smmo_spring_args) == 20
    assert C.sizeof(smmo.smmo_spawn_args) == 24
    assert C.sizeof(smmo.smmo_ls_args) == 24
    assert C.sizeof(smmo.smmo_wator_args) == 64
    assert C.sizeof(smmo.smmo_structure_args) == 32
    assert C.sizeof(smmo.smmo_generation_args) == 40
    assert C.sizeof(smmo.smmo_spring_pi_args) == 32
    assert C.sizeof(smmo.smmo_config) == 64
    assert C.sizeof(smmo.smmo_adjoint_args) == 80


def test_library_refuses_other_sources(lib, tmp_path, monkeypatch):
    """The library carries the hash of the sources it was built from; the
    binding compares it with the sources beside it."""
    from paper_1908_05845_amd import build

    assert lib.smmo_source_hash().decode() == build.source_hash()
    # a changed source changes the hash the binding expects
    h0 = build.source_hash()
    monkeypatch.setattr(build, "CSRC", str(tmp_path))
    assert build.source_hash() != h0


def test_allocator_callback_checks(lib):
    """smmo_alloc_heap without a buffer: refused with no allocator set, and an
    allocator's failures and the heap set-up's failures are handled on the
    host (no GPU needed: the set-up fails before any device call)."""
    s = smmo.smmo_schema_create()
    smmo.smmo_define_class(s, "A", [("x", "f32", 1)])
    out = C.c_void_p()

    def alloc_heap(nbytes):   # the call itself, on the null stream (torch's needs a GPU)
        return lib.smmo_alloc_heap(s, None, nbytes, None, None, C.byref(out))

    keep = smmo.ALLOC_FN(lambda n, c: None)
    no_release = smmo.smmo_allocator(keep, smmo.RELEASE_FN(), None)   # NULL release
    assert lib.smmo_set_allocator(C.byref(no_release)) == smmo.SMMO_EINVAL
    smmo.smmo_set_allocator(None)
    assert alloc_heap(1 << 20) == smmo.SMMO_EINVAL and "allocator" in smmo.smmo_last_error()
    calls = []
    # an allocator that has no memory: ENOMEM, and nothing to release
    smmo.smmo_set_allocator(lambda n: calls.append(("alloc", n)) or 0, lambda p, n: calls.append(("release", p, n)))
    assert alloc_heap(1 << 20) == smmo.SMMO_ENOMEM and calls == [("alloc", 1 << 20)]
    # memory the heap cannot use (misaligned): the set-up fails and the
    # allocation goes back to the allocator
    calls.clear()
    smmo.smmo_set_allocator(lambda n: calls.append(("alloc", n)) or 0x1000010,
                            lambda p, n: calls.append(("release", p, n)))
    assert alloc_heap(4096) == smmo.SMMO_EINVAL
    assert calls == [("alloc", 4096), ("release", 0x1000010, 4096)]
    smmo.smmo_set_allocator(None)
    smmo.smmo_schema_free(s)
