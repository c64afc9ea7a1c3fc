"""Python binding of libsmmo (C ABI in include/smmo.h and include/smmo_methods.h).

The functions keep the C names and only marshal arguments; every step of the
SMMO path runs in the HIP library.  PyTorch supplies device memory (the heap
buffer and the dense arrays handed to parallel_new / gather_soa) and the
stream (``torch.cuda.current_stream().cuda_stream``).  Importing this module
needs no GPU; ``load_library()`` raises if libsmmo.so has not been built.
"""

import ctypes as C
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmmo.so")

SMMO_OK = 0
SMMO_EINVAL = -1
SMMO_ENOMEM = -2
SMMO_ESTATE = -3
SMMO_EHIP = -4
SMMO_EDEVICE = -5
SMMO_EUNSUPPORTED = -6
SMMO_NULL = 0xFFFFFFFF

U8, I32, U32, F32, HANDLE = 1, 2, 3, 4, 5
DTYPE_NAMES = {"u8": U8, "i32": I32, "u32": U32, "f32": F32, "handle": HANDLE}
_STATUS_NAMES = {0: "SMMO_OK", -1: "SMMO_EINVAL", -2: "SMMO_ENOMEM", -3: "SMMO_ESTATE",
                 -4: "SMMO_EHIP", -5: "SMMO_EDEVICE", -6: "SMMO_EUNSUPPORTED"}

MAX_CLASSES = 16
MAX_FIELDS = 32


class SmmoError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (_STATUS_NAMES.get(status, status), message))
        self.status = status


class smmo_field_desc(C.Structure):
    _fields_ = [("name", C.c_char_p), ("dtype", C.c_int32), ("count", C.c_uint32)]


class smmo_config(C.Structure):
    _fields_ = [("lookup_retries", C.c_uint32), ("rotation", C.c_uint32), ("coalescing", C.c_uint32),
                ("bulk_ordered", C.c_uint32), ("spin_limit", C.c_uint32), ("grid_waves", C.c_uint32),
                ("block_group", C.c_uint32), ("sparse_packing", C.c_uint32), ("streaming_loads", C.c_uint32),
                ("reserved", C.c_uint32 * 7)]


class smmo_stats(C.Structure):
    _fields_ = [("live_objects", C.c_uint64 * MAX_CLASSES), ("blocks", C.c_uint64 * MAX_CLASSES),
                ("free_blocks", C.c_uint64), ("total_blocks", C.c_uint64),
                ("fragmentation", C.c_double), ("device_error", C.c_int32),
                ("block_bytes", C.c_uint32), ("slow_paths", C.c_uint64), ("alloc_retries", C.c_uint64),
                ("device_news", C.c_uint64), ("device_deletes", C.c_uint64),
                ("bitmap_spins", C.c_uint64), ("lookups", C.c_uint64)]


class smmo_invariants(C.Structure):
    _fields_ = [("hierarchy_violations", C.c_uint64), ("state_violations", C.c_uint64),
                ("active_violations", C.c_uint64), ("type_violations", C.c_uint64),
                ("empty_allocated", C.c_uint64)]


class smmo_field_init(C.Structure):
    _fields_ = [("field_id", C.c_uint32), ("values", C.c_void_p)]


# ---- method argument structs (include/smmo_methods.h) ----------------------
class smmo_gol_args(C.Structure):
    _fields_ = [("cell_class", C.c_uint32), ("alive_class", C.c_uint32), ("cells", C.c_void_p),
                ("width", C.c_int32), ("height", C.c_int32)]


class smmo_nbody_args(C.Structure):
    _fields_ = [("G", C.c_float), ("eps", C.c_float), ("dt", C.c_float), ("reserved", C.c_uint32)]


SMMO_SPRING_TENSION_ONLY = 1


class smmo_spring_args(C.Structure):
    _fields_ = [("node_class", C.c_uint32), ("spring_class", C.c_uint32), ("dt", C.c_float),
                ("strain_limit", C.c_float), ("flags", C.c_uint32)]


class smmo_adjoint_args(C.Structure):
    _fields_ = [("node_class", C.c_uint32), ("spring_class", C.c_uint32), ("dt", C.c_float),
                ("mode", C.c_uint32), ("tape", C.c_void_p), ("tape_floats", C.c_uint64),
                ("plane", C.c_uint64), ("slot", C.c_uint32), ("seed_count", C.c_uint32),
                ("seed_x", C.c_void_p), ("seed_y", C.c_void_p), ("seed_vx", C.c_void_p),
                ("seed_vy", C.c_void_p)]


class smmo_handle_array(C.Structure):
    _fields_ = [("handles", C.c_void_p), ("count", C.c_uint64)]


class smmo_ls_args(C.Structure):
    _fields_ = [("target_class", C.c_uint32), ("n", C.c_uint32), ("workers", C.c_uint32),
                ("reserved", C.c_uint32), ("handles", C.c_void_p)]


class smmo_wator_args(C.Structure):
    _fields_ = [("cell_class", C.c_uint32), ("fish_class", C.c_uint32), ("shark_class", C.c_uint32),
                ("iteration", C.c_uint32), ("seed", C.c_uint64), ("fish_spawn", C.c_int32),
                ("shark_spawn", C.c_int32), ("energy0", C.c_int32), ("boost", C.c_int32),
                ("kind", C.c_uint32), ("width", C.c_int32), ("height", C.c_int32),
                ("reserved", C.c_uint32), ("cells", C.c_void_p)]


class smmo_spring_pi_args(C.Structure):
    _fields_ = [("node_class", C.c_uint32), ("spring_class", C.c_uint32), ("dt", C.c_float),
                ("strain_limit", C.c_float), ("overflow", C.c_void_p), ("overflow_len", C.c_uint64)]


class smmo_generation_args(C.Structure):
    _fields_ = [("cell_class", C.c_uint32), ("alive_class", C.c_uint32), ("width", C.c_int32),
                ("height", C.c_int32), ("survive", C.c_uint32), ("birth", C.c_uint32), ("dying", C.c_int32),
                ("reserved", C.c_uint32), ("cells", C.c_void_p)]


SMMO_STRUCTURE_FAR = 0x7FFFFFFF
SMMO_BFS_DEVICE_VISITED = 1
SMMO_BFS_SMALL_FRONTIER = 2


class smmo_structure_args(C.Structure):
    _fields_ = [("nodebase_class", C.c_uint32), ("anchor_class", C.c_uint32), ("spring_class", C.c_uint32),
                ("distance", C.c_int32), ("dt", C.c_float), ("bfs_options", C.c_uint32),
                ("flag", C.c_void_p)]


class smmo_axpy_args(C.Structure):
    _fields_ = [("a", C.c_float), ("b", C.c_float)]


class smmo_destroy_if_args(C.Structure):
    _fields_ = [("mod", C.c_int32), ("rem", C.c_int32)]


class smmo_spawn_args(C.Structure):
    _fields_ = [("target_class", C.c_uint32), ("mod", C.c_int32), ("rem", C.c_int32),
                ("copies", C.c_uint32), ("key_mul", C.c_int32), ("key_add", C.c_int32)]


_lock = threading.Lock()
_lib = None

#: every symbol include/smmo.h declares
EXPORTS = [
    "smmo_config_default", "smmo_schema_create", "smmo_schema_free", "smmo_define_class",
    "smmo_define_subclass", "smmo_class_is_a",
    "smmo_field_id", "smmo_block_bytes", "smmo_heap_bytes", "smmo_set_allocator", "smmo_alloc_heap",
    "smmo_heap_free",
    "smmo_parallel_new", "smmo_parallel_do", "smmo_snapshot", "smmo_destroy", "smmo_gather_soa", "smmo_sync",
    "smmo_heap_stats", "smmo_check_invariants", "smmo_clear_error", "smmo_heap_info",
    "smmo_method_id", "smmo_last_error", "smmo_set_launch", "smmo_defragment", "smmo_coalescing_probe",
    "smmo_source_hash", "smmo_structure_remove_disconnected", "smmo_structure_remove_disconnected_noalloc",
]


def load_library(path: str = LIB_PATH):
    """Loads libsmmo.so; raises if it has not been built (no fallback)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise RuntimeError("libsmmo.so not found at %s: build it with "
                               "`python -m paper_1908_05845_amd.build`" % path)
        lib = C.CDLL(path)
        lib.smmo_source_hash.restype = C.c_char_p
        lib.smmo_source_hash.argtypes = []
        from . import build as _build

        built, here = lib.smmo_source_hash().decode(), _build.source_hash()
        if built != here:
            raise RuntimeError("libsmmo.so at %s was built from other sources (%s) than those beside it "
                               "(%s): rebuild it with `python -m paper_1908_05845_amd.build`"
                               % (path, built, here))
        P, S, U32, U64 = C.c_void_p, C.c_int32, C.c_uint32, C.c_uint64
        sig = {
            "smmo_config_default": (None, [P]),
            "smmo_schema_create": (S, [P]),
            "smmo_schema_free": (S, [P]),
            "smmo_define_class": (S, [P, C.c_char_p, P, U32, P]),
            "smmo_define_subclass": (S, [P, C.c_char_p, U32, U32, P, U32, P]),
            "smmo_class_is_a": (S, [P, U32, U32, P]),
            "smmo_field_id": (S, [P, U32, C.c_char_p, P]),
            "smmo_block_bytes": (S, [P, P]),
            "smmo_heap_bytes": (S, [P, U64, P]),
            "smmo_set_allocator": (S, [P]),
            "smmo_alloc_heap": (S, [P, P, C.c_size_t, P, P, P]),
            "smmo_heap_free": (S, [P]),
            "smmo_parallel_new": (S, [P, U32, U32, P, U32, P, P]),
            "smmo_parallel_do": (S, [P, U32, U32, P, C.c_size_t, P]),
            "smmo_snapshot": (S, [P, U32, P]),
            "smmo_destroy": (S, [P, U32, P, U32, P]),
            "smmo_gather_soa": (S, [P, U32, P, U32, P, P, U32, P, P]),
            "smmo_sync": (S, [P]),
            "smmo_heap_stats": (S, [P, P]),
            "smmo_check_invariants": (S, [P, P]),
            "smmo_clear_error": (S, [P, P]),
            "smmo_heap_info": (S, [P, P, P]),
            "smmo_method_id": (S, [C.c_char_p, P]),
            "smmo_set_launch": (S, [P, U32, U32, U32, U32, U32]),
            "smmo_defragment": (S, [P, U32, U32, U32, U32, P, U32, P, P, P]),
            "smmo_coalescing_probe": (S, [P, U64, U32, U32, P]),
            "smmo_structure_remove_disconnected": (S, [P, P, P, U64, P, P]),
            "smmo_structure_remove_disconnected_noalloc": (S, [P, P, P, P]),
            "smmo_last_error": (S, [C.c_char_p, C.c_size_t]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
        return lib


def _last_error(lib) -> str:
    buf = C.create_string_buffer(512)
    lib.smmo_last_error(buf, 512)
    return buf.value.decode(errors="replace")


def _check(lib, status: int) -> None:
    if status != SMMO_OK:
        raise SmmoError(status, _last_error(lib))


def _ptr(x):
    """Device or host address of a torch tensor / int / None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _stream(stream):
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ---- thin wrappers with the C names ----------------------------------------
def smmo_config_default() -> smmo_config:
    cfg = smmo_config()
    load_library().smmo_config_default(C.byref(cfg))
    return cfg


def smmo_schema_create():
    lib = load_library()
    out = C.c_void_p()
    _check(lib, lib.smmo_schema_create(C.byref(out)))
    return out


def smmo_schema_free(schema) -> None:
    lib = load_library()
    _check(lib, lib.smmo_schema_free(schema))


def smmo_define_class(schema, name: str, fields) -> int:
    """fields: sequence of (name, dtype, count); dtype an int or 'u8'/'i32'/'u32'/'f32'/'handle'."""
    lib = load_library()
    arr = (smmo_field_desc * max(1, len(fields)))()
    keep = []
    for i, (fname, dt, cnt) in enumerate(fields):
        b = fname.encode()
        keep.append(b)
        arr[i] = smmo_field_desc(b, DTYPE_NAMES.get(dt, dt) if isinstance(dt, str) else dt, cnt)
    cid = C.c_uint32()
    _check(lib, lib.smmo_define_class(schema, name.encode(), arr, len(fields), C.byref(cid)))
    return cid.value


SMMO_NO_PARENT = 0xFFFFFFFF
SMMO_CLASS_ABSTRACT = 1


def smmo_define_subclass(schema, name: str, parent: int, fields=(), abstract: bool = False) -> int:
    """A class deriving from `parent` (SMMO_NO_PARENT for a root): the
    parent's fields, then `fields` (sequence of (name, dtype, count))."""
    lib = load_library()
    arr = (smmo_field_desc * max(1, len(fields)))()
    keep = []
    for i, (fname, dt, cnt) in enumerate(fields):
        b = fname.encode()
        keep.append(b)
        arr[i] = smmo_field_desc(b, DTYPE_NAMES.get(dt, dt) if isinstance(dt, str) else dt, cnt)
    cid = C.c_uint32()
    _check(lib, lib.smmo_define_subclass(schema, name.encode(), parent, SMMO_CLASS_ABSTRACT if abstract else 0,
                                         arr if fields else None, len(fields), C.byref(cid)))
    return cid.value


def smmo_class_is_a(schema, cls: int, ancestor: int) -> bool:
    lib = load_library()
    out = C.c_uint32()
    _check(lib, lib.smmo_class_is_a(schema, cls, ancestor, C.byref(out)))
    return bool(out.value)


def smmo_field_id(schema, class_id: int, name: str) -> int:
    lib = load_library()
    out = C.c_uint32()
    _check(lib, lib.smmo_field_id(schema, class_id, name.encode(), C.byref(out)))
    return out.value


def smmo_block_bytes(schema) -> int:
    lib = load_library()
    out = C.c_uint32()
    _check(lib, lib.smmo_block_bytes(schema, C.byref(out)))
    return out.value


def smmo_heap_bytes(schema, blocks: int) -> int:
    lib = load_library()
    out = C.c_uint64()
    _check(lib, lib.smmo_heap_bytes(schema, blocks, C.byref(out)))
    return out.value


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)


class smmo_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("release", RELEASE_FN), ("ctx", C.c_void_p)]


# every allocator ever set: a heap keeps the function pointers it was created
# with until it is freed, so their ctypes thunks must never be collected
_allocators = []


def smmo_set_allocator(alloc=None, release=None) -> None:
    """Sets the allocator for heaps created without a buffer: alloc(nbytes)
    returns a 256-byte aligned device address (int) or 0, release(address,
    nbytes) gives it back.  alloc=None unsets it."""
    lib = load_library()
    if alloc is None:
        _check(lib, lib.smmo_set_allocator(None))
        return
    a = smmo_allocator(ALLOC_FN(lambda n, ctx: alloc(n) or None), RELEASE_FN(lambda ptr, n, ctx: release(ptr, n)),
                       None)
    _allocators.append(a)
    _check(lib, lib.smmo_set_allocator(C.byref(a)))


class TorchDeviceAllocator:
    """Device memory from torch's caching allocator on the current device, as
    a heap allocator (smmo_set_allocator(a.alloc, a.release)); counts calls."""

    def __init__(self):
        self.live = {}
        self.allocs = 0
        self.releases = 0

    def alloc(self, nbytes: int) -> int:
        import torch

        t = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        p = (t.data_ptr() + 255) & ~255
        self.live[p] = t
        self.allocs += 1
        return p

    def release(self, ptr: int, nbytes: int) -> None:
        self.live.pop(ptr, None)
        self.releases += 1


def smmo_alloc_heap(schema, dev_buf, nbytes: int, cfg=None, stream=None):
    lib = load_library()
    out = C.c_void_p()
    _check(lib, lib.smmo_alloc_heap(schema, _ptr(dev_buf), nbytes, None if cfg is None else C.byref(cfg),
                                    _stream(stream), C.byref(out)))
    return out


def smmo_heap_free(heap) -> None:
    lib = load_library()
    _check(lib, lib.smmo_heap_free(heap))


def smmo_parallel_new(heap, class_id: int, n: int, inits=(), out_handles=None, stream=None) -> None:
    """inits: sequence of (field_id, device tensor or address)."""
    lib = load_library()
    arr = (smmo_field_init * max(1, len(inits)))()
    for i, (fid, vals) in enumerate(inits):
        arr[i] = smmo_field_init(fid, _ptr(vals))
    _check(lib, lib.smmo_parallel_new(heap, class_id, n, arr if inits else None, len(inits),
                                      _ptr(out_handles), _stream(stream)))


def smmo_parallel_do(heap, class_id: int, method_id: int, args=None, stream=None) -> None:
    lib = load_library()
    _check(lib, lib.smmo_parallel_do(heap, class_id, method_id,
                                     None if args is None else C.byref(args),
                                     0 if args is None else C.sizeof(args), _stream(stream)))


def smmo_snapshot(heap, class_id: int, stream=None) -> None:
    """Takes the iteration snapshot of a class for its next parallel_do."""
    lib = load_library()
    _check(lib, lib.smmo_snapshot(heap, class_id, _stream(stream)))


class BoundLaunch:
    """One do-all with its heap, class, method and argument struct fixed, for
    drivers that issue many launches: a call is one foreign call of
    smmo_parallel_do on the given stream (the struct is kept alive here and
    passed by reference), and a nonzero status raises SmmoError."""

    __slots__ = ("lib", "fn", "h", "cls", "mid", "args", "ref", "size")

    def __init__(self, heap, class_id: int, method_id: int, args):
        self.lib = load_library()
        self.fn = self.lib.smmo_parallel_do
        self.h, self.cls, self.mid, self.args = heap, class_id, method_id, args
        self.ref = C.byref(args)
        self.size = C.sizeof(args)

    def __call__(self, stream) -> None:
        st = self.fn(self.h, self.cls, self.mid, self.ref, self.size, stream)
        if st:
            raise SmmoError(st, _last_error(self.lib))


def smmo_defragment(heap, class_id: int, n: int = 1, k1: int = 0, max_passes: int = 32, external=(),
                    stream=None):
    """Defragments class_id (see smmo.h); external = device tensors of handles
    to rewrite as well.  Returns (passes, moved objects)."""
    lib = load_library()
    arr = (smmo_handle_array * max(1, len(external)))()
    for i, t in enumerate(external):
        arr[i].handles = _ptr(t)
        arr[i].count = t.numel()
    passes = C.c_uint32()
    moved = C.c_uint64()
    _check(lib, lib.smmo_defragment(heap, class_id, n, k1, max_passes, arr if external else None, len(external),
                                    _stream(stream), C.byref(passes), C.byref(moved)))
    return passes.value, moved.value


def smmo_structure_remove_disconnected(heap, args, work, levels, stream=None) -> None:
    """The structure's BFS removal in one call (see smmo.h); work = device
    uint32/int32 tensor (the workspace), levels = device tensor of one word."""
    lib = load_library()
    _check(lib, lib.smmo_structure_remove_disconnected(heap, C.byref(args), _ptr(work), work.numel(), _ptr(levels),
                                                       _stream(stream)))


def smmo_structure_remove_disconnected_noalloc(heap, args, levels, stream=None) -> None:
    """The same without a workspace (the library's own device array; see smmo.h)."""
    lib = load_library()
    _check(lib, lib.smmo_structure_remove_disconnected_noalloc(heap, C.byref(args), _ptr(levels), _stream(stream)))


def smmo_coalescing_probe(data, C: int, grid: int = 0, stream=None) -> None:
    """One pass of the coalescing experiment over a float32 device tensor."""
    lib = load_library()
    _check(lib, lib.smmo_coalescing_probe(_ptr(data), data.numel(), C, grid, _stream(stream)))


def smmo_destroy(heap, class_id: int, handles, n: int, stream=None) -> None:
    lib = load_library()
    _check(lib, lib.smmo_destroy(heap, class_id, _ptr(handles), n, _stream(stream)))


def smmo_gather_soa(heap, class_id: int, field_ids, out_ptrs, out_handles, capacity: int, out_count,
                    stream=None) -> None:
    lib = load_library()
    n = len(field_ids)
    ids = (C.c_uint32 * max(1, n))(*field_ids)
    ptrs = (C.c_void_p * max(1, n))(*[_ptr(p) for p in out_ptrs])
    _check(lib, lib.smmo_gather_soa(heap, class_id, ids, n, ptrs, _ptr(out_handles), capacity,
                                    _ptr(out_count), _stream(stream)))


def smmo_sync(heap) -> None:
    lib = load_library()
    _check(lib, lib.smmo_sync(heap))


def smmo_heap_stats(heap) -> smmo_stats:
    lib = load_library()
    st = smmo_stats()
    _check(lib, lib.smmo_heap_stats(heap, C.byref(st)))
    return st


def smmo_check_invariants(heap) -> smmo_invariants:
    lib = load_library()
    inv = smmo_invariants()
    _check(lib, lib.smmo_check_invariants(heap, C.byref(inv)))
    return inv


def smmo_clear_error(heap, stream=None) -> None:
    lib = load_library()
    _check(lib, lib.smmo_clear_error(heap, _stream(stream)))


def smmo_heap_info(heap):
    lib = load_library()
    blocks = C.c_uint64()
    bb = C.c_uint32()
    _check(lib, lib.smmo_heap_info(heap, C.byref(blocks), C.byref(bb)))
    return blocks.value, bb.value


def smmo_method_id(name: str) -> int:
    lib = load_library()
    out = C.c_uint32()
    _check(lib, lib.smmo_method_id(name.encode(), C.byref(out)))
    return out.value


def smmo_set_launch(heap, method_id: int, class_id: int, wg_threads: int = 0, grid_waves: int = 0,
                    group: int = 0) -> None:
    lib = load_library()
    _check(lib, lib.smmo_set_launch(heap, method_id, class_id, wg_threads, grid_waves, group))


def smmo_last_error() -> str:
    return _last_error(load_library())


# ---- convenience: a heap owning its torch buffer ----------------------------
_TORCH_DT = {U8: "uint8", I32: "int32", U32: "int32", F32: "float32", HANDLE: "int32"}


class Heap:
    """A schema plus a heap in a torch-allocated device buffer.

    classes: {class name: [(field, dtype, count), ...]} in definition order,
    or {class name: {"parent": name or None, "abstract": bool, "fields": [...]}}
    for a class in a hierarchy (its field list starts with the parent's).
    Give either `blocks` (heap size in blocks) or `nbytes`.  With
    from_allocator the heap's buffer comes from the allocator set by
    smmo_set_allocator() and goes back to it when the heap is freed.
    """

    def __init__(self, classes: dict, blocks: int | None = None, nbytes: int | None = None,
                 cfg: smmo_config | None = None, device="cuda", from_allocator: bool = False):
        import torch

        self.torch = torch
        self.dev = torch.device(device)
        self.schema = smmo_schema_create()
        self.cls = {}
        self.fields = {}
        self._field_list = {}
        for cname, spec in classes.items():
            if isinstance(spec, dict):
                parent = spec.get("parent")
                flds = list(spec.get("fields", ()))
                cid = smmo_define_subclass(self.schema, cname, SMMO_NO_PARENT if parent is None else self.cls[parent],
                                           flds, bool(spec.get("abstract", False)))
                inherited = [] if parent is None else self._field_list[parent]
            else:
                flds = list(spec)
                cid = smmo_define_class(self.schema, cname, flds)
                inherited = []
            self.cls[cname] = cid
            full = inherited + flds
            self._field_list[cname] = full
            self.fields[cname] = {f[0]: (i, DTYPE_NAMES.get(f[1], f[1]) if isinstance(f[1], str) else f[1], f[2])
                                  for i, f in enumerate(full)}
        if nbytes is None:
            nbytes = smmo_heap_bytes(self.schema, blocks)
        self.nbytes = nbytes
        if from_allocator:
            self.buf = None
            self.h = smmo_alloc_heap(self.schema, None, nbytes, cfg)
        else:
            self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
            self.base = (self.buf.data_ptr() + 255) & ~255
            self.h = smmo_alloc_heap(self.schema, self.base, nbytes, cfg)
        self.blocks, self.block_bytes = smmo_heap_info(self.h)
        self._count = torch.zeros(1, dtype=torch.int32, device=device)

    def new(self, cname: str, n: int, stream=None, **values):
        """Creates n objects; values: field name -> tensor of n (or n*count) elements. Returns handles."""
        t = self.torch
        inits = []
        keep = []
        for fname, v in values.items():
            fid, dt, cnt = self.fields[cname][fname]
            v = t.as_tensor(v, device=self.dev)
            v = v.reshape(-1).contiguous()
            want = getattr(t, _TORCH_DT[dt])
            if v.dtype != want:
                v = v.to(want)
            assert v.numel() == n * cnt, (fname, v.numel(), n, cnt)
            keep.append(v)
            inits.append((fid, v))
        out = t.empty(max(n, 1), dtype=t.int32, device=self.dev)
        smmo_parallel_new(self.h, self.cls[cname], n, inits, out, stream)
        self._keep = keep   # alive until the next call (stream order keeps them valid)
        return out[:n]

    def do(self, cname: str, method: str, args=None, stream=None):
        smmo_parallel_do(self.h, self.cls[cname], smmo_method_id(method), args, stream)

    def snapshot(self, cname: str, stream=None):
        """Iteration snapshot of class cname for its next do-all."""
        smmo_snapshot(self.h, self.cls[cname], stream)

    def defragment(self, cname: str, n: int = 1, k1: int = 0, max_passes: int = 32, external=(), stream=None):
        """CompactGpu passes on class cname; returns (passes, moved objects).
        `external`: int32 device tensors of handles to rewrite too."""
        return smmo_defragment(self.h, self.cls[cname], n, k1, max_passes, external, stream)

    def destroy(self, cname: str, handles, stream=None):
        handles = handles.to(self.torch.int32).contiguous()
        smmo_destroy(self.h, self.cls[cname], handles, handles.numel(), stream)
        self._keep = [handles]

    def gather(self, cname: str, names=None, capacity: int | None = None, stream=None):
        """Dense copies of fields of the live objects, synchronizing.

        Returns {field: tensor, '_handle': handles, '_count': number of live
        objects (may exceed capacity)}."""
        t = self.torch
        if names is None:
            names = list(self.fields[cname].keys())
        if capacity is None:
            capacity = 64 * self.blocks
        outs = []
        ids = []
        for fname in names:
            fid, dt, cnt = self.fields[cname][fname]
            outs.append(t.empty(max(capacity * cnt, 1), dtype=getattr(t, _TORCH_DT[dt]), device=self.dev))
            ids.append(fid)
        hd = t.empty(max(capacity, 1), dtype=t.int32, device=self.dev)
        smmo_gather_soa(self.h, self.cls[cname], ids, outs, hd, capacity, self._count, stream)
        self.sync()
        n = int(self._count.item())
        k = min(n, capacity)
        res = {"_handle": hd[:k]}
        for fname, o in zip(names, outs):
            cnt = self.fields[cname][fname][2]
            res[fname] = o[: k * cnt].reshape(k, cnt) if cnt > 1 else o[:k]
        res["_count"] = n
        return res

    def sync(self):
        smmo_sync(self.h)

    def stats(self) -> smmo_stats:
        return smmo_heap_stats(self.h)

    def invariants(self) -> smmo_invariants:
        return smmo_check_invariants(self.h)

    def close(self):
        if getattr(self, "h", None):
            smmo_heap_free(self.h)
            self.h = None
        if getattr(self, "schema", None):
            smmo_schema_free(self.schema)
            self.schema = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
