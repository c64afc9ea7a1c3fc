"""Autotuner of do-all launch shapes.

A do-all launch has three knobs (``smmo_set_launch``): the work-group size
(64 .. 1024 threads), the total number of wavefronts and, in the methods that
support it, the group: how many blocks a wavefront loads together before it
computes (1, 2 or 4).  Blocks per wavefront = ceil(blocks / wavefronts).  ``tune`` times every candidate with HIP events over repeated
launches of the method with arguments that make it idempotent (the caller
supplies them, e.g. dt = 0 for an update), keeps the fastest, applies it to
the heap and stores it in a JSON cache keyed by (method, class layout,
power-of-two bucket of the class's block count).  ``apply_cached`` reuses a
stored result without timing.
"""

import hashlib
import json
import math
import os

from . import smmo

DEFAULT_WG = (64, 128, 256, 512, 1024)
DEFAULT_WAVES_PER_CU = (8, 16, 32, 64, 128)


def _key(heap, method: str, cls_name: str, blocks: int) -> str:
    layout = json.dumps(sorted((k, v[1], v[2]) for k, v in heap.fields[cls_name].items()))
    h = hashlib.sha256(layout.encode()).hexdigest()[:12]
    bucket = int(round(math.log2(max(1, blocks))))
    return "%s|%s:%s|2^%d" % (method, cls_name, h, bucket)


def _cu_count(torch):
    return torch.cuda.get_device_properties(0).multi_processor_count


def time_launches(heap, method: str, cls_name: str, args, repeat: int) -> float:
    """Average seconds per launch over `repeat` back-to-back launches."""
    import torch

    mid = smmo.smmo_method_id(method)
    cls = heap.cls[cls_name]
    for _ in range(2):
        smmo.smmo_parallel_do(heap.h, cls, mid, args)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(repeat):
        smmo.smmo_parallel_do(heap.h, cls, mid, args)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / repeat


def tune(heap, method: str, cls_name: str, args, repeat: int = 20, wg_sizes=DEFAULT_WG,
         waves_per_cu=DEFAULT_WAVES_PER_CU, groups=(0,), cache_path: str | None = None,
         timer=None) -> dict:
    """Times every (work-group size, wavefronts, group) candidate, applies the
    best.  groups=(0,) keeps the method's default group.  By default a
    candidate is timed over `repeat` back-to-back launches of the method
    alone; `timer()` (seconds per unit, called with the candidate applied)
    replaces that, e.g. to time whole steps of a loop whose other launches
    evict this method's inputs from the caches.
    Returns {"wg", "waves", "group", "us", "tried": [...]}."""
    import torch

    cus = _cu_count(torch)
    mid = smmo.smmo_method_id(method)
    cls = heap.cls[cls_name]
    st = heap.stats()
    blocks = int(st.blocks[cls])
    tried = []
    best = None
    for grp in groups:
        for wg in wg_sizes:
            for wpc in waves_per_cu:
                waves = wpc * cus
                smmo.smmo_set_launch(heap.h, mid, cls, wg, waves, grp)
                t = timer() if timer is not None else time_launches(heap, method, cls_name, args, repeat)
                tried.append({"wg": wg, "waves": waves, "group": grp, "us": t * 1e6})
                if best is None or t < best[3]:
                    best = (wg, waves, grp, t)
    smmo.smmo_set_launch(heap.h, mid, cls, best[0], best[1], best[2])
    res = {"wg": best[0], "waves": best[1], "group": best[2], "us": best[3] * 1e6, "blocks": blocks,
           "tried": tried}
    if cache_path:
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        cache[_key(heap, method, cls_name, blocks)] = {"wg": best[0], "waves": best[1], "group": best[2],
                                                      "us": best[3] * 1e6}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return res


def apply_cached(heap, method: str, cls_name: str, cache_path: str) -> dict | None:
    """Applies a stored shape for this (method, class layout, size bucket), if any."""
    if not os.path.exists(cache_path):
        return None
    with open(cache_path) as f:
        cache = json.load(f)
    cls = heap.cls[cls_name]
    blocks = int(heap.stats().blocks[cls])
    ent = cache.get(_key(heap, method, cls_name, blocks))
    if ent is None:
        return None
    smmo.smmo_set_launch(heap.h, smmo.smmo_method_id(method), cls, ent["wg"], ent["waves"], ent.get("group", 0))
    return ent
