"""Host logic of the launch-shape autotuner (no GPU): the cache key's parts
(method, class layout, power-of-two bucket of the class's block count), the
choice of the fastest candidate over every (work-group size, wavefronts,
group), and the cache written by tune() and read back by apply_cached()."""

import json
import types

import pytest

from paper_1908_05845_amd import autotune


class FakeHeap:
    """What the autotuner reads from a heap: class ids, field layouts and
    the per-class block counts of heap.stats()."""

    def __init__(self, blocks=1000, layout=None):
        self.h = object()
        self.cls = {"Node": 0, "Spring": 1}
        self.fields = {"Node": layout or {"x": (0, "f32", 1), "adj": (1, "handle", 8)},
                       "Spring": {"a": (0, "handle", 1)}}
        self._blocks = blocks

    def stats(self):
        return types.SimpleNamespace(blocks=[self._blocks, 7 * self._blocks])


def test_key_buckets_and_layout():
    k = lambda heap, b: autotune._key(heap, "spring.node_update", "Node", b)
    h = FakeHeap()
    # power-of-two buckets by rounded log2: 1000 and 1448 share 2^10, 1449 is 2^11
    assert k(h, 1000) == k(h, 1448) and k(h, 1448) != k(h, 1449)
    assert k(h, 1000).endswith("|2^10") and k(h, 1).endswith("|2^0") and k(h, 0).endswith("|2^0")
    # another layout of the class, another method or class: another key
    other = FakeHeap(layout={"x": (0, "f32", 1), "adj": (1, "handle", 4)})
    assert k(other, 1000) != k(h, 1000)
    assert autotune._key(h, "spring.force", "Node", 1000) != k(h, 1000)
    assert autotune._key(h, "spring.node_update", "Spring", 1000) != k(h, 1000)


@pytest.fixture
def fake_lib(monkeypatch):
    """smmo calls replaced by a record of the shapes set; the candidate's
    time is a function of the shape applied last."""
    applied = []
    monkeypatch.setattr(autotune.smmo, "smmo_method_id", lambda name: 3)
    monkeypatch.setattr(autotune.smmo, "smmo_set_launch",
                        lambda h, mid, cls, wg, waves, grp: applied.append((mid, cls, wg, waves, grp)))
    monkeypatch.setattr(autotune, "_cu_count", lambda torch: 256)
    return applied


def test_tune_keeps_the_fastest_and_caches_it(fake_lib, tmp_path, monkeypatch):
    import sys

    monkeypatch.setitem(sys.modules, "torch", types.SimpleNamespace())
    applied = fake_lib
    # fastest: work-group 128, 32 wavefronts per CU, group 2
    cost = lambda wg, waves, grp: abs(wg - 128) + abs(waves - 32 * 256) / 256 + 10 * abs(grp - 2) + 1.0
    timer = lambda: cost(*applied[-1][2:]) * 1e-6
    heap = FakeHeap(blocks=1000)
    cache = tmp_path / "shapes.json"
    r = autotune.tune(heap, "spring.node_update", "Node", None, groups=(1, 2, 4), timer=timer,
                      cache_path=str(cache))
    n = len(autotune.DEFAULT_WG) * len(autotune.DEFAULT_WAVES_PER_CU) * 3
    assert len(r["tried"]) == n and len(applied) == n + 1
    assert (r["wg"], r["waves"], r["group"]) == (128, 32 * 256, 2) and r["us"] == pytest.approx(1.0)
    assert applied[-1] == (3, 0, 128, 32 * 256, 2)            # the best is applied last
    assert r["blocks"] == 1000
    assert min(t["us"] for t in r["tried"]) == r["us"]
    stored = json.loads(cache.read_text())
    key = autotune._key(heap, "spring.node_update", "Node", 1000)
    assert stored == {key: {"wg": 128, "waves": 32 * 256, "group": 2, "us": r["us"]}}
    # another size in the same bucket reads it back; another bucket does not
    applied.clear()
    assert autotune.apply_cached(FakeHeap(blocks=1200), "spring.node_update", "Node", str(cache))["wg"] == 128
    assert applied == [(3, 0, 128, 32 * 256, 2)]
    assert autotune.apply_cached(FakeHeap(blocks=4000), "spring.node_update", "Node", str(cache)) is None
    assert autotune.apply_cached(heap, "spring.node_update", "Node", str(tmp_path / "none.json")) is None
