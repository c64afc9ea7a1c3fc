"""Workload drivers on the SMMO heap: Game of Life, n-body, spring meshes, wa-tor.

Each driver builds a heap, creates its objects with smmo_parallel_new from
dense arrays (as produced by the ``inputs`` package), runs steps as
sequences of smmo_parallel_do, and reads canonical state back with
smmo_gather_soa (ordered by the objects' key fields, since slot placement is
not part of the result).  Everything runs through libsmmo.
"""

import numpy as np

from . import smmo

GOL_CLASSES = {
    "Cell": [("state", "u8", 1), ("count", "i32", 1), ("cell_id", "i32", 1)],
    "Alive": [("cell_id", "i32", 1)],
}

GENERATION_CLASSES = {
    "Cell": [("state", "u8", 1), ("count", "i32", 1), ("cell_id", "i32", 1)],
    "Alive": [("cell_id", "i32", 1), ("left", "i32", 1), ("is_new", "u8", 1)],
}

NBODY_CLASSES = {
    "Body": [("pos_x", "f32", 1), ("pos_y", "f32", 1), ("vel_x", "f32", 1), ("vel_y", "f32", 1),
             ("force_x", "f32", 1), ("force_y", "f32", 1), ("mass", "f32", 1), ("id", "i32", 1)],
}

WATOR_CLASSES = {
    "Cell": [("agent", "handle", 1), ("nb", "handle", 4), ("req", "u8", 5), ("cell_id", "i32", 1)],
    "Fish": [("pos", "handle", 1), ("new_pos", "handle", 1), ("timer", "i32", 1)],
    "Shark": [("pos", "handle", 1), ("new_pos", "handle", 1), ("timer", "i32", 1), ("energy", "i32", 1)],
}

SPRING_CLASSES = {
    "Node": [("x", "f32", 1), ("y", "f32", 1), ("vx", "f32", 1), ("vy", "f32", 1), ("m", "f32", 1),
             ("adj", "handle", 8), ("id", "i32", 1)],
    "Spring": [("a", "handle", 1), ("b", "handle", 1), ("k", "f32", 1), ("L0", "f32", 1),
               ("fx", "f32", 1), ("fy", "f32", 1), ("slot_a", "u8", 1), ("slot_b", "u8", 1),
               ("id", "i32", 1)],
}


STRUCTURE_CLASSES = {
    "NodeBase": {"parent": None, "abstract": True,
                 "fields": [("x", "f32", 1), ("y", "f32", 1), ("springs", "handle", 3), ("nspr", "i32", 1),
                            ("dist", "i32", 1), ("id", "i32", 1)]},
    "AnchorNode": {"parent": "NodeBase"},
    "AnchorPullNode": {"parent": "NodeBase", "fields": [("vx", "f32", 1), ("vy", "f32", 1)]},
    "Node": {"parent": "NodeBase", "fields": [("vx", "f32", 1), ("vy", "f32", 1), ("m", "f32", 1)]},
    "Spring": [("p1", "handle", 1), ("p2", "handle", 1), ("k", "f32", 1), ("L0", "f32", 1), ("maxf", "f32", 1),
               ("fx", "f32", 1), ("fy", "f32", 1), ("s1", "u8", 1), ("s2", "u8", 1), ("del", "u8", 1),
               ("id", "i32", 1)],
}
STRUCTURE_NODE_CLASSES = ("AnchorNode", "AnchorPullNode", "Node")   # node types 0, 1, 2


def _blocks(n: int) -> int:
    return (n + 63) // 64


def _np(t):
    return t.detach().cpu().numpy()


class GolSim:
    """Game of Life in SMMO form on a W x H torus (Cell + Alive classes).

    fused=True runs each generation as one gol.generation do-all (death and
    birth in one launch on heaps of at most 8,192 blocks).
    concurrent=True runs Alive::death on a second stream beside Cell::birth:
    the two decide on disjoint cells (death on live cells whose count is not
    2 or 3, birth on dead cells with count 3).  The Alive snapshot is taken on
    that stream while Cell::count runs, so the death pass walks the Alive
    objects of the generation's start and never meets the ones births
    create."""

    def __init__(self, W: int, H: int, init, cfg=None, extra_blocks: int = 16, concurrent: bool = False,
                 fused: bool = False):
        import torch

        self.W, self.H = W, H
        self.concurrent = concurrent
        self.fused = fused
        n = W * H
        self.heap = smmo.Heap(GOL_CLASSES, blocks=3 * _blocks(n) + extra_blocks, cfg=cfg)
        dev = self.heap.dev
        init = np.ascontiguousarray(init, dtype=np.uint8).reshape(-1)
        ids = torch.arange(n, dtype=torch.int32, device=dev)
        self.cells = self.heap.new("Cell", n, state=torch.from_numpy(init).to(dev), cell_id=ids).clone()
        live = torch.from_numpy(np.flatnonzero(init).astype(np.int32)).to(dev)
        if live.numel():
            self.heap.new("Alive", live.numel(), cell_id=live)
        self.args = smmo.smmo_gol_args(self.heap.cls["Cell"], self.heap.cls["Alive"],
                                       self.cells.data_ptr(), W, H)
        self.m_count = smmo.smmo_method_id("gol.cell_count")
        self.m_death = smmo.smmo_method_id("gol.alive_death")
        self.m_birth = smmo.smmo_method_id("gol.cell_birth")
        self.m_gen = smmo.smmo_method_id("gol.generation")
        if concurrent:
            self._side = torch.cuda.Stream(device=dev)
            self._ev = [torch.cuda.Event() for _ in range(3)]

    def step(self, n: int = 1, stream=None):
        h, c, a = self.heap.h, self.heap.cls["Cell"], self.heap.cls["Alive"]
        if self.fused:
            for _ in range(n):
                smmo.smmo_parallel_do(h, c, self.m_gen, self.args, stream)
            return
        if not self.concurrent:
            for _ in range(n):
                smmo.smmo_parallel_do(h, c, self.m_count, self.args, stream)
                smmo.smmo_parallel_do(h, a, self.m_death, self.args, stream)
                smmo.smmo_parallel_do(h, c, self.m_birth, self.args, stream)
            return
        import torch

        main = torch.cuda.current_stream(self.heap.dev) if stream is None else stream
        if isinstance(main, int):
            main = torch.cuda.ExternalStream(main, device=self.heap.dev)
        side, (fork, counted, died) = self._side, self._ev
        for _ in range(n):
            fork.record(main)
            side.wait_event(fork)
            smmo.smmo_snapshot(h, a, side)
            smmo.smmo_parallel_do(h, c, self.m_count, self.args, main)
            counted.record(main)
            side.wait_event(counted)
            smmo.smmo_parallel_do(h, a, self.m_death, self.args, side)
            smmo.smmo_parallel_do(h, c, self.m_birth, self.args, main)
            died.record(side)
            main.wait_event(died)

    def read(self):
        """(state u8[W*H], count i32[W*H], sorted cell ids of Alive objects)."""
        g = self.heap.gather("Cell", ["state", "count", "cell_id"])
        nc = self.W * self.H
        cid = _np(g["cell_id"])
        state = np.zeros(nc, np.uint8)
        count = np.zeros(nc, np.int32)
        state[cid] = _np(g["state"])
        count[cid] = _np(g["count"])
        a = self.heap.gather("Alive", ["cell_id"])
        return state, count, np.sort(_np(a["cell_id"]))


def spring_pi_classes(K: int) -> dict:
    """Node and Spring classes of a mesh whose node adjacency keeps K slots
    inline (the rest outside the heap)."""
    return {
        "Node": [("x", "f32", 1), ("y", "f32", 1), ("vx", "f32", 1), ("vy", "f32", 1), ("m", "f32", 1),
                 ("adj", "handle", K), ("more", "i32", 1), ("cap", "i32", 1), ("id", "i32", 1)],
        "Spring": [("a", "handle", 1), ("b", "handle", 1), ("k", "f32", 1), ("L0", "f32", 1), ("fx", "f32", 1),
                   ("fy", "f32", 1), ("slot_a", "u8", 1), ("slot_b", "u8", 1), ("id", "i32", 1)],
    }


class SpringPiSim:
    """Spring-mass mesh of any node degree with partially inlined adjacency
    (thesis Ch.4 sec.4.3.1): the first K slots of a node in its block, the
    other slots in one device array, each node's at an offset `more`.
    Springs with alive == 0 (if an 'alive' array is given) are not created;
    a node's slot count is its highest slot in `adj` that names a spring,
    plus one."""

    def __init__(self, mesh: dict, dt: float, K: int, strain_limit: float = 0.3, cfg=None, extra_blocks: int = 16):
        import torch

        adj = np.asarray(mesh["adj"], np.int32)
        N = int(np.asarray(mesh["x"]).size)
        adj = adj.reshape(N, -1)
        S_all = int(np.asarray(mesh["a"]).size)
        alive = np.ones(S_all, bool) if mesh.get("alive") is None else np.asarray(mesh["alive"]).astype(bool)
        sid = np.flatnonzero(alive).astype(np.int64)
        used = adj >= 0
        cap = np.where(used.any(axis=1), adj.shape[1] - np.argmax(used[:, ::-1], axis=1), 0).astype(np.int32)
        extra = np.maximum(cap - K, 0).astype(np.int64)
        more = (np.cumsum(extra) - extra).astype(np.int32)
        S = sid.size
        self.N, self.S, self.K, self.D = N, S_all, K, adj.shape[1]
        self.cap, self.more = cap, more
        self.heap = smmo.Heap(spring_pi_classes(K), blocks=_blocks(N) + _blocks(S) + extra_blocks, cfg=cfg)
        dev = self.heap.dev
        f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
        i32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(dev)
        self.overflow = torch.full((max(int(extra.sum()), 1),), -1, dtype=torch.int32, device=dev)
        self.node_h = self.heap.new("Node", N, x=f32(mesh["x"]), y=f32(mesh["y"]), vx=f32(mesh["vx"]),
                                    vy=f32(mesh["vy"]), m=f32(mesh["m"]),
                                    adj=torch.full((N * K,), -1, dtype=torch.int32, device=dev),
                                    more=i32(more), cap=i32(cap), id=i32(np.arange(N))).clone()
        u8 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint8)).to(dev)
        if S:
            a_idx = torch.from_numpy(np.asarray(mesh["a"], np.int64)[sid]).to(dev)
            b_idx = torch.from_numpy(np.asarray(mesh["b"], np.int64)[sid]).to(dev)
            self.heap.new("Spring", S, a=self.node_h[a_idx], b=self.node_h[b_idx],
                          k=f32(np.asarray(mesh["k"])[sid]), L0=f32(np.asarray(mesh["L0"])[sid]),
                          slot_a=u8(np.asarray(mesh["slot_a"])[sid]), slot_b=u8(np.asarray(mesh["slot_b"])[sid]),
                          id=i32(sid))
        self.args = smmo.smmo_spring_pi_args(self.heap.cls["Node"], self.heap.cls["Spring"], dt, strain_limit,
                                             self.overflow.data_ptr(), int(extra.sum()))
        self.m_force = smmo.smmo_method_id("spring_pi.force")
        self.m_node = smmo.smmo_method_id("spring_pi.node_update")
        if S:
            smmo.smmo_parallel_do(self.heap.h, self.heap.cls["Spring"], smmo.smmo_method_id("spring_pi.link"),
                                  self.args)

    def step(self, n: int = 1, stream=None):
        h, cs, cn = self.heap.h, self.heap.cls["Spring"], self.heap.cls["Node"]
        for _ in range(n):
            smmo.smmo_parallel_do(h, cs, self.m_force, self.args, stream)
            smmo.smmo_parallel_do(h, cn, self.m_node, self.args, stream)

    def read(self) -> dict:
        """Node arrays by id; adjacency (N, D) as spring ids (-1 empty, -2 a
        handle of no live spring), from the inline and out-of-line slots."""
        N, S, K, D = self.N, self.S, self.K, self.D
        gs = self.heap.gather("Spring", ["id", "fx", "fy"])
        sid = _np(gs["id"])
        sh = _np(gs["_handle"]).astype(np.int64)
        out = {"alive": np.zeros(S, np.uint8), "fx": np.zeros(S, np.float32), "fy": np.zeros(S, np.float32)}
        out["alive"][sid] = 1
        out["fx"][sid] = _np(gs["fx"])
        out["fy"][sid] = _np(gs["fy"])
        gn = self.heap.gather("Node", ["id", "x", "y", "vx", "vy", "m", "adj"])
        order = np.argsort(_np(gn["id"]))
        for key in ("x", "y", "vx", "vy", "m"):
            out[key] = _np(gn[key])[order]
        raw = np.full((N, D), 0xFFFFFFFF, np.int64)
        raw[:, :min(K, D)] = (_np(gn["adj"]).reshape(-1, K)[order].astype(np.int64) & 0xFFFFFFFF)[:, :min(K, D)]
        ovf = _np(self.overflow).astype(np.int64) & 0xFFFFFFFF
        for i in np.flatnonzero(self.cap > K):
            raw[i, K:self.cap[i]] = ovf[self.more[i]:self.more[i] + self.cap[i] - K]
        used = raw != 0xFFFFFFFF
        hh = raw & 0x7FFFFFFF
        hs = np.argsort(sh)
        sh_sorted, sid_sorted = sh[hs], sid[hs]
        if sh_sorted.size:
            pos = np.clip(np.searchsorted(sh_sorted, hh), 0, sh_sorted.size - 1)
            adj = np.where(used, np.where(sh_sorted[pos] == hh, sid_sorted[pos], -2), -1)
        else:
            adj = np.where(used, -2, -1)
        out["adj"] = adj.astype(np.int32)
        out["adj_is_b"] = np.where(used, raw >> 31, 0).astype(np.uint8)
        return out


def _rule_mask(counts) -> int:
    m = 0
    for c in counts:
        m |= 1 << int(c)
    return m


class GenerationSim:
    """The generational cellular automaton of thesis Ch.7 "generation" (Game
    of Life with dying cells; rule Burst by default) on a W x H torus, in the
    Cell + Alive form: an Alive object per live or dying cell."""

    def __init__(self, W: int, H: int, init, survive=(0, 2, 3, 5, 6, 7, 8), birth=(3, 4, 6, 8), dying: int = 255,
                 cfg=None, extra_blocks: int = 16):
        import torch

        self.W, self.H = W, H
        n = W * H
        self.heap = smmo.Heap(GENERATION_CLASSES, blocks=3 * _blocks(n) + extra_blocks, cfg=cfg)
        dev = self.heap.dev
        init = np.ascontiguousarray(init, dtype=np.uint8).reshape(-1)
        assert init.size == n and init.max(initial=0) <= 1
        ids = torch.arange(n, dtype=torch.int32, device=dev)
        self.cells = self.heap.new("Cell", n, state=torch.from_numpy(init).to(dev), cell_id=ids).clone()
        live = np.flatnonzero(init).astype(np.int32)
        if live.size:
            self.heap.new("Alive", live.size, cell_id=torch.from_numpy(live).to(dev))
        self.args = smmo.smmo_generation_args(self.heap.cls["Cell"], self.heap.cls["Alive"], W, H,
                                              _rule_mask(survive), _rule_mask(birth), dying, 0,
                                              self.cells.data_ptr())
        self.m_count = smmo.smmo_method_id("generation.cell_count")
        self.m_birth = smmo.smmo_method_id("generation.cell_birth")
        self.m_update = smmo.smmo_method_id("generation.alive_update")

    def step(self, n: int = 1, stream=None):
        h, c, a = self.heap.h, self.heap.cls["Cell"], self.heap.cls["Alive"]
        for _ in range(n):
            smmo.smmo_parallel_do(h, c, self.m_count, self.args, stream)
            smmo.smmo_parallel_do(h, c, self.m_birth, self.args, stream)
            smmo.smmo_parallel_do(h, a, self.m_update, self.args, stream)

    def read(self):
        """(state u8[W*H], left i32[W*H], number of Alive objects); raises if
        a cell and its Alive object disagree."""
        n = self.W * self.H
        g = self.heap.gather("Cell", ["state", "cell_id"])
        state = np.zeros(n, np.uint8)
        state[_np(g["cell_id"])] = _np(g["state"])
        a = self.heap.gather("Alive", ["cell_id", "left", "is_new"])
        cid = _np(a["cell_id"])
        left = np.zeros(n, np.int32)
        left[cid] = _np(a["left"])
        occupied = np.zeros(n, np.int64)
        np.add.at(occupied, cid, 1)
        if np.any(occupied > 1) or not np.array_equal(occupied > 0, state > 0) or np.any(_np(a["is_new"])):
            raise AssertionError("generation: cells and Alive objects disagree")
        return state, left, int(cid.size)


class NbodySim:
    """All-pairs n-body (class Body) with Plummer softening."""

    def __init__(self, state: dict, G: float, eps: float, dt: float, cfg=None, extra_blocks: int = 8):
        import torch

        n = int(np.asarray(state["x"]).size)
        self.n = n
        self.heap = smmo.Heap(NBODY_CLASSES, blocks=_blocks(n) + extra_blocks, cfg=cfg)
        dev = self.heap.dev

        def t(a):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)

        self.handles = self.heap.new("Body", n, pos_x=t(state["x"]), pos_y=t(state["y"]),
                                     vel_x=t(state["vx"]), vel_y=t(state["vy"]), mass=t(state["m"]),
                                     id=torch.arange(n, dtype=torch.int32, device=dev)).clone()
        self.args = smmo.smmo_nbody_args(G, eps, dt, 0)
        self.m_force = smmo.smmo_method_id("nbody.force")
        self.m_update = smmo.smmo_method_id("nbody.update")
        self.cls = self.heap.cls["Body"]

    def force(self, stream=None):
        smmo.smmo_parallel_do(self.heap.h, self.cls, self.m_force, self.args, stream)

    def update(self, stream=None):
        smmo.smmo_parallel_do(self.heap.h, self.cls, self.m_update, self.args, stream)

    def step(self, n: int = 1, stream=None):
        for _ in range(n):
            self.force(stream)
            self.update(stream)

    def read(self):
        g = self.heap.gather("Body")
        order = np.argsort(_np(g["id"]))
        out = {}
        for key, f in (("x", "pos_x"), ("y", "pos_y"), ("vx", "vel_x"), ("vy", "vel_y"),
                       ("fx", "force_x"), ("fy", "force_y"), ("m", "mass")):
            out[key] = _np(g[f])[order]
        out["id"] = _np(g["id"])[order]
        return out


class SpringSim:
    """Spring-mass mesh (classes Node and Spring) built from a mesh dict.

    The mesh dict has the arrays of ``inputs.spring_mesh`` (ids local to the
    arrays).  Springs with alive == 0 (if an 'alive' array is given) are not
    created.  Node adjacency is built on the device by spring.link.
    tension_only: springs pull only (no force while shorter than L0).
    """

    def __init__(self, mesh: dict, dt: float, strain_limit: float = 0.3, cfg=None, extra_blocks: int = 16,
                 blocks: int | None = None, tension_only: bool = False):
        import torch

        N = int(np.asarray(mesh["x"]).size)
        S_all = int(np.asarray(mesh["a"]).size)
        alive = np.ones(S_all, bool) if mesh.get("alive") is None else np.asarray(mesh["alive"]).astype(bool)
        sid = np.flatnonzero(alive).astype(np.int32)
        S = sid.size
        self.N, self.S_all = N, S_all
        if blocks is None:
            blocks = _blocks(N) + _blocks(S) + extra_blocks
        self.heap = smmo.Heap(SPRING_CLASSES, blocks=blocks, cfg=cfg)
        dev = self.heap.dev

        def f32(a):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)

        def i32(a):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(dev)

        null_adj = torch.full((N * 8,), -1, dtype=torch.int32, device=dev)
        self.node_h = self.heap.new("Node", N, x=f32(mesh["x"]), y=f32(mesh["y"]), vx=f32(mesh["vx"]),
                                    vy=f32(mesh["vy"]), m=f32(mesh["m"]), adj=null_adj,
                                    id=torch.arange(N, dtype=torch.int32, device=dev)).clone()
        a_idx = i32(np.asarray(mesh["a"])[sid]).long()
        b_idx = i32(np.asarray(mesh["b"])[sid]).long()
        fx = mesh.get("fx")
        fy = mesh.get("fy")
        kw = {}
        if fx is not None:
            kw["fx"] = f32(np.asarray(fx)[sid])
            kw["fy"] = f32(np.asarray(fy)[sid])
        if S:
            self.spring_h = self.heap.new(
                "Spring", S, a=self.node_h[a_idx], b=self.node_h[b_idx], k=f32(np.asarray(mesh["k"])[sid]),
                L0=f32(np.asarray(mesh["L0"])[sid]),
                slot_a=torch.from_numpy(np.asarray(mesh["slot_a"])[sid].astype(np.uint8)).to(dev),
                slot_b=torch.from_numpy(np.asarray(mesh["slot_b"])[sid].astype(np.uint8)).to(dev),
                id=i32(sid), **kw).clone()
        self.args = smmo.smmo_spring_args(self.heap.cls["Node"], self.heap.cls["Spring"], dt, strain_limit,
                                          smmo.SMMO_SPRING_TENSION_ONLY if tension_only else 0)
        self.m_force = smmo.smmo_method_id("spring.force")
        self.m_node = smmo.smmo_method_id("spring.node_update")
        self.m_link = smmo.smmo_method_id("spring.link")
        if S:
            smmo.smmo_parallel_do(self.heap.h, self.heap.cls["Spring"], self.m_link, self.args)

    def spring_force(self, stream=None):
        smmo.smmo_parallel_do(self.heap.h, self.heap.cls["Spring"], self.m_force, self.args, stream)

    def node_update(self, stream=None):
        smmo.smmo_parallel_do(self.heap.h, self.heap.cls["Node"], self.m_node, self.args, stream)

    def step(self, n: int = 1, stream=None):
        for _ in range(n):
            self.spring_force(stream)
            self.node_update(stream)

    def read(self):
        """Canonical state: node arrays by node id, spring arrays by spring id
        (alive flags for springs; adjacency as spring ids, -1 empty)."""
        gs = self.heap.gather("Spring", ["id", "fx", "fy", "a", "b"])
        gn = self.heap.gather("Node", ["id", "x", "y", "vx", "vy", "m", "adj"])
        S = self.S_all
        sid = _np(gs["id"])
        sh = _np(gs["_handle"]).astype(np.int64)
        alive = np.zeros(S, np.uint8)
        alive[sid] = 1
        fx = np.zeros(S, np.float32)
        fy = np.zeros(S, np.float32)
        fx[sid] = _np(gs["fx"])
        fy[sid] = _np(gs["fy"])
        hs = np.argsort(sh)
        sh_sorted, sid_sorted = sh[hs], sid[hs]
        nid = _np(gn["id"])
        order = np.argsort(nid)
        out = {"alive": alive, "fx": fx, "fy": fy}
        for key in ("x", "y", "vx", "vy", "m"):
            out[key] = _np(gn[key])[order]
        raw = _np(gn["adj"]).reshape(-1, 8)[order].astype(np.int64) & 0xFFFFFFFF
        used = raw != 0xFFFFFFFF
        hh = raw & 0x7FFFFFFF
        pos = np.clip(np.searchsorted(sh_sorted, hh), 0, max(sh_sorted.size - 1, 0))
        found = (sh_sorted[pos] == hh) if sh_sorted.size else np.zeros(raw.shape, bool)
        # -1 empty slot; -2 a handle that names no live spring (an error)
        adj = np.where(used, np.where(found, sid_sorted[pos] if sid_sorted.size else -2, -2), -1)
        out["adj"] = adj.astype(np.int32)
        out["adj_is_b"] = np.where(used, raw >> 31, 0).astype(np.uint8)
        out["node_handles_by_id"] = _np(gn["_handle"])[order]
        return out


class WatorSim:
    """wa-tor (classes Cell, Fish, Shark) on a W x H torus.

    params = (fish_spawn, shark_spawn, energy0, boost); init = per-cell arrays
    kind / timer / energy as made by ``inputs.wator_init``; seed keys the
    random choices.  The heap holds the cells plus room for `agent_room`
    agents of each kind (default: one per cell)."""

    STEPS = (("Cell", "wator.cell_prepare", 0), ("Fish", "wator.fish_prepare", 0),
             ("Cell", "wator.cell_decide", 1), ("Fish", "wator.fish_update", 0),
             ("Cell", "wator.cell_prepare", 0), ("Shark", "wator.shark_prepare", 0),
             ("Cell", "wator.cell_decide", 2), ("Shark", "wator.shark_update", 0))

    def __init__(self, W: int, H: int, seed: int, params, init: dict, cfg=None, agent_room: int | None = None):
        import torch

        self.torch = torch
        self.W, self.H = W, H
        n = W * H
        room = n if agent_room is None else agent_room
        self.heap = smmo.Heap(WATOR_CLASSES, blocks=_blocks(n) + 2 * (2 * _blocks(room) + 64), cfg=cfg)
        dev = self.heap.dev
        self.dev = dev
        ids = torch.arange(n, dtype=torch.int32, device=dev)
        null = torch.full((n,), -1, dtype=torch.int32, device=dev)
        self.cells = self.heap.new("Cell", n, agent=null, nb=torch.full((4 * n,), -1, dtype=torch.int32,
                                                                       device=dev),
                                   cell_id=ids).clone()
        c = self.heap.cls
        fs, ss, e0, boost = (int(v) for v in params)
        self.args = smmo.smmo_wator_args(c["Cell"], c["Fish"], c["Shark"], 0, seed & ((1 << 64) - 1),
                                         fs, ss, e0, boost, 0, W, H, 0, self.cells.data_ptr())
        self.heap.do("Cell", "wator.cell_link", self.args)
        kind = np.asarray(init["kind"])
        for k, cname in ((1, "Fish"), (2, "Shark")):
            where = np.flatnonzero(kind == k)
            if where.size == 0:
                continue
            idx = torch.from_numpy(where.astype(np.int64)).to(dev)
            pos = self.cells[idx]
            vals = {"pos": pos, "new_pos": pos,
                    "timer": torch.from_numpy(np.asarray(init["timer"])[where].astype(np.int32)).to(dev)}
            if k == 2:
                vals["energy"] = torch.from_numpy(np.asarray(init["energy"])[where].astype(np.int32)).to(dev)
            self.heap.new(cname, where.size, **vals)
            self.args.kind = k
            self.heap.do(cname, "wator.link", self.args)
        self.t = 0
        self._launch = [(c[cn], smmo.smmo_method_id(m), kd) for cn, m, kd in self.STEPS]

    def step(self, n: int = 1, stream=None):
        lib = smmo.load_library()
        st = smmo._stream(stream)
        ref = smmo.C.byref(self.args)
        size = smmo.C.sizeof(self.args)
        for _ in range(n):
            self.args.iteration = self.t
            for cls, mid, kd in self._launch:
                self.args.kind = kd
                status = lib.smmo_parallel_do(self.heap.h, cls, mid, ref, size, st)
                if status:
                    raise smmo.SmmoError(status, smmo._last_error(lib))
            self.t += 1

    def read(self):
        """Per cell index: kind (u8), timer, energy (i32; 0 where they do not
        apply); (live fish, live sharks).  Raises if a cell and its agent
        disagree."""
        n = self.W * self.H
        cells = self.cells.cpu().numpy().view(np.uint32)
        order = np.argsort(cells)
        sc = cells[order]

        def cell_of(handles):
            hh = handles.cpu().numpy().view(np.uint32)
            j = np.searchsorted(sc, hh)
            if hh.size and (np.any(j >= n) or np.any(sc[np.minimum(j, n - 1)] != hh)):
                raise RuntimeError("an agent names no cell")
            return order[j]

        g = self.heap.gather("Cell", ["cell_id", "agent"])
        agent = np.full(n, 0xFFFFFFFF, np.uint32)
        agent[g["cell_id"].cpu().numpy()] = g["agent"].cpu().numpy().view(np.uint32)
        kind = np.zeros(n, np.uint8)
        timer = np.zeros(n, np.int32)
        energy = np.zeros(n, np.int32)
        f = self.heap.gather("Fish", ["pos", "timer"])
        fc = cell_of(f["pos"])
        sh = self.heap.gather("Shark", ["pos", "timer", "energy"])
        scl = cell_of(sh["pos"])
        if np.unique(np.concatenate([fc, scl])).size != fc.size + scl.size:
            raise RuntimeError("two agents on one cell")
        kind[fc] = 1
        timer[fc] = f["timer"].cpu().numpy()
        kind[scl] = 2
        timer[scl] = sh["timer"].cpu().numpy()
        energy[scl] = sh["energy"].cpu().numpy()
        want = np.full(n, 0xFFFFFFFF, np.uint32)
        want[fc] = f["_handle"].cpu().numpy().view(np.uint32)
        want[scl] = sh["_handle"].cpu().numpy().view(np.uint32) | np.uint32(0x80000000)
        if not np.array_equal(agent, want):
            raise RuntimeError("cell agent fields disagree with the agents' positions in %d cells"
                               % int(np.sum(agent != want)))
        return kind, timer, energy, (int(fc.size), int(scl.size))


class StructureSim:
    """The fracture simulation (thesis Ch.7 "structure") on a mesh dict of
    ``inputs.structure_mesh``: classes NodeBase (abstract), AnchorNode,
    AnchorPullNode, Node and Spring.  One iteration: AnchorPullNode::pull,
    `substeps` x (Spring::force, Node::update), then the removal of the nodes
    no longer connected to an anchor node: a BFS whose frontier is a queue,
    all levels run on the device by one call (bfs="queue", the default), or
    the thesis's form, the level passes launched `bfs_batch` at a time
    between reads of their frontier flags (bfs="levels").  bfs_options
    (SMMO_BFS_* bits) selects the queue BFS's forms for large meshes.
    A state with deleted objects loads too: nodes with nalive == 0 and
    springs with salive == 0 (where those arrays are given) are not created;
    nspr, dist and (where given) the spring forces fx, fy are taken from the
    state."""

    def __init__(self, mesh: dict, dt: float, cfg=None, extra_blocks: int = 16, bfs_batch: int = 8,
                 bfs: str = "queue", bfs_options: int = 0):
        import torch

        if bfs not in ("queue", "levels"):
            raise ValueError("bfs must be 'queue' or 'levels'")
        self.torch = torch
        self.dt = dt
        self.bfs_batch = bfs_batch
        self.bfs = bfs
        ntype = np.asarray(mesh["ntype"], np.int32)
        N = ntype.size
        S = int(np.asarray(mesh["p1"]).size)
        self.N, self.S = N, S
        self.ntype_all = ntype.copy()
        nalive = np.ones(N, bool) if mesh.get("nalive") is None else np.asarray(mesh["nalive"]).astype(bool)
        salive = np.ones(S, bool) if mesh.get("salive") is None else np.asarray(mesh["salive"]).astype(bool)
        dist0 = np.zeros(N, np.int32) if mesh.get("dist") is None else np.asarray(mesh["dist"], np.int32)
        per = [int(((ntype == t) & nalive).sum()) for t in range(3)]
        blocks = sum(_blocks(n) for n in per) + _blocks(int(salive.sum())) + extra_blocks
        self.heap = smmo.Heap(STRUCTURE_CLASSES, blocks=blocks, cfg=cfg)
        dev = self.heap.dev
        self.dev = dev
        f32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
        i32 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(dev)
        node_h = torch.full((max(N, 1),), -1, dtype=torch.int32, device=dev)
        self.node_ids = []
        for t, cname in enumerate(STRUCTURE_NODE_CLASSES):
            ids = np.flatnonzero((ntype == t) & nalive)
            self.node_ids.append(ids)
            if ids.size == 0:
                continue
            vals = dict(x=f32(np.asarray(mesh["x"])[ids]), y=f32(np.asarray(mesh["y"])[ids]),
                        springs=torch.full((ids.size * 3,), -1, dtype=torch.int32, device=dev),
                        nspr=i32(np.asarray(mesh["nspr"])[ids]), dist=i32(dist0[ids]), id=i32(ids))
            if cname != "AnchorNode":
                vals["vx"] = f32(np.asarray(mesh["vx"])[ids])
                vals["vy"] = f32(np.asarray(mesh["vy"])[ids])
            if cname == "Node":
                vals["m"] = f32(np.asarray(mesh["m"])[ids])
            node_h[torch.from_numpy(ids).to(dev)] = self.heap.new(cname, ids.size, **vals)
        self.node_h = node_h
        c = self.heap.cls
        self.flags = torch.zeros(max(bfs_batch, 1), dtype=torch.int32, device=dev)
        # the queue BFS's workspace (header, queue, block positions, visited
        # bits, neighbour table), sized by the heap's block count
        self.bfs_work = torch.empty(68 + 324 * self.heap.blocks, dtype=torch.int32, device=dev)
        self.bfs_levels = torch.zeros(1, dtype=torch.int32, device=dev)
        self.args = smmo.smmo_structure_args(c["NodeBase"], c["AnchorNode"], c["Spring"], 0, dt, bfs_options, None)
        self.m = {n: smmo.smmo_method_id("structure." + n) for n in
                  ("pull", "force", "node_update", "bfs_init", "bfs_visit", "bfs_mark", "bfs_delete", "link")}
        sid = np.flatnonzero(salive)
        if sid.size:
            p1 = torch.from_numpy(np.asarray(mesh["p1"], np.int64)[sid]).to(dev)
            p2 = torch.from_numpy(np.asarray(mesh["p2"], np.int64)[sid]).to(dev)
            u8 = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint8)).to(dev)
            sel = lambda key: np.asarray(mesh[key])[sid]
            # "del" is a Python keyword: the field values go in as a dict
            vals = {"p1": node_h[p1], "p2": node_h[p2], "k": f32(sel("k")), "L0": f32(sel("L0")),
                    "maxf": f32(sel("maxf")), "s1": u8(sel("s1")), "s2": u8(sel("s2")),
                    "del": u8(np.zeros(sid.size)), "id": i32(sid)}
            if mesh.get("fx") is not None:
                vals["fx"] = f32(sel("fx"))
                vals["fy"] = f32(sel("fy"))
            self.heap.new("Spring", sid.size, **vals)
            self.do("Spring", "link")
        self.levels = 0

    def do(self, cname: str, method: str, stream=None):
        smmo.smmo_parallel_do(self.heap.h, self.heap.cls[cname], self.m[method], self.args, stream)

    def pull(self, dt: float, stream=None):
        self.args.dt = dt
        self.do("AnchorPullNode", "pull", stream)

    def compute_step(self, stream=None):
        self.args.dt = self.dt
        self.do("Spring", "force", stream)
        self.do("Node", "node_update", stream)

    def remove_disconnected(self, stream=None) -> int:
        """BFS from the anchor nodes, then deletion of the unvisited nodes and
        their springs.  Returns the number of visit passes until the first
        empty frontier (as the thesis's loop runs them)."""
        if self.bfs == "queue":
            smmo.smmo_structure_remove_disconnected(self.heap.h, self.args, self.bfs_work, self.bfs_levels, stream)
            self.heap.sync()
            self.levels = int(self.bfs_levels.cpu().item())
            return self.levels
        self.do("NodeBase", "bfs_init", stream)
        d = 0
        while True:
            # the flags are cleared and read back between host synchronizations
            # with the heap's stream, which the visit launches run on
            self.heap.sync()
            self.flags.zero_()
            self.torch.cuda.synchronize()
            for j in range(self.bfs_batch):
                self.args.distance = d + j
                self.args.flag = self.flags.data_ptr() + 4 * j
                self.do("NodeBase", "bfs_visit", stream)
            self.args.flag = None
            self.heap.sync()
            fl = self.flags.cpu().numpy()
            empty = np.flatnonzero(fl == 0)
            if empty.size:
                self.levels = d + int(empty[0]) + 1
                break
            d += self.bfs_batch
        self.do("NodeBase", "bfs_mark", stream)
        self.do("Spring", "bfs_delete", stream)
        return self.levels

    def iterate(self, substeps: int, stream=None) -> int:
        self.pull(self.dt * substeps, stream)
        for _ in range(substeps):
            self.compute_step(stream)
        return self.remove_disconnected(stream)

    def read(self) -> dict:
        """Canonical state in the layout of ``inputs.structure_mesh`` (node
        arrays by node id, spring arrays by spring id, alive flags, slots as
        spring ids)."""
        N, S = self.N, self.S
        gs = self.heap.gather("Spring", ["id", "fx", "fy", "del"])
        sid = _np(gs["id"])
        sh = _np(gs["_handle"]).astype(np.int64)
        out = {"nalive": np.zeros(N, np.uint8), "salive": np.zeros(S, np.uint8)}
        out["salive"][sid] = 1
        for key, dt in (("fx", np.float32), ("fy", np.float32), ("sdel", np.uint8)):
            out[key] = np.zeros(S, dt)
            out[key][sid] = _np(gs["del" if key == "sdel" else key])
        hs = np.argsort(sh)
        sh_sorted, sid_sorted = sh[hs], sid[hs]
        for key, dt in (("x", np.float32), ("y", np.float32), ("vx", np.float32), ("vy", np.float32),
                        ("m", np.float32), ("nspr", np.int32), ("dist", np.int32), ("ntype", np.int32)):
            out[key] = np.zeros(N, dt)
        out["m"][:] = 1
        raw = np.full((N, 3), 0xFFFFFFFF, np.int64)
        for t, cname in enumerate(STRUCTURE_NODE_CLASSES):
            names = ["id", "x", "y", "springs", "nspr", "dist"] + (["vx", "vy"] if cname != "AnchorNode" else []) \
                + (["m"] if cname == "Node" else [])
            g = self.heap.gather(cname, names)
            ids = _np(g["id"])
            out["nalive"][ids] = 1
            out["ntype"][ids] = t
            for key in names[1:]:
                if key == "springs":
                    raw[ids] = _np(g["springs"]).reshape(-1, 3).astype(np.int64) & 0xFFFFFFFF
                else:
                    out[key][ids] = _np(g[key])
        dead = out["nalive"] == 0
        out["ntype"][:] = self.ntype_all
        used = raw != 0xFFFFFFFF
        hh = raw & 0x7FFFFFFF
        if sh_sorted.size:
            pos = np.clip(np.searchsorted(sh_sorted, hh), 0, sh_sorted.size - 1)
            found = sh_sorted[pos] == hh
            slot = np.where(used, np.where(found, sid_sorted[pos], -2), -1)
        else:
            slot = np.where(used, -2, -1)
        slot[dead] = -1
        out["slot"] = slot.astype(np.int32).reshape(-1)
        out["isp2"] = np.where(used & ~dead[:, None], raw >> 31, 0).astype(np.uint8).reshape(-1)
        return out
