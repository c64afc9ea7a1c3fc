"""Differentiable spring mesh: reverse mode through the spring-mesh step.

``DiffSpringSim`` runs the forward steps (breaking off) with (x, v)
checkpoints every ``every`` steps and, given dL/dx_T, the reverse sweep:
each segment is recomputed from its checkpoint by the forward step whose
node pass (``adjoint.step_node``) also writes the new positions to a tape,
then reversed step by step with the ``adjoint.node`` / ``adjoint.spring``
methods (the segment's first step reads its positions from the
checkpoint).  All of it runs in libsmmo;
this module only orders the calls.

``SpringRollout`` wraps it as a ``torch.autograd.Function`` of the spring
stiffnesses and the initial velocities.
"""

import math

import numpy as np

from . import smmo
from .sims import SPRING_CLASSES

ADJ_CLASSES = {
    "Node": SPRING_CLASSES["Node"] + [("lx", "f32", 1), ("ly", "f32", 1), ("lvx", "f32", 1),
                                      ("lvy", "f32", 1), ("wx", "f32", 1), ("wy", "f32", 1)],
    "Spring": SPRING_CLASSES["Spring"] + [("cx", "f32", 1), ("cy", "f32", 1), ("gk", "f32", 1)],
}


def _blocks(n: int) -> int:
    return (n + 63) // 64


class DiffSpringSim:
    """Spring mesh with fixed topology and a reverse sweep.

    mesh: arrays as made by ``inputs.spring_mesh`` (ids local to the arrays);
    k, vx, vy may be overridden by torch tensors (device) or arrays.
    """

    def __init__(self, mesh: dict, dt: float, steps: int, every: int = 20, k=None, vx=None, vy=None,
                 cfg=None):
        import torch

        self.torch = torch
        N = int(np.asarray(mesh["x"]).size)
        S = int(np.asarray(mesh["a"]).size)
        self.N, self.S = N, S
        self.dt, self.T, self.every = float(dt), int(steps), max(1, int(every))
        self.heap = smmo.Heap(ADJ_CLASSES, blocks=_blocks(N) + _blocks(S) + 8, cfg=cfg)
        dev = self.heap.dev
        self.dev = dev

        def f32(a):
            if isinstance(a, torch.Tensor):
                return a.detach().to(device=dev, dtype=torch.float32).contiguous()
            return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)

        def i32(a):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to(dev)

        null_adj = torch.full((N * 8,), -1, dtype=torch.int32, device=dev)
        self.node_h = self.heap.new("Node", N, x=f32(mesh["x"]), y=f32(mesh["y"]),
                                    vx=f32(mesh["vx"] if vx is None else vx),
                                    vy=f32(mesh["vy"] if vy is None else vy), m=f32(mesh["m"]),
                                    adj=null_adj, id=torch.arange(N, dtype=torch.int32, device=dev)).clone()
        a_idx = i32(mesh["a"]).long()
        b_idx = i32(mesh["b"]).long()
        if S:
            self.spring_h = self.heap.new(
                "Spring", S, a=self.node_h[a_idx], b=self.node_h[b_idx],
                k=f32(mesh["k"] if k is None else k), L0=f32(mesh["L0"]),
                slot_a=torch.from_numpy(np.asarray(mesh["slot_a"]).astype(np.uint8)).to(dev),
                slot_b=torch.from_numpy(np.asarray(mesh["slot_b"]).astype(np.uint8)).to(dev),
                id=torch.arange(S, dtype=torch.int32, device=dev)).clone()
        self.cn, self.cs = self.heap.cls["Node"], self.heap.cls["Spring"]
        self.fargs = smmo.smmo_spring_args(self.cn, self.cs, self.dt, math.inf)
        ids = {n: smmo.smmo_method_id(n) for n in (
            "spring.force", "spring.link", "adjoint.record", "adjoint.save", "adjoint.load",
            "adjoint.seed", "adjoint.zero", "adjoint.node", "adjoint.spring", "adjoint.step_node")}
        self.mid = ids
        if S:
            self._do(self.cs, "spring.link", self.fargs)
        # tapes: one float per handle and plane
        self.plane = 64 * self.heap.blocks
        nck = (self.T + self.every - 1) // self.every if self.T else 0
        self.ckpt = torch.empty(max(1, nck) * 4 * self.plane, dtype=torch.float32, device=dev)
        seg = max(1, min(self.every, max(self.T, 1)))
        # two tapes when there are several segments: the reverse steps of one
        # segment read one while the next segment is recomputed into the other
        self.tapes = [torch.empty(seg * 2 * self.plane, dtype=torch.float32, device=dev)
                      for _ in range(2 if nck > 1 else 1)]
        self.tape = self.tapes[0]
        self.overlap = nck > 1
        self._side = torch.cuda.Stream(device=dev) if self.overlap else None
        self._main = torch.cuda.Stream(device=dev) if self.overlap else None
        # events of the overlapped sweep, kept for the sim's life (a captured
        # graph refers to them): fork, recompute of segment s done, reverse
        # steps of segment s done
        self._ev_fork = torch.cuda.Event() if self.overlap else None
        self._ev_rec = [torch.cuda.Event() for _ in range(nck)] if self.overlap else []
        self._ev_rev = [torch.cuda.Event() for _ in range(nck)] if self.overlap else []
        # every launch of forward and backward, bound once (the seed launch
        # names the caller's tensors and is bound per backward call)
        B = smmo.BoundLaunch
        hp = self.heap.h
        self.L_force = B(hp, self.cs, ids["spring.force"], self.fargs) if S else None
        # the forward node pass: the same kernel as the recompute's, without a tape
        self.L_node = B(hp, self.cn, ids["adjoint.step_node"], self._aargs(None))
        self.L_save = [B(hp, self.cn, ids["adjoint.save"], self._aargs(self.ckpt, slot=c)) for c in range(nck)]
        self.L_load = [B(hp, self.cn, ids["adjoint.load"], self._aargs(self.ckpt, slot=c)) for c in range(nck)]
        # recompute: step t of a segment writes the positions of step t + 1 to
        # tape slot t + 1; the spring pass of step 0 reads the checkpoint's
        # (x, y), its planes 4c, 4c + 1 being plane pair 2c of that tape
        self.L_stepr = [[B(hp, self.cn, ids["adjoint.step_node"], self._aargs(tp, slot=t)) for t in range(seg)]
                        for tp in self.tapes]
        self.L_anode = {m: B(hp, self.cn, ids["adjoint.node"], self._aargs(self.tape, mode=m)) for m in (1, 2, 3)}
        self.L_aspring = [[B(hp, self.cs, ids["adjoint.spring"], self._aargs(tp, slot=t)) for t in range(seg)]
                          for tp in self.tapes] if S else None
        self.L_aspring0 = [B(hp, self.cs, ids["adjoint.spring"], self._aargs(self.ckpt, slot=2 * c))
                           for c in range(nck)] if S else None
        self.L_zero = B(hp, self.cs, ids["adjoint.zero"], self._aargs(self.tape)) if S else None

    # ------------------------------------------------------------ helpers --
    def _do(self, cls, name, args):
        smmo.smmo_parallel_do(self.heap.h, cls, self.mid[name], args)

    def _aargs(self, tape, slot=0, mode=0, seeds=(None, None, None, None), count=0):
        P = [0 if s is None else s.data_ptr() for s in seeds]
        tp, tn = (None, 0) if tape is None else (tape.data_ptr(), tape.numel())
        return smmo.smmo_adjoint_args(self.cn, self.cs, self.dt, mode, tp, tn,
                                      self.plane, slot, count, P[0] or None, P[1] or None,
                                      P[2] or None, P[3] or None)

    def _stream(self):
        return self.torch.cuda.current_stream().cuda_stream

    def step(self, stream=None):
        st = self._stream() if stream is None else stream
        if self.L_force is not None:
            self.L_force(st)
        self.L_node(st)

    # ------------------------------------------------------------ forward --
    def forward(self):
        """T steps; checkpoints at 0, every, 2 every, ...  Returns x_T as (N, 2) by node id."""
        self.run_forward()
        return self.positions()

    def restart(self, stream=None):
        """Restores positions and velocities saved at step 0 by the last
        forward run, so that forward and backward can run again (for
        instance replayed from a captured HIP graph)."""
        if not self.L_save:
            return
        self.L_load[0](self._stream() if stream is None else stream)

    def run_forward(self, stream=None):
        """The T forward steps with their checkpoints, launched on `stream`
        (default: the current stream); no host synchronization."""
        st = self._stream() if stream is None else stream
        for n in range(self.T):
            if n % self.every == 0:
                self.L_save[n // self.every](st)
            self.step(st)

    def positions(self):
        torch = self.torch
        g = self.heap.gather("Node", ["id", "x", "y"])
        out = torch.empty((self.N, 2), dtype=torch.float32, device=self.dev)
        idx = g["id"].long()
        out[idx, 0] = g["x"]
        out[idx, 1] = g["y"]
        return out

    # ----------------------------------------------------------- backward --
    def backward(self, gx, gy, gvx=None, gvy=None):
        """Reverse sweep from dL/dx_T (and dL/dv_T, default 0), tensors of N by
        node id.  Returns (dL/dk by spring id, dL/dv0 (N, 2), dL/dx0 (N, 2))."""
        torch = self.torch
        if self.overlap and not self._stream():
            # on the legacy null stream the sweep goes to a created stream
            # between two host synchronizations, so that only events of
            # created streams order its two streams
            torch.cuda.current_stream().synchronize()
            with torch.cuda.stream(self._main):
                self.run_backward(gx, gy, gvx, gvy)
                self.heap.sync()
        else:
            self.run_backward(gx, gy, gvx, gvy)
            self.heap.sync()
        return self.gradients()

    def _recompute(self, seg):
        """Launches recomputing segment seg from its checkpoint into tape seg % 2."""
        n0 = seg * self.every
        n1 = min(n0 + self.every, self.T)
        out = [self.L_load[seg]]
        for t in range(n1 - n0 - 1):      # the segment's last step is not needed
            if self.L_force is not None:
                out.append(self.L_force)
            out.append(self.L_stepr[seg % 2][t + 1])
        return out

    def _reverse(self, seg, first):
        """Launches of segment seg's reverse steps, last step first, reading
        tape seg % 2 (step 0: the checkpoint)."""
        n0 = seg * self.every
        n1 = min(n0 + self.every, self.T)
        out = []
        for t in range(n1 - n0 - 1, -1, -1):
            out.append(self.L_anode[2 if first else 3])
            first = False
            if self.L_aspring is not None:
                out.append(self.L_aspring[seg % 2][t] if t else self.L_aspring0[seg])
        return out

    def run_backward(self, gx, gy, gvx=None, gvy=None, stream=None, overlap=None):
        """The reverse sweep's launches on `stream` (default: the current
        stream); no host synchronization.  The seed tensors must stay alive
        until the sweep has run.

        With overlap (the default when there are several segments) each
        segment but the last is recomputed on a second stream while the
        segment after it is reversed on `stream`: the recompute writes x, v,
        the springs' forces and its own tape, the reverse steps the adjoint
        fields, and events order each tape's reuse.  The second stream forks
        from `stream` and joins it again, so the sweep can be captured in a
        HIP graph like the single-stream one, and the results are the same
        bit for bit.  The ordering needs a created stream: on the legacy null
        stream (torch's default) the sweep runs on that stream alone.  One
        sweep of a sim at a time: its tapes, heap and events are shared."""
        torch = self.torch
        st = self._stream() if stream is None else stream
        seeds = [t.detach().to(device=self.dev, dtype=torch.float32).contiguous() if t is not None else None
                 for t in (gx, gy, gvx, gvy)]
        self._seeds = seeds
        smmo.BoundLaunch(self.heap.h, self.cn, self.mid["adjoint.seed"],
                         self._aargs(self.tape, seeds=seeds, count=self.N))(st)
        if self.L_zero is not None:
            self.L_zero(st)
        nseg = (self.T + self.every - 1) // self.every
        if overlap is None:
            overlap = self.overlap
        if not (overlap and self.overlap) or not st:
            for seg in range(nseg - 1, -1, -1):
                for launch in self._recompute(seg) + self._reverse(seg, seg == nseg - 1):
                    launch(st)
        else:
            A = torch.cuda.ExternalStream(st, device=self.dev)
            side = self._side
            sst = side.cuda_stream
            self._ev_fork.record(A)       # the forward run and the seeds come first
            side.wait_event(self._ev_fork)
            for launch in self._recompute(nseg - 1):
                launch(sst)
            self._ev_rec[nseg - 1].record(side)
            for seg in range(nseg - 1, -1, -1):
                A.wait_event(self._ev_rec[seg])       # tape seg % 2 holds segment seg
                rev, rec = self._reverse(seg, seg == nseg - 1), []
                if seg > 0:
                    if seg + 1 < nseg:    # the reverse of seg + 1 is done with tape (seg - 1) % 2
                        side.wait_event(self._ev_rev[seg + 1])
                    rec = self._recompute(seg - 1)
                for i in range(max(len(rev), len(rec))):
                    if i < len(rev):
                        rev[i](st)
                    if i < len(rec):
                        rec[i](sst)
                self._ev_rev[seg].record(A)
                if seg > 0:
                    self._ev_rec[seg - 1].record(side)
        if nseg:
            self.L_anode[1](st)

    def gradients(self):
        torch = self.torch
        gk = torch.zeros(self.S, dtype=torch.float32, device=self.dev)
        if self.S:
            g = self.heap.gather("Spring", ["id", "gk"])
            gk[g["id"].long()] = g["gk"]
        g = self.heap.gather("Node", ["id", "lvx", "lvy", "lx", "ly"])
        idx = g["id"].long()
        gv = torch.empty((self.N, 2), dtype=torch.float32, device=self.dev)
        gx = torch.empty((self.N, 2), dtype=torch.float32, device=self.dev)
        gv[idx, 0], gv[idx, 1] = g["lvx"], g["lvy"]
        gx[idx, 0], gx[idx, 1] = g["lx"], g["ly"]
        return gk, gv, gx


def _autograd_function():
    import torch

    class SpringRollout(torch.autograd.Function):
        """x_T = rollout(k, v0): T spring-mesh steps from the mesh's initial
        positions with stiffnesses k (S,) and initial velocities v0 (N, 2);
        the backward runs the checkpointed reverse sweep on the GPU."""

        @staticmethod
        def forward(ctx, k, v0, mesh, dt, steps, every=20):
            sim = DiffSpringSim(mesh, dt, steps, every, k=k, vx=v0[:, 0], vy=v0[:, 1])
            xT = sim.forward()
            ctx.sim = sim
            return xT

        @staticmethod
        def backward(ctx, g):
            sim = ctx.sim
            gk, gv, _ = sim.backward(g[:, 0], g[:, 1])
            sim.heap.close()
            ctx.sim = None
            return gk, gv, None, None, None, None

    return SpringRollout


_SR = None


def spring_rollout(k, v0, mesh, dt, steps, every=20):
    """Differentiable rollout: returns x_T (N, 2); gradients flow to k and v0."""
    global _SR
    if _SR is None:
        _SR = _autograd_function()
    return _SR.apply(k, v0, mesh, dt, steps, every)
