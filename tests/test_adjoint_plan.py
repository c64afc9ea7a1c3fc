"""Host logic of the checkpointed reverse sweep (no GPU): the launches that
recompute a segment and reverse it.  Launch objects are replaced by
recorders, so the plan is checked without a heap."""

import pytest

from paper_1908_05845_amd.adjoint import DiffSpringSim


class Rec:
    def __init__(self, log, *name):
        self.log, self.name = log, name

    def __call__(self, stream):
        self.log.append(self.name)


def plan_sim(T, every, springs=True):
    log = []
    sim = DiffSpringSim.__new__(DiffSpringSim)
    sim.T, sim.every = T, every
    nck = (T + every - 1) // every
    seg = max(1, min(every, T))
    sim.L_load = [Rec(log, "load", c) for c in range(nck)]
    sim.L_force = Rec(log, "force") if springs else None
    sim.L_stepr = [[Rec(log, "step", b, t) for t in range(seg)] for b in range(2)]
    sim.L_anode = {m: Rec(log, "anode", m) for m in (1, 2, 3)}
    sim.L_aspring = [[Rec(log, "aspring", b, t) for t in range(seg)] for b in range(2)] if springs else None
    sim.L_aspring0 = [Rec(log, "aspring_ckpt", c) for c in range(nck)] if springs else None
    return sim, log, nck


@pytest.mark.parametrize("T,every", [(200, 20), (60, 7), (41, 20), (5, 20), (20, 1), (1, 1), (21, 20)])
def test_segment_plans(T, every):
    sim, log, nseg = plan_sim(T, every)
    written = {}
    first = True
    for s in range(nseg - 1, -1, -1):
        n0, n1 = s * every, min(s * every + every, T)
        L = n1 - n0
        log.clear()
        for launch in sim._recompute(s):
            launch(None)
        # load of the segment's checkpoint, then L - 1 forward steps, each
        # writing the positions of step t + 1 to slot t + 1 of tape s % 2
        assert log[0] == ("load", s)
        steps = [e for e in log if e[0] == "step"]
        assert steps == [("step", s % 2, t + 1) for t in range(L - 1)]
        assert sum(e == ("force",) for e in log) == L - 1
        written[s % 2] = {t for _, _, t in steps}
        log.clear()
        for launch in sim._reverse(s, first):
            launch(None)
        nodes = [e for e in log if e[0] == "anode"]
        springs = [e for e in log if e[0] in ("aspring", "aspring_ckpt")]
        assert len(nodes) == L and len(springs) == L
        # mode 2 (no spring terms yet) only on the sweep's very first step
        assert nodes[0] == ("anode", 2 if first else 3) and all(n == ("anode", 3) for n in nodes[1:])
        # reverse order; step 0 reads the checkpoint, the others the tape the
        # recompute of this segment wrote
        assert springs[-1] == ("aspring_ckpt", s)
        reads = [e for e in springs if e[0] == "aspring"]
        assert reads == [("aspring", s % 2, t) for t in range(L - 1, 0, -1)]
        assert {t for _, _, t in reads} == written[s % 2]
        first = False


def test_without_springs():
    sim, log, nseg = plan_sim(30, 10, springs=False)
    for launch in sim._recompute(2) + sim._reverse(2, True):
        launch(None)
    assert ("force",) not in log and not any(e[0].startswith("aspring") for e in log)
    assert sum(e[0] == "anode" for e in log) == 10
