"""Oracle steps taken from a GPU state, with break-decision ties accounted for.

The oracle decides whether a spring breaks in float64 from the float32 state
it is given (thesis Ch.7 "structure": a spring breaks when stretched past its
limit); the kernels decide in float32.  The two may disagree only on a spring
whose float64 strain (mesh springs) or force (structure springs) lies within
float32 rounding of the limit: a tie, where both decisions are correct.

`mesh_step` and `structure_compute_step` run one oracle step, check that
every spring on which the GPU decided differently is such a tie, and then
rerun the step with the GPU's decision fixed for those springs (the oracle
refuses fixed decisions outside the band), so that everything else - the
other springs, every adjacency slot, forces and node states - is compared
with a single valid outcome.  Ties are counted in TIES and reported at the
end of the session.
"""

import numpy as np

from oracle import (STRUCTURE_TIE_REL, spring_steps, spring_steps_deg, spring_tie_band,
                    structure_step)

# springs within the tie band at checked steps, and those the GPU decided
# the other way, summed over the session (the conftest prints them)
TIES = {"checked_spring_steps": 0, "near": 0, "flipped": 0}


def _account(diff, near, what):
    bad = diff & ~near
    assert not bad.any(), "%s: break decision differs from the oracle outside the tie band (springs %s)" % (
        what, np.flatnonzero(bad)[:10].tolist())
    TIES["near"] += int(near.sum())
    TIES["flipped"] += int(diff.sum())


def mesh_step(state, dt, limit, alive, fx, fy, gpu_alive_after, tension_only=False, any_degree=False):
    """One oracle step of the spring mesh from `state` (the GPU's state before
    the step: alive flags and forces passed separately), matched to the GPU's
    break decisions at ties.  Returns (oracle result, near-tie count, flipped)."""
    S = int(np.asarray(state["a"]).size)
    if any_degree:
        run = lambda tie: spring_steps_deg(state, dt, limit, 1, alive=alive, fx=fx, fy=fy, tie=tie)
    else:
        run = lambda tie: spring_steps(state, dt, limit, 1, alive=alive, fx=fx, fy=fy,
                                       tension_only=tension_only, tie=tie)
    ref = run(None)
    live = np.asarray(alive).astype(bool)
    near = live & (np.abs(ref["strain"] - limit) <= spring_tie_band())
    got = np.asarray(gpu_alive_after).astype(bool)
    diff = live & (got != ref["alive"].astype(bool))
    _account(diff, near, "spring mesh")
    TIES["checked_spring_steps"] += 1
    if diff.any():
        tie = np.full(S, -1, np.int8)
        tie[diff] = (~got[diff]).astype(np.int8)
        ref = run(tie)
    return ref, int(near.sum()), int(diff.sum())


def structure_compute_step(state, dt, gpu_salive_after):
    """One oracle compute step of "structure" from `state`, matched to the
    GPU's break decisions at ties (|F - limit| <= STRUCTURE_TIE_REL k (l + L0))."""
    ref = structure_step(state, dt)
    live = np.asarray(state["salive"]).astype(bool)
    p1 = np.asarray(state["p1"])
    p2 = np.asarray(state["p2"])
    x = np.asarray(state["x"], np.float64)
    y = np.asarray(state["y"], np.float64)
    l = np.hypot(x[p2] - x[p1], y[p2] - y[p1])
    k = np.asarray(state["k"], np.float64)
    L0 = np.asarray(state["L0"], np.float64)
    maxf = np.asarray(state["maxf"], np.float64)
    with np.errstate(invalid="ignore"):
        near = live & (np.abs(ref["F"] - maxf) <= STRUCTURE_TIE_REL * k * (l + L0))
    got = np.asarray(gpu_salive_after).astype(bool)
    diff = live & (got != ref["salive"].astype(bool))
    _account(diff, near, "structure")
    TIES["checked_spring_steps"] += 1
    if diff.any():
        tie = np.full(p1.size, -1, np.int8)
        tie[diff] = (~got[diff]).astype(np.int8)
        ref = structure_step(state, dt, tie=tie)
    return ref, int(near.sum()), int(diff.sum())
