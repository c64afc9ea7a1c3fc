"""CPU oracle of SMMO execution.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or runs it.
"""

from .oracle import (  # noqa: F401
    set_threads,
    threads,
    build,
    GolWorld,
    WatorWorld,
    nbody_steps,
    nbody_force_at,
    nbody_update,
    spring_steps,
    spring_adjoint,
    spring_adjoint_step,
    spring_breaks,
    spring_tie_band,
    spring_steps_deg,
    structure_pull,
    structure_step,
    STRUCTURE_TIE_REL,
    structure_bfs,
    STRUCTURE_ANCHOR,
    STRUCTURE_PULL,
    STRUCTURE_NODE,
    STRUCTURE_MAXDIST,
    generation_steps,
    BURST_SURVIVE,
    BURST_BIRTH,
    BURST_DYING,
)
