"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This package holds only random-number generation and the construction of
initial states (grids, meshes, particle clouds).  It contains none of the
simulation arithmetic: no force laws, no update rules, no cellular-automaton
rule.  Both the CPU oracle and the HIP path receive the arrays built here.
"""

from .rng import BASE_SEED, config_seed, splitmix64_mix, uniform, normal  # noqa: F401
from .workloads import (  # noqa: F401
    gol_init,
    nbody_init,
    spring_mesh,
    batched_meshes,
    concat_meshes,
    wator_init,
    structure_mesh,
    hub_mesh,
)
