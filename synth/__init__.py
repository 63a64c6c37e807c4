"""Seeded synthetic inputs (media k^2 and sources f) shared by the CPU oracle, the tests and the bench.

This package samples input fields only. It holds none of the solver's arithmetic: no difference operators,
no right-hand-side modification, no preconditioner and no Krylov step.
"""
from .media import (  # noqa: F401
    halo_coords,
    gaussian_source,
    inclusions_k2,
    filtered_noise_k2,
    unit_directions,
    plane_wave_sources,
    uneven_problem_set,
    warmstart_problem,
    staggered_coords,
    single_inclusion_problem,
    paper_test_problem,
    workload,
)
