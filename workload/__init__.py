"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and evaluates the analytic problem data
(mesh vertex positions, load functions, target fields, noise). It holds none of
the discretisation or solver arithmetic: no quadrature, no operators, no
multigrid. Every generator uses numpy's PCG64 with an explicit seed.
"""
from .gen import (  # noqa: F401
    box_vertices,
    deformed_box,
    batched_box,
    manufactured_load,
    manufactured_solution,
    uniform_noise,
    fd_rhs,
    batched_specs,
    target_field,
    target_coeffs,
    gaussian_directions,
    BoxSpec,
    box_as_mesh,
    shuffled_mesh,
    face_flags,
)
