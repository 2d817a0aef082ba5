"""Seeded synthetic inputs for the SGF solver: random streams and PDE matrices.

This package holds no arithmetic of the factorization itself. It builds the
problem ``A x = b`` (a sparse SPD matrix from a PDE discretization on a
Cartesian grid, the grid coordinates, and right-hand sides) that both the CPU
oracle and the GPU library consume.
"""
from .rng import splitmix64_uniform, uniform, normal
from .problems import (
    Problem,
    poisson_fd,
    gaussian_field_fourier,
    blocky_log_field,
    elasticity_q1,
    random_rhs,
    config_problem,
)

__all__ = [
    "splitmix64_uniform", "uniform", "normal", "Problem", "poisson_fd",
    "gaussian_field_fourier", "blocky_log_field", "elasticity_q1",
    "random_rhs", "config_problem",
]
