"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package builds particle sets only: lattices, Gaussian random displacement
fields and the Zel'dovich-approximation initial conditions built from them.
It holds none of the particle-mesh step's arithmetic (no deposit, no metric
solve, no particle update), and it imports neither the oracle nor the HIP
library.
"""
from .ics import (  # noqa: F401
    CONFIGS,
    eds_a_of_tau,
    eds_tau_of_a,
    gaussian_displacement,
    lattice_positions,
    plane_wave_particles,
    spectrum_power_law_m2,
    spectrum_k_transfer,
    zeldovich_particles,
    config_particles,
)
