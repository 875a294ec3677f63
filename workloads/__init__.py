"""Seeded synthetic inputs shared by the GPU path and by the oracle.

This package holds only input generation: uniform streams, parameter draws
and the quiet-start particle loading that turns them into initial particle
states.  It contains none of the time-stepping arithmetic of the method.
"""
from .configs import WORKLOADS, workload
from .ensembles import (
    philox_uniforms,
    hammersley_uniforms,
    draw_parameters,
    load_particles,
    make_ensemble,
    parameter_matrix,
    particle_uniforms,
)

__all__ = [
    "WORKLOADS",
    "workload",
    "philox_uniforms",
    "hammersley_uniforms",
    "draw_parameters",
    "load_particles",
    "make_ensemble",
    "parameter_matrix",
    "particle_uniforms",
]
