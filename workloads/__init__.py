"""Seeded synthetic workloads for the space-time inverse source problem.

This package only draws inputs: coefficient fields, moving Gaussian sources,
sensor sets and noisy observation data.  It holds none of the space-time KKT
arithmetic (no finite-element matrices, no KKT rows, no Schwarz or Krylov
code); both the CPU oracle and the GPU library receive what it produces.
Observation data come from an independent finite-volume forward solve of the
convection-diffusion model (eq. (1) of the paper), standing in for the paper's
separate fine-mesh data generation (Section 4, data generation paragraph).
"""
from .generate import (Problem, SolverConfig, make_problem, config, CONFIGS,
                       sensor_lattice, batch_instances)

__all__ = ["Problem", "SolverConfig", "make_problem", "config", "CONFIGS",
           "sensor_lattice", "batch_instances"]
