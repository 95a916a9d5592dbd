"""Seeded synthetic inputs shared by the FP64 oracle, the tests and the benchmark.

This package holds problem descriptions and input generators only: sample
refractive-index volumes, incident fields and output grids. It contains none of
the coupled-wave arithmetic, so the oracle and the HIP library can both draw
their inputs from it without sharing any of the method's code.
"""
from .problem import Problem, Grid, PlaneWave
from .generators import (
    sphere_sample,
    smoothed_field,
    random_index_sample,
    focused_pupil_image,
    lorentzian_kappa,
)
from .configs import (
    sphere_config,
    random_field_config,
    spectral_sweep_jobs,
    sweep_problem,
    surrogate_patch,
    surrogate_problem,
    SURROGATE_SEED0,
    CONFIG_NAMES,
)

__all__ = [
    "Problem", "Grid", "PlaneWave",
    "sphere_sample", "smoothed_field", "random_index_sample",
    "focused_pupil_image", "lorentzian_kappa",
    "sphere_config", "random_field_config", "spectral_sweep_jobs", "sweep_problem", "surrogate_patch", "surrogate_problem",
    "SURROGATE_SEED0", "CONFIG_NAMES",
]
