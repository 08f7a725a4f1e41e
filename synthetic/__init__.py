"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark."""
from .rng import splitmix64, uniform, uniform_stream  # noqa: F401
from .workloads import (S0, NU_230, NU_VLBI, Grid, Camera, make_grid, constant_grid, make_code_grid,  # noqa: F401
                        small_image, production_set, slow_light_set, spectrum_freqs,
                        batch_jobs, mlp_samples, cell_centres, PROD_SPINS, PROD_INCLS)
