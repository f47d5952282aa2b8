"""Seeded synthetic inputs (magnetograms, points, lambda) and the Low & Lou exact field.

Shared by the CPU oracle and the GPU path; holds no DBIE arithmetic."""
from .synth import (Boundary, Workload, CONFIGS, config1, config2, config3, config4, config5,
                    z_stratified_subsample, grid_points, to_fp32_once, lowlou_table1)
from .lowlou import LowLou
