"""Seeded synthetic inputs shared by the HIP library's tests and the CPU oracle."""
from .workloads import (PARAM_NAMES, Workload, WORKLOADS, small_workload, sample_y,
                        sketch_draws, SIGMA2_256)

__all__ = ["PARAM_NAMES", "Workload", "WORKLOADS", "small_workload", "sample_y",
           "sketch_draws", "SIGMA2_256"]
