"""Seeded synthetic inputs shared by the HIP library's tests and the CPU oracle."""
from .workloads import (PARAM_NAMES, Workload, WORKLOADS, small_workload, sample_y,
                        sketch_draws, SIGMA2_256, BATCH_SIDES, batched_fields, scattered_points,
                        scattered_sample, OpWorkload, OP_WORKLOADS, AdrWorkload, ADR_WORKLOADS,
                        SelWorkload, SEL_WORKLOADS, BivWorkload, BIV_WORKLOADS, BIV_PARAM_NAMES)

__all__ = ["PARAM_NAMES", "Workload", "WORKLOADS", "small_workload", "sample_y",
           "sketch_draws", "SIGMA2_256", "BATCH_SIDES", "batched_fields", "scattered_points",
           "scattered_sample", "OpWorkload", "OP_WORKLOADS", "AdrWorkload", "ADR_WORKLOADS",
           "SelWorkload", "SEL_WORKLOADS", "BivWorkload", "BIV_WORKLOADS", "BIV_PARAM_NAMES"]
