"""pprs: prefix-scan registration of micrograph series on MI355X (gfx950).

The work runs in libpprs.so (HIP kernels behind a C ABI, include/pprs.h). This package only
marshals arguments: torch tensors supply device memory and the stream. Importing it does not
load the library; the first call does, and fails loudly if it has not been built.
"""
from .api import (Params, PairStats, SeriesStats, compose_deformations, default_params,
                  kernel_names, kernel_timing, prefix_register_series,
                  prefix_register_series_rigid, register_pair,
                  register_pairs, register_pairs_rigid, register_series_batch, PprsError,
                  scan_plan, scan_program, series_average, series_average_refine, set_kernel_timing, set_pool, get_tuning, set_tuning,
                  set_metric_solve,
                  Context, WarmStartNet, pair_inputs,
                  level7_targets, set_warm_start, workspace_query, reserve_workspace,
                  workspace_bytes, prefix_register_series_batch, register_pair_noalloc, DecisionLog)

__all__ = ["Params", "PairStats", "SeriesStats", "compose_deformations", "default_params",
           "kernel_names", "kernel_timing", "prefix_register_series",
           "prefix_register_series_rigid", "register_pair",
           "register_pairs", "register_pairs_rigid", "register_series_batch", "PprsError",
           "scan_plan", "scan_program", "series_average", "series_average_refine", "set_kernel_timing", "set_pool", "get_tuning", "set_tuning",
           "set_metric_solve", "Context", "WarmStartNet", "pair_inputs",
           "level7_targets", "set_warm_start", "workspace_query", "reserve_workspace",
           "workspace_bytes", "prefix_register_series_batch", "register_pair_noalloc", "DecisionLog"]
