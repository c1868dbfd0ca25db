"""Seeded synthetic micrograph series (blob lattices with drift, smooth warps and Poisson noise).

This module only produces inputs and their analytic ground truth. It holds none of the
registration arithmetic, so both the FP64 oracle and the GPU path can draw from it.
"""
from .blobs import (SeriesSpec, make_series, ground_truth, ground_truth_pair, CONFIGS,
                    config_spec)

__all__ = ["SeriesSpec", "make_series", "ground_truth", "ground_truth_pair", "CONFIGS",
           "config_spec"]
