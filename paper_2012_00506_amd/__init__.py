"""MI355X-native banded FEAST spectrum slicing (the spectrum-slicing stage of
PDESHEP, arXiv 2012.00506).

The compute path is the HIP library ``libfeastband.so`` (C ABI in
``include/feastband.h``); this package is its Python binding.  Importing the
binding raises if the library has not been built: there is no CPU fallback.
"""
from .api import (DeviceBand, FeastFilter, FilterResult, SliceResult, SolveResult, band_inertia,
                  contour_nodes,
                  band_shifted_solve, colmajor, rayleigh_ritz, RitzResult, device_info, feast_band_slice, feast_filter,
                  profile_enable, profile_read, slice_plan, slice_plan_prev, slice_certify, m0_rule, to_colmajor,
                  autotune, tune_load,
                  band_features, cheb_moments, planner_bytes, planner_forward,
                  planner_train_step)

__all__ = ["DeviceBand", "FeastFilter", "FilterResult", "SliceResult", "SolveResult", "contour_nodes",
           "band_inertia", "band_shifted_solve", "colmajor", "device_info", "feast_band_slice",
           "feast_filter", "rayleigh_ritz", "RitzResult", "profile_enable", "profile_read", "slice_plan", "slice_plan_prev", "slice_certify", "m0_rule",
           "to_colmajor",
           "autotune", "tune_load", "band_features", "cheb_moments", "planner_bytes",
           "planner_forward", "planner_train_step"]
