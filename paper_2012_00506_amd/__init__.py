"""MI355X-native banded FEAST spectrum slicing (the spectrum-slicing stage of
PDESHEP, arXiv 2012.00506).

The compute path is the HIP library ``libfeastband.so`` (C ABI in
``include/feastband.h``); this package is its Python binding.  Importing the
binding raises if the library has not been built: there is no CPU fallback.
"""
from .api import (DeviceBand, SliceResult, SolveResult, band_inertia, band_shifted_solve,
                  colmajor, feast_band_slice, slice_plan,
                  device_info, to_colmajor)

__all__ = ["DeviceBand", "SliceResult", "feast_band_slice", "slice_plan", "SolveResult", "band_inertia", "band_shifted_solve", "colmajor",
           "device_info", "to_colmajor"]
