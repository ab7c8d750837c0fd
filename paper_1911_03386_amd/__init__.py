"""MI355X-native Cahn-Hilliard ensemble engine (arXiv:1911.03386 hot path).

The compute path is libch.so (HIP kernels for gfx950 behind the C ABI in
include/ch.h); ``ch`` is its ctypes binding.
"""
from .ch import (CH_ENERGY_PAPER_PRINTED, CH_ENERGY_QUARTER, CH_F32_BULK, CH_F64, ChError,
                 Ensemble, ch_solver_coefficients, ch_workspace_bytes, load, make_desc)

__all__ = ["Ensemble", "ChError", "make_desc", "load", "ch_workspace_bytes",
           "ch_solver_coefficients", "CH_F64", "CH_F32_BULK", "CH_ENERGY_QUARTER",
           "CH_ENERGY_PAPER_PRINTED"]
