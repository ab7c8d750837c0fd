"""MI355X-native Cahn-Hilliard ensemble engine (arXiv:1911.03386 hot path).

The compute path is libch.so (HIP kernels for gfx950 behind the C ABIs in
include/ch.h and include/dp.h); ``ch`` and ``dp`` are their ctypes bindings:
``Ensemble`` for Cahn-Hilliard ensembles, ``DropletEnsemble`` for Model 1
droplet-population ensembles.
"""
from .ch import (CH_ENERGY_PAPER_PRINTED, CH_ENERGY_QUARTER, CH_F32_BULK, CH_F64, ChError,
                 Ensemble, ch_solver_coefficients, ch_workspace_bytes, load, make_desc)
from .dp import DpError, DropletEnsemble

__all__ = ["Ensemble", "ChError", "make_desc", "load", "ch_workspace_bytes",
           "ch_solver_coefficients", "CH_F64", "CH_F32_BULK", "CH_ENERGY_QUARTER",
           "CH_ENERGY_PAPER_PRINTED", "DropletEnsemble", "DpError"]
