"""MI355X-native multilevel lattice Boltzmann hot path (HIP, gfx950).

Python side of the C ABI in include/mlbm.h: argument marshalling only.
Device memory and streams come from PyTorch; every step of the method runs
in the HIP kernels of lib/libmlbm.so.
"""
from ._lib import (D2Q9, D3Q19, D3Q27, F16S, F32, F64, MLBMError, DIAG_FORCE, DIAG_KE,
                   DIAG_MASS, STATUS_F16_OVERFLOW, STATUS_GRAPH_FALLBACK,
                   STATUS_NONFINITE, lib)
from .api import Plan, Sim, lattice, set_morton_policy, set_gfc_layers
from . import autograd

__all__ = ["Plan", "Sim", "lattice", "set_morton_policy", "set_gfc_layers", "autograd", "MLBMError", "lib", "D2Q9", "D3Q19", "D3Q27",
           "F64", "F32", "F16S", "DIAG_MASS", "DIAG_KE", "DIAG_FORCE",
           "STATUS_NONFINITE", "STATUS_F16_OVERFLOW", "STATUS_GRAPH_FALLBACK"]
