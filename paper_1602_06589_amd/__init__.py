"""MI355X-native generation of the FLAPW muffin-tin Hamiltonian and overlap matrices.

The computation lives in the HIP library ``libflapw_hip.so`` (C-ABI in include/flapw.h);
``flapw`` is its Python binding.
"""
from .flapw import FP64, SPLIT_BF16, SPLIT_FP32, SPLIT_I8, SPLIT_I8_MOD, Flapw, FlapwError, Plan, hermitian_full, load_library  # noqa: F401

__all__ = ["Flapw", "FlapwError", "Plan", "hermitian_full", "load_library", "FP64", "SPLIT_BF16", "SPLIT_FP32", "SPLIT_I8",
           "SPLIT_I8_MOD"]
