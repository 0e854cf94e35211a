"""MI355X (gfx950) implementation of the fused time step of the REV-scale
double-distribution-function MRT lattice Boltzmann model for convection in
porous media (Liu & He, arXiv:1611.03329): HIP kernels behind a C ABI
(include/lbm.h), bound here with ctypes.  Importing the package loads the
built library and raises if it is missing."""
from .lbm import (FP16_STORAGE, Batch, FP32, FP64, LBMError, Lattice, UnstableError, library, make_params,
                  required_bytes)

__all__ = ["Batch", "Lattice", "LBMError", "UnstableError", "FP16_STORAGE", "FP32", "FP64", "library", "make_params",
           "required_bytes"]
