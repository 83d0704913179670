"""MI355X (gfx950) implementation of the additive overlapping domain
decomposition method for the Helmholtz equation (Leng & Ju, arXiv 1807.04180).

The compute path is the HIP library libddm.so (C-ABI in include/ddm.h); this
package only marshals arguments (torch tensors give device memory and the
stream).  There is no CPU fallback: if libddm.so is missing, constructing a
solver raises.
"""
from ._ffi import (DDM_FGMRES, DDM_FP64, DDM_MIXED, DDM_STATIONARY, LIB_PATH,  # noqa: F401
                   LibraryMissing, header_functions, lib)
from .solver import DDMError, HelmholtzDDM, Problem  # noqa: F401

__all__ = ["HelmholtzDDM", "Problem", "DDMError", "lib", "LIB_PATH", "DDM_FP64", "DDM_MIXED",
           "DDM_STATIONARY", "DDM_FGMRES"]
