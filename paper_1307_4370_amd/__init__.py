"""MI355X (gfx950) implementation of the SDMM radio-interferometric imaging hot
path of arXiv:1307.4370: the measurement operator Phi = G F D Z and its
adjoint, the SARA dictionary Psi (Dirac + Db1..Db8), the proximal steps and the
conjugate-gradient x-update of SDMM (Algorithm 1).

All computation runs in the HIP library libriop.so (C interface in
include/riop.h); this package only binds it.
"""
from ._lib import (FULL_MASK, Batch, Plan, RiopError, autotune_tile, device_bytes, lib, noise_bound,  # noqa: F401
                   version)

__all__ = ["Plan", "Batch", "RiopError", "autotune_tile", "device_bytes", "lib", "noise_bound", "version",
           "FULL_MASK"]
