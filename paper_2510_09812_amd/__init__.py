"""MI355X (gfx950) library for the hot path of the Gauss-Seidel projection
method time step of finite-element micromagnetics with magnetostriction.

The numerical work lives in libgspm.so (HIP kernels behind the C ABI of
include/gspm.h); `gspm` is its argument-marshalling binding.
"""
from . import gspm
from .gspm import GspmError, Simulation

__all__ = ["gspm", "GspmError", "Simulation"]
