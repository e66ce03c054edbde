"""MI355X-native treecode boundary-element Poisson-Boltzmann solver.

The work runs in libpbt.so (HIP kernels for gfx950 behind the C ABI of
include/pbt.h); ``pbt`` is its ctypes binding and ``build`` compiles it.
"""
from .pbt import (CAVITY, CHARGED, FP64, MIXED, MOLECULE, POTENTIAL, STERN, PbtError, Result, Solver,
                  from_problem, lib, quadrature_rule)

__all__ = ["Solver", "from_problem", "lib", "quadrature_rule", "PbtError", "Result",
           "MOLECULE", "CHARGED", "POTENTIAL", "STERN", "CAVITY", "FP64", "MIXED"]
