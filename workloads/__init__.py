"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This package holds only workload descriptions (model constants, sizes, seeds)
and seeded random draws.  It contains none of the method's arithmetic: no
Hamiltonian, no eigen-solve, no propagation, no hopping.  Both the CPU oracle
(``oracle/``) and the HIP library consume its outputs as plain arrays.
"""
from .configs import CONFIGS, get_config  # noqa: F401
from .sampling import boltzmann_harmonic, scattering_initial, fixed_paths, uniforms  # noqa: F401
