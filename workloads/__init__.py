"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This package holds only workload descriptions (model constants, sizes, seeds)
and seeded random draws, plus the input matrices H0, H1 of the dense model
kind (H(x) = H0 + x H1, data a caller hands to the library).  It contains none
of the method's arithmetic: no eigen-solve, no couplings, no propagation, no
hopping.  Both the CPU oracle (``oracle/``) and the HIP library consume its
outputs as plain arrays.
"""
from .configs import CONFIGS, dense_matrices, get_config  # noqa: F401
from .sampling import boltzmann_harmonic, scattering_initial, fixed_paths, uniforms  # noqa: F401
