"""MI355X ensemble engine for independent electron surface hopping (IESH).

The hot path (eigen-solve, couplings and forces, orbital propagation, hop
probabilities, hop, rescaling, velocity Verlet) runs in the HIP library
libiesh.so behind the C ABI of include/iesh.h; this package only marshals
arguments (``_lib``) and builds ensembles from workload descriptions
(``ensemble``).
"""
from ._lib import Ensemble, IeshError, bath, discretize, eigh_batched, model_desc, lib  # noqa: F401
from .ensemble import bath_levels, from_config, pack_states, unpack_C  # noqa: F401
