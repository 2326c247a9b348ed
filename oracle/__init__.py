"""Plain FP64 CPU oracle for independent electron surface hopping (IESH).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, calls or links this package; only the tests,
the smoke check and the CPU-baseline leg of the benchmark do.  It shares no
code with the HIP path: the two meet only through the seeded inputs of the
``workloads`` package.

The oracle is written for clarity, not speed: dense Hamiltonians, LAPACK
``eigh`` for every diagonalisation, explicit inverses/solves, Python loops
over trajectories.  Each module cites the part of the paper (Gardner et al.,
"Efficient implementation and performance analysis of the independent
electron surface hopping method for dynamics at metal surfaces") it follows.

Readings of passages that are silent, garbled or inconsistent are listed in
the module docstrings where they are applied.

Parity unpinned: the hole-impurity population estimator of the paper's
double-well study (it defers to another reference without giving the
formula); the oracle reports two plain estimators instead (see
``dynamics.observables``).
"""
from . import bath, models, electronic, dynamics, rng  # noqa: F401
