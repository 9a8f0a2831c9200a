"""FP64 CPU oracle for the face-staggered EPI susceptibility-correction method.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, the smoke check in ``__graft_entry__`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The product path (the HIP
library and its Python binding) never calls it, and this package never imports the
product path. It is a plain, slow, obviously correct transcription of the discretised
method of Macdonald & Ruthotto, "Efficient Numerical Optimization for Susceptibility
Artifact Correction of EPI-MRI" (Sections 3 and 4), in float64 NumPy.

Parity status per function (see the tests under ``tests/test_oracle_*.py`` for the pins):
every function here is pinned by at least one check that does not re-type its formula
(finite differences, dense assembly from the Kronecker definitions, brute-force QP
enumeration, library DCT/solve routines, closed-form special cases, the sparsity patterns
printed in Figure 2, the generator's known field). The ADMM and GN-PCG *trajectories* as a
whole have no independent reference beyond those per-step pins and the stationarity checks.
"""
from .epi_oracle import *  # noqa: F401,F403
from .epi_oracle import __all__  # noqa: F401
