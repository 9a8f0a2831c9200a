"""FP64 CPU oracle for the face-staggered EPI susceptibility-correction method.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, the smoke check in ``__graft_entry__`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The product path (the HIP
library and its Python binding) never calls it, and this package never imports the
product path. It is a plain, slow, obviously correct transcription of the discretised
method of Macdonald & Ruthotto, "Efficient Numerical Optimization for Susceptibility
Artifact Correction of EPI-MRI" (Sections 3 and 4), in float64 NumPy.

Parity status per function (the pins live in ``tests/test_oracle_pins.py`` and
``tests/test_oracle_pins_solvers.py``): every function here is pinned by at least one
check that does not re-type its formula -- finite differences (objective, residual, phi,
and the b-step QP gradient c against the b-subproblem), dense assembly from the Kronecker
definitions (H_D, H_JGN and its Jacobi diagonal, the QP matrix G, P_block), brute-force QP
enumeration, library DCT and solve routines, closed-form special cases, the sparsity
patterns printed in Figure 2, the rho sequences of Figure 7, hand-checked eq. admmStop
tolerances, each test of eq. stopping1 made the binding one, the generator's known field,
and fixed points (ADMM converges to a stationary point of D + alpha S, GN-PCG to one of
J_GN). Parity unpinned: the ADMM and GN-PCG trajectories between the start and the limit
(the iterates of a run as a whole) have no reference other than this oracle.
"""
from .epi_oracle import *  # noqa: F401,F403
from .epi_oracle import __all__  # noqa: F401
