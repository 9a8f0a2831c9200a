"""Writes the stored oracle reference of the converged ADMM solve at the benchmark size:
240 x 200 x 110 cells, PE along the first axis (5,302,000 faces), alpha = 50, rho = 1e3,
from b = z = u = 0 to the relative residual 1e-3 (eq. admmStop with eps_abs = 0,
eps_rel = 1e-3). The FP64 oracle needs minutes for it, so the GPU test compares against
this file: the iteration count, both residual histories, the norms of b, z, u, the
objective at b, max|b - z| in voxels over all faces, and b, z, u at 16384 faces drawn
with a fixed seed.

Calls only the oracle and the seeded generator. Run from the repository root:
    python tests/oracle_samples/make_admm_converged.py [seed ...]
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

SHAPE, PE_AXIS, ALPHA, RHO, TOL, MAX_ITER = (240, 200, 110), 0, 50.0, 1e3, 1e-3, 2000
N_SAMPLES = 16384


def path_for(seed: int) -> str:
    return os.path.join(HERE, f"admm_240x200x110_seed{seed}.npz")


def make(seed: int) -> str:
    import oracle as O
    from synth import generate
    v = generate(seed, SHAPE, PE_AXIS)
    P = O.make_problem(v.Ip, v.Im, v.h, ALPHA)
    t0 = time.time()
    b, z, u, rep = O.solve_admm(P, rho=RHO, max_iter=MAX_ITER, eps_abs=0.0, eps_rel=TOL)
    dt = time.time() - t0
    idx = np.sort(np.random.default_rng(1000 + seed).choice(P.n, N_SAMPLES, replace=False))
    flat = lambda a: np.asarray(a).reshape(-1)
    out = path_for(seed)
    np.savez_compressed(
        out, seed=seed, shape=np.array(SHAPE), pe_axis=PE_AXIS, alpha=ALPHA, rho=RHO, tol=TOL,
        iters=rep.iters, converged=int(rep.converged), r_pri=np.array(rep.r_pri),
        r_dual=np.array(rep.r_dual), norms=np.array([np.linalg.norm(flat(x)) for x in (b, z, u)]),
        J=O.objective(P, P.lines(b), False)["J"], bz_max_vox=float(np.abs(b - z).max() * SHAPE[PE_AXIS]),
        idx=idx, b=flat(b)[idx], z=flat(z)[idx],
        u=flat(u)[idx], image_sums=np.array([float(np.sum(v.Ip)), float(np.sum(v.Im))]),
        oracle_seconds=dt)
    print(f"seed {seed}: {rep.iters} iterations, converged {rep.converged}, {dt:.0f} s -> {out}")
    return out


if __name__ == "__main__":
    for s in (sys.argv[1:] or ["3"]):
        make(int(s))
