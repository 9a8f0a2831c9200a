"""Writes the stored oracle reference of the GN-PCG run of the 128 x 128 x 64 workload
(PE along the second axis, 1,056,768 faces, alpha = 50, beta = 10, gamma = 1e-3): 30
inexact Gauss-Newton steps from b = 0 with the block-Jacobi preconditioner (eta = 0.1, at
most 30 PCG iterations per step, Armijo line search), without the stopping tests. The FP64
oracle needs about two minutes for it, so the GPU test compares against this file: the J
history, the PCG iteration counts and relative residuals, the gradient norms, and the
field at 16384 faces drawn with a fixed seed (plus its norm).

Calls only the oracle and the seeded generator. Run from the repository root:
    python tests/oracle_samples/make_gnpcg_trajectory.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

NAME, SEED, ITERS, N_SAMPLES = "3d_128x128x64", 0, 30, 16384
PATH = os.path.join(HERE, "gnpcg_128x128x64_seed0.npz")


def make() -> str:
    import oracle as O
    from synth import config_volume, CONFIGS
    c = CONFIGS[NAME]
    v = config_volume(NAME, SEED)
    P = O.make_problem(v.Ip, v.Im, v.h, c["alpha"], c["beta"])
    t0 = time.time()
    b, rep = O.solve_gnpcg(P, max_iter=ITERS, use_stopping=False)
    dt = time.time() - t0
    flat = np.asarray(b).reshape(-1)
    idx = np.sort(np.random.default_rng(2000 + SEED).choice(P.n, N_SAMPLES, replace=False))
    np.savez_compressed(
        PATH, name=NAME, seed=SEED, iters=rep.iters, J=np.array(rep.J),
        grad_norm=np.array(rep.grad_norm), pcg_iters=np.array(rep.pcg_iters),
        pcg_relres=np.array(rep.pcg_relres), idx=idx, b=flat[idx],
        b_norm=float(np.linalg.norm(flat)),
        image_sums=np.array([float(np.sum(v.Ip)), float(np.sum(v.Im))]), oracle_seconds=dt)
    print(f"{rep.iters} GN steps, {sum(rep.pcg_iters)} PCG iterations, {dt:.0f} s -> {PATH}")
    return PATH


if __name__ == "__main__":
    make()
