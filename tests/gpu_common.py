"""Helpers shared by the GPU parity tests (inputs, tolerances)."""
import numpy as np

# Tolerances of the GPU path against the FP64 oracle.
#  * objective: relative 1e-5 (float32 per-cell arithmetic, float64 sums);
#  * field: 1e-3 voxel (max abs difference / h_p);
#  * residual histories: relative 1e-4, or an absolute floor of EPS_HIST[prec] * scale where
#    scale = max(|b|, |z|) of the oracle (the float32 / split-bfloat16 rounding of b and z
#    bounds how small a difference |b - z| can be resolved).
J_REL = 1e-5
FIELD_VOX = 1e-3
HIST_REL = 1e-4
EPS_HIST = {"fp32": 2e-6, "mixed": 4e-5}


def torch_dev():
    import torch
    return torch.device("cuda:0")


def T(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=torch_dev())


def N(t):
    return t.detach().cpu().numpy().astype(np.float64)


def hist_ok(gpu, cpu, scale, prec):
    """Residual history against the oracle: every entry within HIST_REL relative or within
    the absolute floor EPS_HIST[prec] * scale. Returns (ok, message); the message names the
    first failing entry, or says how many entries needed the floor (the relative bar alone
    held for the others)."""
    gpu, cpu = np.asarray(gpu), np.asarray(cpu)
    if gpu.shape != cpu.shape:
        return False, f"length {gpu.shape} vs {cpu.shape}"
    err = np.abs(gpu - cpu)
    rel = HIST_REL * np.abs(cpu)
    lim = np.maximum(rel, EPS_HIST[prec] * scale)
    bad = np.nonzero(err > lim)[0]
    if bad.size:
        i = bad[0]
        return False, f"iteration {i}: gpu {gpu[i]:.6e} cpu {cpu[i]:.6e} limit {lim[i]:.2e}"
    floor = int(np.count_nonzero(err > rel))
    worst = float(np.max(err / np.maximum(np.abs(cpu), 1e-300))) if err.size else 0.0
    used = float(np.max(err[err > rel]) / scale) if floor and scale > 0 else 0.0
    return True, (f"{err.size - floor} of {err.size} entries within {HIST_REL:g} relative "
                  f"(worst {worst:.1e}), {floor} at the absolute floor (largest "
                  f"{used:.1e} of the scale, floor {EPS_HIST[prec]:g})")


def oracle_precond(P, tri, r, precond):
    """z = P^-1 r by the oracle for the four GN-PCG preconditioners."""
    import oracle as O
    if precond == "block":
        return O.thomas(*O.pblock_tridiag(P, tri), r)
    if precond == "jacobi":
        return r / O.jacobi_diag(P, tri)
    if precond == "sgs":
        return O.sgs_apply(P, tri, r)
    return r.copy()


def precond_tol(P, tri, r, precond, zo, seed=1):
    """Bar for z = P^-1 r against the oracle, relative to max|z|: 16 times the change of z
    under a random relative perturbation of 2^-24 (one float32 rounding) of every entry of
    the Hessian blocks, plus 1e-6. The GPU assembles those entries in float32, so its z can
    differ by a few such roundings amplified by the conditioning of P (up to ~5e5 for the
    block-Jacobi lines of 500 faces)."""
    rng = np.random.default_rng(seed)
    trp = tuple(t * (1.0 + 2.0 ** -24 * rng.uniform(-1.0, 1.0, size=t.shape)) for t in tri)
    sens = np.abs(oracle_precond(P, trp, r, precond) - zo).max() / np.abs(zo).max()
    return 16.0 * sens + 1e-6


# The Armijo test of the line search compares J(b + lambda d) with J(b) on the device, each a
# float64 sum of float32 per-cell terms, whose rounding moves J by ~1e-7 relative. Once the
# decrease of a step is below that, the GPU can reject a step the float64 oracle accepts
# (the decision is taken on values that differ only by rounding); the GPU then stops with
# ls_failed at that step, leaving b unchanged.
LS_RESOLUTION = 1e-6


def gn_history_compare(rep, ro, rtol):
    """Compare a GN-PCG report with the oracle's. Returns the number of GN steps both took
    (the GPU's last step may be a rejected one, see LS_RESOLUTION) after asserting the
    J history over those steps at rtol."""
    k = rep["iters"]
    assert k == ro.iters, (k, ro.iters)
    if rep["ls_failed"]:
        dec = ro.J[k - 1] - ro.J[k]
        assert dec <= LS_RESOLUTION * abs(ro.J[k - 1]), ("rejected step decreases J by", dec)
        np.testing.assert_allclose(rep["J"][:k], ro.J[:k], rtol=rtol)
        return k - 1
    np.testing.assert_allclose(rep["J"], ro.J, rtol=rtol)
    return k


def gn_step_tol(P, b, precond="block", eta=0.1, maxit=30, seeds=(1, 2)):
    """Bar for J after one GN-PCG step from b against the oracle's: J_REL |J(b)| plus 16
    times the change of J(b + d) when every Hessian block entry and every gradient entry
    takes one random relative perturbation of 2^-24 (one float32 rounding) before the PCG
    solve, the largest over `seeds`. The GPU assembles both in float32; on PE lines of a
    few hundred faces the block-Jacobi systems amplify those roundings to ~1e-4 voxels in
    the direction, and J after a step that removes most of the misfit inherits that."""
    import oracle as O
    bl = P.lines(b)
    g = O.gradient(P, bl, True)
    tri = O.hessian_tridiag(P, bl, True)
    d, _, _ = O.pcg(P, tri, -g, precond, eta, maxit)
    J1 = O.objective(P, bl + d, True)["J"]
    sens = 0.0
    for seed in seeds:
        rng = np.random.default_rng(seed)
        trp = tuple(t * (1.0 + 2.0 ** -24 * rng.uniform(-1.0, 1.0, size=t.shape)) for t in tri)
        gp = g * (1.0 + 2.0 ** -24 * rng.uniform(-1.0, 1.0, size=g.shape))
        dp, _, _ = O.pcg(P, trp, -gp, precond, eta, maxit)
        sens = max(sens, abs(O.objective(P, bl + dp, True)["J"] - J1))
    return J_REL * abs(O.objective(P, bl, True)["J"]) + 16.0 * sens
