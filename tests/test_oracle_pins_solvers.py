"""Pins of the oracle's solver internals that the per-operator pins do not reach.

* the b-step QP data of Section 4.2 (c and G of eq. qp) against a finite difference of the
  b-subproblem and against the dense Gauss-Newton matrix assembled from its definition;
* fixed points: ADMM (eq. admmStep1-3) run to convergence ends at a stationary point of
  J = D + alpha S, and GN-PCG (eq. GNstep) at one of J_GN, with the gradients that the
  finite-difference pins already fix;
* the Jacobi preconditioner against the diagonal of the dense H_JGN;
* the three relative tests of eq. stopping1, each made the binding one in turn;
* the tolerances of eq. admmStop at nonzero eps_abs and eps_rel on hand-checked vectors.

A few tests plant a plausible mistake in a copy of the oracle's arithmetic (on the CPU) and
check that the corresponding pin rejects it, so the pins are known to be sensitive to it.
"""
import math

import numpy as np
import pytest

import oracle as O
import oracle.epi_oracle as OE
from synth import generate


def rand_problem(M, m2, m3, seed=0, alpha=0.7, beta=10.0, amp=1.0):
    r = np.random.default_rng(seed)
    h = (1.0 / M, 1.0 / m2, 1.0 / m3 if m3 > 1 else 1.0)
    Ip = amp * r.uniform(0.2, 1.0, size=(m3, m2, M))
    Im = amp * r.uniform(0.2, 1.0, size=(m3, m2, M))
    return O.make_problem(Ip, Im, h, alpha, beta)


def smooth_field(P, seed=1, gmax=0.4):
    r = np.random.default_rng(seed)
    b = r.normal(size=(P.L, P.M + 1))
    g = np.diff(b, axis=1) / P.hp
    return b * (gmax / np.abs(g).max())


def dense_residual_jacobian(P, b, eps=1e-7):
    """J_r = d r / d b column by column by central differences (r is a product of two affine
    functions of b on each interpolation segment, so this is exact up to rounding)."""
    n = P.n
    Jr = np.zeros((P.L * P.M, n))
    bf = b.reshape(-1)
    for i in range(n):
        bp, bm = bf.copy(), bf.copy()
        bp[i] += eps
        bm[i] -= eps
        Jr[:, i] = (O.line_eval(P, bp)["r"].reshape(-1) - O.line_eval(P, bm)["r"].reshape(-1)) / (2 * eps)
    return Jr


def bsub_objective(P, b, z, u, rho):
    """The b-subproblem of eq. admmStep1 without the indicator of C:
    f(b) + (rho v / 2)|b - z + u|^2 with f = D + (alpha v / 2)|D1 b|^2, D1 dense from its
    Kronecker definition (eq. D1)."""
    _, D1, _, _ = O.dense_operators(P.M, P.m2, P.m3, P.hp, P.h2, P.h3)
    bb = b.reshape(-1)
    f = O.distance(P, b) + 0.5 * P.alpha * P.v * float(np.sum((D1 @ bb) ** 2))
    return f + 0.5 * rho * P.v * float(np.sum((bb - z.reshape(-1) + u.reshape(-1)) ** 2))


def _qp_state(P, seed):
    r = np.random.default_rng(seed)
    b = smooth_field(P, seed, 0.5)
    z = b + 0.4 * P.hp * r.normal(size=b.shape)
    u = 0.2 * P.hp * r.normal(size=b.shape)
    return b, z, u


def _check_qp_c(P, qp_data, b, z, u, rho):
    """c of the QP data equals the gradient of the b-subproblem at b^k (central differences
    along random directions)."""
    _, _, c, _ = qp_data(P, b, z, u, rho)
    r = np.random.default_rng(3)
    for _ in range(6):
        d = r.normal(size=b.shape)
        eps = 1e-6 * P.hp
        fd = (bsub_objective(P, b + eps * d, z, u, rho) - bsub_objective(P, b - eps * d, z, u, rho)) / (2 * eps)
        an = float(np.sum(c * d))
        assert abs(fd - an) <= 1e-6 * np.abs(c).sum() * np.abs(d).max(), (fd, an)


# ------------------------------------------------------------------------- QP data, eq. qp
@pytest.mark.parametrize("shape,alpha,rho", [((7, 3, 2), 0.6, 40.0), ((9, 4, 1), 3.0, 5.0)])
def test_qp_gradient_c_is_the_gradient_of_the_b_subproblem(shape, alpha, rho):
    P = rand_problem(*shape, seed=31, alpha=alpha)
    b, z, u = _qp_state(P, 32)
    _check_qp_c(P, OE._qp_data, b, z, u, rho)


def test_qp_matrix_G_is_the_dense_gauss_newton_matrix():
    """G = v J_r^T J_r + alpha v D1^T D1 + rho v I with J_r from differences of r and D1 from
    eq. D1; it is tridiagonal within each PE line and zero across lines."""
    P = rand_problem(6, 3, 2, seed=33, alpha=0.8)
    rho = 25.0
    b, z, u = _qp_state(P, 34)
    Jr = dense_residual_jacobian(P, b)
    _, D1, _, _ = O.dense_operators(P.M, P.m2, P.m3, P.hp, P.h2, P.h3)
    G = P.v * Jr.T @ Jr + P.alpha * P.v * D1.T @ D1 + rho * P.v * np.eye(P.n)
    Gd, Go, _, g = OE._qp_data(P, b, z, u, rho)
    nf = P.M + 1
    band = np.zeros_like(G)
    for ln in range(P.L):
        s = ln * nf
        band[s:s + nf, s:s + nf] = np.diag(Gd[ln]) + np.diag(Go[ln], 1) + np.diag(Go[ln], -1)
    np.testing.assert_allclose(band, G, rtol=1e-6, atol=1e-7 * np.abs(G).max())
    np.testing.assert_allclose(g.reshape(-1), D1 @ b.reshape(-1), rtol=0, atol=1e-13)


def _qp_data_dropped_term(P, bl, zl, ul, rho):
    Gd, Go, c, g = OE._qp_data(P, bl, zl, ul, rho)
    return Gd, Go, c - P.alpha * P.v * O.apply_D1tD1(P, bl), g


def _qp_data_flipped_sign(P, bl, zl, ul, rho):
    Gd, Go, c, g = OE._qp_data(P, bl, zl, ul, rho)
    return Gd, Go, c - 2.0 * rho * P.v * (P.lines(bl) - P.lines(zl) + P.lines(ul)), g


@pytest.mark.parametrize("mutant", [_qp_data_dropped_term, _qp_data_flipped_sign])
def test_qp_gradient_pin_rejects_planted_mistakes(mutant):
    """The finite-difference pin of c fails for a dropped alpha v D1'D1 b^k and for a sign
    slip in rho v (b - z + u)."""
    P = rand_problem(7, 3, 2, seed=31, alpha=0.6)
    b, z, u = _qp_state(P, 32)
    with pytest.raises(AssertionError):
        _check_qp_c(P, mutant, b, z, u, 40.0)


# ------------------------------------------------------------------------- fixed points
def _admm_stationarity(P, rho, max_iter=3000):
    g0 = np.linalg.norm(O.gradient(P, np.zeros((P.L, P.M + 1)), False))
    b, z, u, rep = O.solve_admm(P, rho=rho, max_iter=max_iter, eps_abs=0.0, eps_rel=1e-11)
    g = np.linalg.norm(O.gradient(P, b, False))
    return rep, g / g0, float(np.abs(b - z).max() / P.hp), b


# (seed, shape, alpha, rho): a case whose iterates never touch the constraint and one in
# which the active-set path runs during the iteration (|D1 b| reaches the bound on the way)
ADMM_FIXED = [(1, (14, 10, 6), 2.0, 400.0, False), (1, (14, 10, 6), 0.05, 50.0, True)]


@pytest.mark.parametrize("seed,shape,alpha,rho,active", ADMM_FIXED)
def test_admm_converges_to_a_stationary_point_of_J(seed, shape, alpha, rho, active):
    """At a fixed point of the scaled ADMM iteration b = z, the b-step's QP step is zero,
    and the multiplier identity rho u = alpha (D2'D2 + D3'D3) z holds, so
    grad D + alpha v (D1'D1 + D2'D2 + D3'D3) b = 0: the limit is a stationary point of
    J = D + alpha S whenever it lies inside the feasible set. The gradient used here is the
    finite-difference-pinned one."""
    v = generate(seed, shape, 0, noise=0.0)
    P = O.make_problem(v.Ip, v.Im, v.h, alpha)
    rep, grel, bz, b = _admm_stationarity(P, rho)
    assert rep.converged
    assert (max(rep.max_active) > 0) == active
    assert np.abs(np.diff(b, axis=1)).max() / P.hp < 1.0 - 1e-6     # interior limit
    assert grel <= 1e-9, grel
    assert bz <= 1e-9, bz


_QP_DATA_ORIG = OE._qp_data


def test_admm_fixed_point_pin_rejects_a_dropped_term(monkeypatch):
    """With alpha v D1'D1 b^k dropped from c the iteration goes elsewhere: after 100
    iterations (the correct one is within 1e-3 of the limit by then) the gradient of J is
    still a sizeable fraction of its value at zero."""
    v = generate(1, (14, 10, 6), 0, noise=0.0)
    P = O.make_problem(v.Ip, v.Im, v.h, 2.0)

    def mutant(P_, bl, zl, ul, rho):
        Gd, Go, c, g = _QP_DATA_ORIG(P_, bl, zl, ul, rho)
        return Gd, Go, c - P_.alpha * P_.v * O.apply_D1tD1(P_, bl), g

    monkeypatch.setattr(OE, "_qp_data", mutant)
    rep, grel, _, _ = _admm_stationarity(P, 400.0, max_iter=100)
    assert grel > 1e-1, grel


def test_gnpcg_converges_to_a_stationary_point_of_J_GN():
    """GN-PCG with an essentially exact inner solve and the Armijo step ends at a point
    where the finite-difference-pinned gradient of J_GN = D + alpha S + P vanishes. (With
    linear interpolation J_GN is only piecewise smooth: its derivative jumps where a sample
    crosses a knot, and many runs end on such a kink with a one-sided gradient that does not
    vanish; this case has a smooth limit.)"""
    v = generate(2, (16, 8, 5), 0, noise=0.0)
    P = O.make_problem(v.Ip, v.Im, v.h, 8.0)
    b, rep = O.solve_gnpcg(P, max_iter=60, eta=1e-10, pcg_max=3000, use_stopping=False,
                           rel_grad_tol=1e-11, ls_max=40)
    g = np.linalg.norm(O.gradient(P, b, True))
    g0 = np.linalg.norm(O.gradient(P, np.zeros((P.L, P.M + 1)), True))
    assert rep.converged and not rep.ls_failed
    assert g / g0 <= 1e-10
    assert all(lam > 0 for lam in rep.step)
    # no accepted step increased J_GN (beyond rounding of J itself)
    assert all(b_ <= a_ * (1 + 1e-13) for a_, b_ in zip(rep.J[:-1], rep.J[1:]))


# ------------------------------------------------------------------------- Jacobi, eq. Pblock
def test_jacobi_diag_is_the_diagonal_of_the_dense_H_JGN():
    """H_JGN = v J_r^T J_r + alpha v (D1'D1 + D2'D2 + D3'D3) + beta v D1' diag(phi''(D1 b)) D1
    + gamma I, assembled densely from its definition; the Jacobi preconditioner is its
    diagonal and block-Jacobi keeps its line blocks."""
    P = rand_problem(6, 4, 3, seed=35, alpha=0.9, beta=10.0)
    b = smooth_field(P, 36, 0.5)
    Jr = dense_residual_jacobian(P, b)
    _, D1, D2, D3 = O.dense_operators(P.M, P.m2, P.m3, P.hp, P.h2, P.h3)
    g = D1 @ b.reshape(-1)
    H = (P.v * Jr.T @ Jr + P.alpha * P.v * (D1.T @ D1 + D2.T @ D2 + D3.T @ D3)
         + P.beta * P.v * D1.T @ np.diag(O.d2phi(g)) @ D1 + P.gamma * np.eye(P.n))
    tri = O.hessian_tridiag(P, b, True)
    np.testing.assert_allclose(O.jacobi_diag(P, tri).reshape(-1), np.diag(H), rtol=1e-7,
                               atol=1e-9 * np.abs(H).max())
    pd, po = O.pblock_tridiag(P, tri)
    nf = P.M + 1
    for ln in range(P.L):
        s = ln * nf
        blk = H[s:s + nf, s:s + nf]
        np.testing.assert_allclose(pd[ln], np.diag(blk), rtol=1e-7, atol=1e-9 * np.abs(H).max())
        np.testing.assert_allclose(po[ln], np.diag(blk, 1), rtol=1e-7, atol=1e-9 * np.abs(H).max())


# ------------------------------------------------------------------------- eq. stopping1
@pytest.fixture(scope="module")
def gn_path():
    """Iterates of one GN-PCG run without stopping tests: b_k and J_k for k = 0..K (the
    solver is deterministic, so the run stopped after k steps reproduces the prefix)."""
    v = generate(3, (16, 8, 5), 0)
    P = O.make_problem(v.Ip, v.Im, v.h, 2.0)
    K = 6
    bs, Js, gs = [], [], []
    for k in range(K + 1):
        b, rep = O.solve_gnpcg(P, max_iter=k, use_stopping=False)
        bs.append(b.reshape(-1))
        Js.append(rep.J[-1])
        gs.append(rep.grad_norm[-1])
    return P, bs, Js, gs


def _stopping_quantities(bs, Js, gs):
    """Per step k >= 1 the three quantities of eq. stopping1 scaled by their right-hand
    sides without the tolerance: |J_k - J_k-1| / (1 + |J_0|), |b_k - b_k-1| / (1 + |b_k-1|),
    |grad J_k| / (1 + |J_0|)."""
    J0 = abs(Js[0])
    q = {"obj": [], "iter": [], "grad": []}
    for k in range(1, len(Js)):
        q["obj"].append(abs(Js[k] - Js[k - 1]) / (1.0 + J0))
        q["iter"].append(np.linalg.norm(bs[k] - bs[k - 1]) / (1.0 + np.linalg.norm(bs[k - 1])))
        q["grad"].append(gs[k] / (1.0 + J0))
    return q


def _tol_first_at(vals, k):
    """A tolerance that the sequence vals (index 0 = step 1) first meets at step k, or None
    if every earlier value is already below the value at k."""
    t = vals[k - 1]
    if any(x <= t * (1 + 1e-9) for x in vals[:k - 1]):
        return None
    return t * (1 + 1e-9)


@pytest.mark.parametrize("binding", ["obj", "iter", "grad"])
def test_stopping1_each_test_can_be_the_binding_one(gn_path, binding):
    """With the binding test's tolerance chosen so that it first holds after step k* and the
    other two met from an earlier step on, GN-PCG stops after exactly k* steps; tightening
    the binding tolerance below its value at k* moves the stop to a later step."""
    P, bs, Js, gs = gn_path
    q = _stopping_quantities(bs, Js, gs)
    kstar = None
    for k in range(2, len(Js)):
        if _tol_first_at(q[binding], k) is not None:
            kstar = k
            break
    assert kstar is not None
    tol = {name: max(q[name][:kstar]) * 1.01 for name in q}   # met from step 1 on
    for name in q:
        if name != binding:
            tol[name] = max(q[name]) * 2.0
    tol[binding] = _tol_first_at(q[binding], kstar)
    kw = dict(eps_obj=tol["obj"], eps_iter=tol["iter"], eps_grad=tol["grad"])
    _, rep = O.solve_gnpcg(P, max_iter=len(Js) - 1, use_stopping=True, **kw)
    assert rep.converged and rep.iters == kstar, (binding, rep.iters, kstar)
    tight = dict(kw)
    key = {"obj": "eps_obj", "iter": "eps_iter", "grad": "eps_grad"}[binding]
    tight[key] = q[binding][kstar - 1] * (1 - 1e-6)
    _, rep2 = O.solve_gnpcg(P, max_iter=len(Js) - 1, use_stopping=True, **tight)
    assert rep2.iters > kstar


def test_stopping1_needs_all_three_tests(gn_path):
    """Two tests met from step 1 on and the third never: GN-PCG runs to max_iter."""
    P, bs, Js, gs = gn_path
    q = _stopping_quantities(bs, Js, gs)
    kw = dict(eps_obj=max(q["obj"]) * 2, eps_iter=max(q["iter"]) * 2,
              eps_grad=min(q["grad"]) * 0.5)
    _, rep = O.solve_gnpcg(P, max_iter=len(Js) - 1, use_stopping=True, **kw)
    assert not rep.converged and rep.iters == len(Js) - 1


# ------------------------------------------------------------------------- eq. admmStop
def test_admm_tolerances_on_hand_checked_vectors():
    """n = 4 faces (one line of 3 cells): b = 3, z = 1, z_old = 0, u = 1/2 on every face, so
    |b| = 6, |z| = 2, |u| = 1, |b - z| = 4, |z - z_old| = 2, sqrt(n) = 2. With
    eps_abs = 0.1, eps_rel = 0.01, rho = 10 and v = h_p = 1/3 (2D, h2 = h3 = 1):
    r_pri = 4, r_dual = rho v 2 = 20/3, eps_pri = 2 (0.1) + 0.01 (6) = 0.26,
    eps_dual = 2 (0.1) + 0.01 (10/3)(1) = 0.2 + 1/30."""
    P = O.make_problem(np.ones((1, 1, 3)), np.ones((1, 1, 3)), (1 / 3, 1.0, 1.0), 1.0)
    one = np.ones((1, 4))
    rp, rd, ep, ed = O.admm_residuals(P, 3 * one, one, 0 * one, 0.5 * one, 10.0, 0.1, 0.01)
    assert math.isclose(rp, 4.0, rel_tol=1e-15)
    assert math.isclose(rd, 20.0 / 3.0, rel_tol=1e-15)
    assert math.isclose(ep, 0.26, rel_tol=1e-14)
    assert math.isclose(ed, 0.2 + 1.0 / 30.0, rel_tol=1e-14)
    # the relative part takes the larger of |b| and |z|
    _, _, ep2, _ = O.admm_residuals(P, one, 3 * one, 0 * one, 0.5 * one, 10.0, 0.1, 0.01)
    assert math.isclose(ep2, 0.26, rel_tol=1e-14)


def test_admm_stops_exactly_when_both_residuals_meet_their_tolerances():
    """A run with nonzero eps_abs and eps_rel stops at the first iteration at which both
    r_pri <= eps_pri and r_dual <= eps_dual hold (checked against the reported histories of
    a run without stopping)."""
    P = rand_problem(8, 5, 3, seed=37, alpha=0.5)
    kw = dict(rho=20.0, eps_abs=2e-4, eps_rel=1e-2)
    _, _, _, full = O.solve_admm(P, max_iter=60, **dict(kw, eps_abs=0.0, eps_rel=0.0))
    n = P.n
    # recompute the tolerances of each iteration from the histories of the unstopped run
    _, _, _, rep = O.solve_admm(P, max_iter=60, **kw)
    k = rep.iters
    assert rep.converged
    for i in range(k - 1):
        assert not (full.r_pri[i] <= rep.eps_pri[i] and full.r_dual[i] <= rep.eps_dual[i])
    assert full.r_pri[k - 1] <= rep.eps_pri[k - 1] and full.r_dual[k - 1] <= rep.eps_dual[k - 1]
    assert all(e >= math.sqrt(n) * 2e-4 for e in rep.eps_pri + rep.eps_dual)


# ---------------------------------------------------------------- augmented Lagrangian (eq. Lp)
def test_augmented_lagrangian_reduces_to_J_and_is_affine_in_the_multiplier():
    """L_rho(b, z, y) = f(b) + g(z) + y'(b - z) + (rho v / 2)|b - z|^2 (eq. Lp) with
    f = D + (alpha v / 2)|D1 b|^2 and g = (alpha v / 2)(|D2 z|^2 + |D3 z|^2):
      * at z = b the multiplier and penalty terms vanish and f + g is J = D + alpha S
        (the objective without the penalty, itself pinned by finite differences);
      * it is affine in u with slope rho v (b - z), and a quadratic in rho v at u = 0
        whose coefficient is |b - z|^2 / 2."""
    P = rand_problem(11, 6, 5, seed=23, alpha=0.8)
    r = np.random.default_rng(5)
    b = smooth_field(P, 4, 0.5)
    z = b + 0.2 * P.hp * r.normal(size=b.shape)
    u = 0.3 * P.hp * r.normal(size=b.shape)
    for rho in (3.0, 40.0):
        L_bb = O.augmented_lagrangian(P, b, b, u, rho)
        J = O.objective(P, b, False)["J"]
        assert math.isclose(L_bb, J, rel_tol=1e-12)
        L0 = O.augmented_lagrangian(P, b, z, 0.0 * u, rho)
        L1 = O.augmented_lagrangian(P, b, z, u, rho)
        L2 = O.augmented_lagrangian(P, b, z, 2.0 * u, rho)
        slope = rho * P.v * float(np.sum(u * (b - z)))
        assert math.isclose(L1 - L0, slope, rel_tol=1e-9, abs_tol=1e-15)
        assert math.isclose(L2 - L1, slope, rel_tol=1e-9, abs_tol=1e-15)
    # the rho-dependence at u = 0: L(rho) - L(0+) = (rho v / 2)|b - z|^2
    La = O.augmented_lagrangian(P, b, z, 0.0 * u, 1e-12)
    Lb = O.augmented_lagrangian(P, b, z, 0.0 * u, 10.0)
    assert math.isclose(Lb - La, 0.5 * 10.0 * P.v * float(np.sum((b - z) ** 2)), rel_tol=1e-9)
    # g(z) alone: with b = z the part that depends on z only is alpha v / 2 of the
    # transverse differences, i.e. J(z) minus D(z) minus the D1 part
    S = O.objective(P, z, False)
    d1 = np.diff(P.lines(z), axis=1) / P.hp
    g_z = P.alpha * S["S"] - 0.5 * P.alpha * P.v * float(np.sum(d1 * d1))
    L_zz = O.augmented_lagrangian(P, z, z, u, 5.0)
    f_z = S["D"] + 0.5 * P.alpha * P.v * float(np.sum(d1 * d1))
    assert math.isclose(L_zz, f_z + g_z, rel_tol=1e-12)
