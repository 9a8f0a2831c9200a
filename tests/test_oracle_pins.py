"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these checks re-types an oracle formula: they use finite differences, dense
operators assembled from the Kronecker definitions of Section 3, library routines
(numpy.linalg.solve, scipy.fft.dct, scipy.linalg.solve_banded), brute-force enumeration,
closed-form special cases and the sparsity patterns printed in Figure 2.
"""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.fft
import scipy.linalg

import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rand_problem(M, m2, m3, seed=0, alpha=0.7, beta=10.0, h=None, amp=1.0):
    r = np.random.default_rng(seed)
    if h is None:
        h = (1.0 / M, 1.0 / m2, 1.0 / m3 if m3 > 1 else 1.0)
    Ip = amp * r.uniform(0.2, 1.0, size=(m3, m2, M))
    Im = amp * r.uniform(0.2, 1.0, size=(m3, m2, M))
    return O.make_problem(Ip, Im, h, alpha, beta)


def smooth_field(P, seed=1, gmax=0.4):
    """Random field with max|D1 b| = gmax, generic (samples off the knots)."""
    r = np.random.default_rng(seed)
    b = r.normal(size=(P.L, P.M + 1))
    g = np.diff(b, axis=1) / P.hp
    b *= gmax / np.abs(g).max()
    return b


def dense_from_apply(fn, n):
    E = np.eye(n)
    return np.stack([fn(E[i]).reshape(-1) for i in range(n)], axis=1)


# ----------------------------------------------------------------------------- image model
def test_integer_shift_reads_shifted_samples():
    """b = k h_p (constant, integer k): a = k h_p, D1 b = 0, so r_c = I+[c+k] - I-[c-k]
    with zero outside the line (compact support)."""
    P = rand_problem(9, 4, 3, seed=3)
    for k in (-3, -1, 0, 2, 5, 9, 12):
        b = np.full((P.L, P.M + 1), k * P.hp)
        r = O.line_eval(P, b)["r"]
        exp = np.zeros_like(r)
        for c in range(P.M):
            if 0 <= c + k < P.M:
                exp[:, c] += P.Ip[:, c + k]
            if 0 <= c - k < P.M:
                exp[:, c] -= P.Im[:, c - k]
        np.testing.assert_allclose(r, exp, rtol=0, atol=1e-14)


def test_half_integer_shift_averages_two_samples():
    P = rand_problem(8, 3, 2, seed=4)
    k = 1.5
    b = np.full((P.L, P.M + 1), k * P.hp)
    r = O.line_eval(P, b)["r"]
    pad = lambda T, i: T[:, i] if 0 <= i < P.M else 0.0  # noqa: E731
    for c in range(P.M):
        ep = 0.5 * (pad(P.Ip, c + 1) + pad(P.Ip, c + 2))
        em = 0.5 * (pad(P.Im, c - 2) + pad(P.Im, c - 1))
        np.testing.assert_allclose(r[:, c], ep - em, atol=1e-14)


def test_constant_field_beyond_the_domain_is_a_global_minimiser():
    """A constant field of M voxels shifts both images out of the domain: D = S = 0
    (the degeneracy noted for large constant fields in Section 2)."""
    P = rand_problem(10, 5, 2, seed=5)
    b = np.full((P.L, P.M + 1), P.M * P.hp)
    assert O.distance(P, b) == 0.0
    assert O.reg_S(P, b) == 0.0
    assert O.distance(P, np.zeros_like(b)) > 0.0


def test_distance_symmetry_swap_images_and_sign():
    P = rand_problem(12, 5, 3, seed=6)
    Q = O.Problem(P.Im, P.Ip, P.M, P.m2, P.m3, P.hp, P.h2, P.h3, P.alpha)
    b = smooth_field(P, 2, 0.6)
    assert math.isclose(O.distance(P, b), O.distance(Q, -b), rel_tol=1e-13)


# ----------------------------------------------------------------------------- derivatives
def test_residual_jacobian_by_finite_differences():
    """r is a product of two affine functions of b on each interpolation segment, so a
    central difference reproduces the Jacobian up to rounding."""
    P = rand_problem(7, 3, 2, seed=7)
    b = smooth_field(P, 3, 0.5)
    e = O.line_eval(P, b)
    eps = 1e-7
    for ln in range(P.L):
        for i in range(P.M + 1):
            bp = b.copy(); bp[ln, i] += eps
            bm = b.copy(); bm[ln, i] -= eps
            dr = (O.line_eval(P, bp)["r"][ln] - O.line_eval(P, bm)["r"][ln]) / (2 * eps)
            exp = np.zeros(P.M)
            if i < P.M:
                exp[i] += e["Jl"][ln, i]
            if i > 0:
                exp[i - 1] += e["Jr"][ln, i - 1]
            np.testing.assert_allclose(dr, exp, rtol=1e-6, atol=1e-6 * np.abs(exp).max())


@pytest.mark.parametrize("shape", [(16, 12, 1), (9, 6, 5)])
def test_gradient_by_finite_differences(shape):
    M, m2, m3 = shape
    P = rand_problem(M, m2, m3, seed=8, alpha=0.3, beta=10.0)
    b = smooth_field(P, 4, 0.6)
    g = O.gradient(P, b, True)
    r = np.random.default_rng(9)
    for _ in range(4):
        d = r.normal(size=b.shape)
        eps = 1e-6
        Jp = O.objective(P, b + eps * d, True)["J"]
        Jm = O.objective(P, b - eps * d, True)["J"]
        fd = (Jp - Jm) / (2 * eps)
        an = float(np.sum(g * d))
        assert abs(fd - an) <= 1e-5 * (abs(an) + 1e-3 * np.abs(g).sum() * 1e-3), (fd, an)


def test_phi_derivatives_by_finite_differences():
    x = np.linspace(-0.95, 0.95, 37)
    eps = 1e-6
    np.testing.assert_allclose((O.phi(x + eps) - O.phi(x - eps)) / (2 * eps), O.dphi(x),
                               rtol=1e-6, atol=1e-8)
    np.testing.assert_allclose((O.dphi(x + eps) - O.dphi(x - eps)) / (2 * eps), O.d2phi(x),
                               rtol=1e-6, atol=1e-7)
    assert O.phi(np.array([0.0]))[0] == 0.0
    assert np.all(np.isinf(O.phi(np.array([-1.0, 1.0, 1.2, -3.0]))))


def test_gauss_newton_hessian_equals_dense_JtJ():
    """H_D = v J_r^T J_r with J_r from finite differences of r; the regulariser and penalty
    Hessians from the dense Kronecker operators of eq. D1 and eq. d2d3."""
    P = rand_problem(6, 4, 3, seed=10, alpha=0.9, beta=10.0)
    b = smooth_field(P, 5, 0.5)
    n = P.n
    eps = 1e-7
    Jr = np.zeros((P.L * P.M, n))
    for i in range(n):
        bp = b.reshape(-1).copy(); bp[i] += eps
        bm = b.reshape(-1).copy(); bm[i] -= eps
        Jr[:, i] = (O.line_eval(P, bp)["r"].reshape(-1) - O.line_eval(P, bm)["r"].reshape(-1)) / (2 * eps)
    A1, D1, D2, D3 = O.dense_operators(P.M, P.m2, P.m3, P.hp, P.h2, P.h3)
    g = D1 @ b.reshape(-1)
    HS = P.v * (D1.T @ D1 + D2.T @ D2 + D3.T @ D3)
    HP = P.beta * P.v * D1.T @ np.diag(O.d2phi(g)) @ D1
    H = P.v * Jr.T @ Jr + P.alpha * HS + P.gamma * np.eye(n) + HP
    tri = O.hessian_tridiag(P, b, True)
    Hd = dense_from_apply(lambda x: O.hessian_apply(P, tri, x), n)
    np.testing.assert_allclose(Hd, H, rtol=1e-6, atol=1e-6 * np.abs(H).max())
    # gradient of S is the Hessian of S times b
    gS = (O.gradient(P, b, False) - O.gradient(O.Problem(P.Ip, P.Im, P.M, P.m2, P.m3, P.hp,
                                                           P.h2, P.h3, 0.0), b, False))
    np.testing.assert_allclose(gS.reshape(-1), P.alpha * HS @ b.reshape(-1), rtol=1e-10,
                               atol=1e-12)
    # S itself from the dense operators
    bb = b.reshape(-1)
    S = 0.5 * P.v * (np.sum((D1 @ bb) ** 2) + np.sum((D2 @ bb) ** 2) + np.sum((D3 @ bb) ** 2))
    assert math.isclose(O.reg_S(P, b), S, rel_tol=1e-12)
    # the averaging operator A1 of eq. A gives the sample displacement
    np.testing.assert_allclose(O.line_eval(P, b)["a"].reshape(-1), A1 @ bb, atol=1e-15)


def _pattern(Mx):
    rr, cc = np.nonzero(np.abs(Mx) > 1e-14 * np.abs(Mx).max())
    return set(zip((rr + 1).tolist(), (cc + 1).tolist()))


def _gold(name):
    out = set()
    for line in open(os.path.join(GOLD, f"sparsity_4x4_{name}.txt")):
        if line.startswith("#") or not line.strip():
            continue
        a, b = line.split()
        out.add((int(a), int(b)))
    return out


def test_sparsity_patterns_match_figure_2():
    """4x4 cells in 2D, PE along the first axis: 5 faces per line, 20 faces."""
    P = rand_problem(4, 4, 1, seed=11, alpha=1.0)
    b = smooth_field(P, 6, 0.4)
    n = P.n
    eps = 1e-7
    Jr = np.zeros((P.L * P.M, n))
    for i in range(n):
        bp = b.reshape(-1).copy(); bp[i] += eps
        bm = b.reshape(-1).copy(); bm[i] -= eps
        Jr[:, i] = (O.line_eval(P, bp)["r"].reshape(-1) - O.line_eval(P, bm)["r"].reshape(-1)) / (2 * eps)
    _, D1, D2, D3 = O.dense_operators(4, 4, 1, P.hp, P.h2, P.h3)
    g = D1 @ b.reshape(-1)
    # from the oracle's own operators
    diag, off = O.hessian_tridiag(P, b, False, with_gamma=False)
    Q0 = O.Problem(P.Ip, P.Im, P.M, P.m2, P.m3, P.hp, P.h2, P.h3, 0.0)
    dD, oD = O.hessian_tridiag(Q0, b, False, with_gamma=False)
    HD = np.diag(dD.reshape(-1))
    for ln in range(P.L):
        for c in range(P.M):
            i = ln * (P.M + 1) + c
            HD[i, i + 1] = HD[i + 1, i] = oD[ln, c]
    assert _pattern(HD) == _gold("H_D") == _pattern(Jr.T @ Jr)
    HS = dense_from_apply(lambda x: O.apply_D1tD1(P, x) + O.apply_laplacian_cross(P, x), n)
    assert _pattern(HS) == _gold("hess_S")
    assert _pattern(dense_from_apply(lambda x: O.apply_D1tD1(P, x), n)) == _gold("D1tD1")
    assert _pattern(dense_from_apply(lambda x: O.apply_laplacian_cross(P, x), n)) == _gold("D2tD2")
    assert _pattern(D2.T @ D2) == _gold("D2tD2")
    HP = D1.T @ np.diag(O.d2phi(g)) @ D1
    assert _pattern(HP) == _gold("hess_P")


# ----------------------------------------------------------------------------- linear algebra
def test_thomas_matches_dense_and_banded_solvers():
    r = np.random.default_rng(12)
    L, N = 5, 17
    off = r.normal(size=(L, N - 1))
    diag = np.abs(r.normal(size=(L, N))) + 2.5 * (np.abs(np.pad(off, ((0, 0), (1, 0)))) +
                                                 np.abs(np.pad(off, ((0, 0), (0, 1)))))
    rhs = r.normal(size=(L, N))
    x = O.thomas(diag, off, rhs)
    for ln in range(L):
        A = np.diag(diag[ln]) + np.diag(off[ln], 1) + np.diag(off[ln], -1)
        np.testing.assert_allclose(x[ln], np.linalg.solve(A, rhs[ln]), rtol=1e-12, atol=1e-12)
        ab = np.zeros((3, N))
        ab[0, 1:] = off[ln]
        ab[1] = diag[ln]
        ab[2, :-1] = off[ln]
        np.testing.assert_allclose(x[ln], scipy.linalg.solve_banded((1, 1), ab, rhs[ln]),
                                   rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("m", [1, 2, 5, 8, 13, 110])
def test_dct_matrix_is_scipy_orthonormal_dct2_and_diagonalises_Dt_D(m):
    C = O.dct_matrix(m)
    np.testing.assert_allclose(C, scipy.fft.dct(np.eye(m), type=2, norm="ortho", axis=0),
                               atol=1e-13)
    np.testing.assert_allclose(C @ C.T, np.eye(m), atol=1e-12)
    h = 0.37
    D = np.zeros((max(m - 1, 0), m))
    for r_ in range(m - 1):
        D[r_, r_], D[r_, r_ + 1] = -1 / h, 1 / h
    np.testing.assert_allclose(C.T @ np.diag(O.dct_eigs(m, h)) @ C, D.T @ D,
                               atol=1e-10 * max(1.0, 4 / h ** 2))


@pytest.mark.parametrize("shape", [(3, 5, 4), (4, 6, 1), (2, 1, 7)])
def test_zstep_is_the_dense_smoothness_solve(shape):
    M, m2, m3 = shape
    P = rand_problem(M, m2, m3, seed=13, alpha=2.5)
    rho = 7.0
    _, _, D2, D3 = O.dense_operators(M, m2, m3, P.hp, P.h2, P.h3)
    Gt = P.alpha * P.v * (D2.T @ D2 + D3.T @ D3) + rho * P.v * np.eye(P.n)
    w = np.random.default_rng(14).normal(size=P.n)
    z = np.linalg.solve(Gt, rho * P.v * w)
    np.testing.assert_allclose(O.zstep(P, w, rho).reshape(-1), z, rtol=1e-11, atol=1e-12)


def test_pcg_converges_to_the_dense_gn_step_and_is_descent():
    P = rand_problem(8, 5, 3, seed=15, alpha=0.4)
    b = smooth_field(P, 7, 0.5)
    g = O.gradient(P, b, True)
    tri = O.hessian_tridiag(P, b, True)
    H = dense_from_apply(lambda x: O.hessian_apply(P, tri, x), P.n)
    d_exact = np.linalg.solve(H, -g.reshape(-1))
    for pc in ("block", "jacobi", "none"):
        d, it, rel = O.pcg(P, tri, -g, pc, tol=1e-12, maxit=500)
        np.testing.assert_allclose(d.reshape(-1), d_exact, rtol=1e-8, atol=1e-10 * np.abs(d_exact).max())
    d, it, rel = O.pcg(P, tri, -g, "block", tol=0.1, maxit=30)
    assert float(np.sum(g * d)) < 0
    assert np.linalg.norm(H @ d.reshape(-1) + g.reshape(-1)) <= 0.1 * np.linalg.norm(g) * (1 + 1e-9)
    # the block-Jacobi preconditioner is the dense Hessian with the cross-line part
    # replaced by its diagonal (eq. Pblock)
    _, _, D2, D3 = O.dense_operators(P.M, P.m2, P.m3, P.hp, P.h2, P.h3)
    X = D2.T @ D2 + D3.T @ D3
    Pb = H - P.alpha * P.v * (X - np.diag(np.diag(X)))
    pd, po = O.pblock_tridiag(P, tri)
    rhs = np.random.default_rng(3).normal(size=(P.L, P.M + 1))
    np.testing.assert_allclose(O.thomas(pd, po, rhs).reshape(-1), np.linalg.solve(Pb, rhs.reshape(-1)),
                               rtol=1e-9, atol=1e-12)


def _textbook_sgs_sweep(A, rhs):
    """One symmetric Gauss-Seidel iteration from x = 0 on a dense A: a forward sweep that
    updates x_i in place from the newest values, then a backward sweep."""
    n = len(rhs)
    x = np.zeros(n)
    for order in (range(n), range(n - 1, -1, -1)):
        for i in order:
            s = rhs[i]
            for j in range(n):
                if j != i:
                    s -= A[i, j] * x[j]
            x[i] = s / A[i, i]
    return x


@pytest.mark.parametrize("shape", [(6, 4, 3), (7, 5, 1), (5, 1, 4)])
def test_sgs_is_one_forward_backward_gauss_seidel_sweep(shape):
    """P_SGS^{-1} r (eq. Psgs) equals one textbook symmetric Gauss-Seidel iteration from
    zero on H_JGN (the identity behind eq. Psgs in Saad's Ch. 4 and 10)."""
    P = rand_problem(*shape, seed=31, alpha=0.6)
    b = smooth_field(P, 32, 0.5)
    tri = O.hessian_tridiag(P, b, True)
    H = dense_from_apply(lambda x: O.hessian_apply(P, tri, x), P.n)
    np.testing.assert_allclose(O.hessian_sparse(P, tri).toarray(), H, rtol=0, atol=1e-12 * np.abs(H).max())
    r = np.random.default_rng(33).normal(size=(P.L, P.M + 1))
    np.testing.assert_allclose(O.sgs_apply(P, tri, r).reshape(-1), _textbook_sgs_sweep(H, r.reshape(-1)),
                               rtol=1e-10, atol=1e-12)


def test_sgs_on_one_line_adds_the_diagonal_of_L_Dinv_U():
    """A single PE line: H is tridiagonal with diagonal d and off-diagonal o, and
    (L + D) D^-1 (U + D) = H + L D^-1 U is tridiagonal with o_{i-1}^2 / d_{i-1} added to
    the diagonal at i >= 1; solved here with the banded LAPACK routine."""
    P = rand_problem(23, 1, 1, seed=34, alpha=0.8)
    b = smooth_field(P, 35, 0.6)
    tri = O.hessian_tridiag(P, b, True)
    d, o = tri[0][0], tri[1][0]
    dd = d.copy()
    dd[1:] += o ** 2 / d[:-1]
    ab = np.zeros((3, P.M + 1))
    ab[0, 1:], ab[1], ab[2, :-1] = o, dd, o
    r = np.random.default_rng(36).normal(size=(1, P.M + 1))
    np.testing.assert_allclose(O.sgs_apply(P, tri, r)[0], scipy.linalg.solve_banded((1, 1), ab, r[0]),
                               rtol=1e-11, atol=1e-13)


def test_sgs_of_a_diagonal_matrix_is_jacobi():
    P = rand_problem(9, 1, 1, seed=37, alpha=0.0)
    diag = np.random.default_rng(38).uniform(0.5, 2.0, size=(1, P.M + 1))
    tri = (diag, np.zeros((1, P.M)))
    r = np.random.default_rng(39).normal(size=(1, P.M + 1))
    np.testing.assert_allclose(O.sgs_apply(P, tri, r), r / diag, rtol=1e-15)


def test_sgs_inverse_is_spd_and_its_spectrum_lies_in_0_1():
    """For SPD H, P_SGS = H + L D^-1 L' with D > 0, so P_SGS is SPD and the eigenvalues of
    P_SGS^-1 H lie in (0, 1]; a transposed factor or D in place of D^-1 breaks one of these."""
    P = rand_problem(7, 4, 3, seed=40, alpha=0.9)
    b = smooth_field(P, 41, 0.5)
    tri = O.hessian_tridiag(P, b, True)
    H = dense_from_apply(lambda x: O.hessian_apply(P, tri, x), P.n)
    Pinv = dense_from_apply(lambda x: O.sgs_apply(P, tri, x), P.n)
    np.testing.assert_allclose(Pinv, Pinv.T, rtol=0, atol=1e-12 * np.abs(Pinv).max())
    assert np.linalg.eigvalsh(0.5 * (Pinv + Pinv.T)).min() > 0
    ev = np.linalg.eigvals(Pinv @ H).real
    assert ev.min() > 0 and ev.max() <= 1 + 1e-10
    g = O.gradient(P, b, True)
    d, it, _ = O.pcg(P, tri, -g, "sgs", tol=1e-12, maxit=500)
    np.testing.assert_allclose(d.reshape(-1), np.linalg.solve(H, -g.reshape(-1)), rtol=1e-8,
                               atol=1e-10 * np.abs(d).max())


def test_armijo_accepts_sufficient_decrease_and_rejects_infeasible():
    P = rand_problem(10, 4, 2, seed=16, alpha=0.4)
    b = smooth_field(P, 8, 0.3)
    d, g, _, _ = O.gn_direction(P, b)
    J0 = O.objective(P, b)["J"]
    gTd = float(np.sum(g * d))
    lam, Jt, _ = O.armijo(P, b, d, J0, gTd)
    assert lam > 0 and Jt <= J0 + 1e-4 * lam * gTd
    # a direction that leaves the feasible set for lambda >= 1/2 is cut back
    big = np.zeros_like(b)
    big[:, 1:] = np.cumsum(np.full((P.L, P.M), 3.0 * P.hp), axis=1)   # D1 big = 3
    lam2, _, _ = O.armijo(P, np.zeros_like(b), big, O.objective(P, np.zeros_like(b))["J"], -1.0)
    assert lam2 == 0.0 or lam2 * 3.0 < 1.0


# ----------------------------------------------------------------------------- QP / b-step
def _brute_force_qp(Gd, Go, c, g, hp):
    """Enumerate every assignment (free / lower / upper) of the cells; the unique KKT point
    of the strictly convex QP is the optimum."""
    Mc = len(g)
    N = Mc + 1
    G = np.diag(Gd) + np.diag(Go, 1) + np.diag(Go, -1)
    best = None
    for assign in itertools.product((0, 1, 2), repeat=Mc):
        rows, rhs, sg = [], [], []
        for cc, a in enumerate(assign):
            if a == 0:
                continue
            row = np.zeros(N)
            row[cc], row[cc + 1] = -1 / hp, 1 / hp
            target = -1.0 - g[cc] if a == 1 else 1.0 - g[cc]
            rows.append(row)
            rhs.append(target)
            sg.append(1.0 if a == 1 else -1.0)
        k = len(rows)
        K = np.zeros((N + k, N + k))
        K[:N, :N] = G
        if k:
            A = np.array(rows)
            K[:N, N:] = -A.T * np.array(sg)[None, :]
            K[N:, :N] = A
        sol = np.linalg.solve(K, np.concatenate([-c, rhs]))
        x, lam = sol[:N], sol[N:]
        gn = g + np.diff(x) / hp
        if np.all(np.abs(gn) <= 1 + 1e-9) and np.all(lam >= -1e-9):
            val = 0.5 * x @ G @ x + c @ x
            if best is None or val < best[0] - 1e-14:
                best = (val, x)
    return best[1]


@pytest.mark.parametrize("seed", range(6))
def test_active_set_qp_matches_brute_force(seed):
    r = np.random.default_rng(100 + seed)
    Mc = 5
    hp = 0.2
    Go = r.normal(size=Mc) * 0.3
    Gd = np.abs(r.normal(size=Mc + 1)) + 1.0 + np.abs(np.pad(Go, (1, 0))) + np.abs(np.pad(Go, (0, 1)))
    g = r.uniform(-0.9, 0.9, size=Mc)
    if seed % 2 == 0:
        g[r.integers(0, Mc)] = 1.0           # start on a bound
    c = r.normal(size=Mc + 1) * 3.0          # unconstrained step far outside the box
    x, W, lam, its = O.qp_active_set(Gd, Go, c, g, hp)
    xb = _brute_force_qp(Gd, Go, c, g, hp)
    np.testing.assert_allclose(x, xb, rtol=1e-9, atol=1e-10)
    gn = g + np.diff(x) / hp
    assert np.all(np.abs(gn) <= 1 + 1e-10)
    assert np.all(lam >= -1e-12)


def test_bstep_kkt_and_vectorised_order():
    """The batched first iteration of the b-step equals the per-line active-set method,
    and every line's result satisfies the KKT conditions of its QP."""
    P = rand_problem(12, 6, 4, seed=17, alpha=0.02, amp=3.0)
    b = smooth_field(P, 9, 0.7)
    r = np.random.default_rng(18)
    z = b + 0.3 * P.hp * r.normal(size=b.shape)
    u = 0.1 * P.hp * r.normal(size=b.shape)
    rho = 50.0
    bn, nact, _ = O.bstep(P, b, z, u, rho)
    assert nact.max() > 0 and (nact == 0).any()      # both branches exercised
    for ln in range(P.L):
        x, W, lam, _ = O.bstep_line(P, b[ln], z[ln], u[ln], P.Ip[ln], P.Im[ln], rho)
        np.testing.assert_allclose(bn[ln], b[ln] + x, rtol=1e-12, atol=1e-14)
    assert np.all(np.abs(np.diff(bn, axis=1) / P.hp) <= 1 + 1e-10)


# ----------------------------------------------------------------------------- ADMM identities
def test_admm_multiplier_is_gradient_of_g_and_zstep_descent():
    """y^{k+1} = grad g(z^{k+1}) (proof of Lemma zdescent), i.e.
    rho u^{k+1} = alpha (D2'D2 + D3'D3) z^{k+1}; and the z-step lowers L_rho by at least
    (rho v / 2)|z^k - z^{k+1}|^2."""
    P = rand_problem(10, 6, 4, seed=19, alpha=0.5)
    rho = 30.0
    b, z, u = np.zeros((P.L, P.M + 1)), np.zeros((P.L, P.M + 1)), np.zeros((P.L, P.M + 1))
    for k in range(4):
        bn, _, _ = O.bstep(P, b, z, u, rho)
        zn = O.zstep(P, bn + u, rho)
        L1 = O.augmented_lagrangian(P, bn, z, u, rho)
        L2 = O.augmented_lagrangian(P, bn, zn, u, rho)
        assert L1 - L2 >= 0.5 * rho * P.v * np.sum((zn - z) ** 2) * (1 - 1e-9) - 1e-15
        un = u + bn - zn
        lhs = rho * un
        rhs = P.alpha * O.apply_laplacian_cross(P, zn)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-8, atol=1e-10 * np.abs(rhs).max())
        b, z, u = bn, zn, un


def test_admm_residuals_identities():
    """r_pri = |b - z| = |u^{k+1} - u^k|; the tolerances reduce to eps_rel times the norms
    when eps_abs = 0."""
    P = rand_problem(8, 5, 3, seed=20, alpha=0.5)
    b, z, u, rep = O.solve_admm(P, rho=20.0, max_iter=3, eps_abs=0.0, eps_rel=0.0)
    b2, z2, u2, rep2 = O.solve_admm(P, b0=None, rho=20.0, max_iter=4, eps_abs=0.0, eps_rel=0.0)
    assert math.isclose(rep2.r_pri[3], float(np.linalg.norm((u2 - u).reshape(-1))), rel_tol=1e-10)
    assert math.isclose(rep2.r_dual[3], 20.0 * P.v * float(np.linalg.norm((z2 - z).reshape(-1))),
                        rel_tol=1e-10)
    assert rep2.eps_pri[3] == 0.0 and rep2.eps_dual[3] == 0.0
    assert not rep2.converged


def test_admm_is_resumable():
    P = rand_problem(8, 5, 3, seed=21, alpha=0.5)
    b, z, u, rep = O.solve_admm(P, rho=20.0, max_iter=5, eps_abs=0.0, eps_rel=0.0)
    b1, z1, u1, _ = O.solve_admm(P, rho=20.0, max_iter=2, eps_abs=0.0, eps_rel=0.0)
    b2, z2, u2, _ = O.solve_admm(P, b0=b1, z0=z1, u0=u1, rho=20.0, max_iter=3, eps_abs=0.0,
                                 eps_rel=0.0)
    np.testing.assert_array_equal(b, b2)
    np.testing.assert_array_equal(u, u2)


# ----------------------------------------------------------------------------- 2D vs 3D
def test_2d_is_3d_with_one_slice():
    r = np.random.default_rng(22)
    M, m2 = 11, 7
    Ip, Im = r.uniform(size=(1, m2, M)), r.uniform(size=(1, m2, M))
    P2 = O.make_problem(Ip, Im, (1 / M, 1 / m2, 1.0), 0.8)
    h3 = 0.25
    P3 = O.make_problem(Ip, Im, (1 / M, 1 / m2, h3), 0.8, gamma=h3 * 1e-3)
    b = smooth_field(P2, 10, 0.5)
    for key in ("J", "D", "S", "P"):
        assert math.isclose(O.objective(P3, b)[key], h3 * O.objective(P2, b)[key], rel_tol=1e-12)
    bA, _ = O.solve_gnpcg(P2, max_iter=3, use_stopping=False)
    bB, _ = O.solve_gnpcg(P3, max_iter=3, use_stopping=False)
    np.testing.assert_allclose(bA, bB, rtol=1e-6, atol=1e-9)


# ---------------------------------------------------------------------------------------
# Adaptive penalty (Section 4.3, closing paragraph: Boyd's residual balancing, optionally
# bounded below by rho_min) and the rescale of the scaled dual
# ---------------------------------------------------------------------------------------
def _fig7_rho(name):
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    return np.loadtxt(path)[:, 1]


def test_adapt_rho_rule_cases():
    A, F = O.RHO_ADAPT, O.RHO_ADAPT_FLOOR
    assert O.adapt_rho(1e3, 11.0, 1.0, A) == 1e3 * 1.3          # primal residual dominates
    assert O.adapt_rho(1e3, 1.0, 11.0, A) == 1e3 / 1.3          # dual residual dominates
    assert O.adapt_rho(1e3, 9.0, 1.0, A) == 1e3                 # within the band mu = 10
    assert O.adapt_rho(1e3, 11.0, 1.0, O.RHO_FIXED) == 1e3
    assert O.adapt_rho(120.0, 1.0, 11.0, F) == 120.0            # 120 / 1.3 < 100: skipped
    assert O.adapt_rho(140.0, 1.0, 11.0, F) == 140.0 / 1.3
    assert O.adapt_rho(120.0, 1.0, 11.0, A) == 120.0 / 1.3      # no bound without the floor


@pytest.mark.parametrize("name,mode", [("fig7_rho_adaptive.txt", O.RHO_ADAPT),
                                       ("fig7_rho_adaptive_bounded.txt", O.RHO_ADAPT_FLOOR)])
def test_adaptive_rho_reproduces_figure7(name, mode):
    """On the coarsest level of Figure 7 every iteration asks for a decrease. From
    rho^0 = 1e6 the rule reproduces the printed sequences: divisions by tau = 1.3, and with
    rho_min = 1e2 the decrease that would go below the bound is skipped, so rho stays at
    1e6 / 1.3^35 = 102.7975... (clamping to the bound would give 100)."""
    ref = _fig7_rho(name)
    rho, seq = 1e6, []
    for _ in range(len(ref)):
        seq.append(rho)
        rho = O.adapt_rho(rho, 1.0, 100.0, mode, tau=1.3, mu=10.0, rho_min=1e2)
    np.testing.assert_allclose(seq, ref, rtol=1e-12)


def test_adaptive_admm_equals_the_unscaled_iteration():
    """The scaled iteration (eq. admmStep1-3) with u rescaled by rho_old / rho_new at every
    change of rho is the unscaled iteration (eq. UadmmStep1-3) in y = rho v u, which keeps y
    across a change of rho: b and z agree and u^k = y^k / (rho_k v) throughout."""
    from synth import generate
    v = generate(1, (20, 24, 12), 1)
    P = O.make_problem(v.Ip, v.Im, v.h, 0.5)
    its = 14
    b, z, u, rep = O.solve_admm(P, rho=10.0, max_iter=its, eps_abs=0.0, eps_rel=0.0,
                                rho_mode=O.RHO_ADAPT)
    assert len(set(rep.rho)) > 3                       # rho changed several times
    bb = np.zeros((P.L, P.M + 1))
    zz, y, rho = bb.copy(), bb.copy(), 10.0
    for k in range(its):
        assert rho == rep.rho[k]
        uk = y / (rho * P.v)                           # the b- and z-steps of eq. UadmmStep
        bb, _, _ = O.bstep(P, bb, zz, uk, rho)
        zn = O.zstep(P, bb + uk, rho)
        y = y + rho * P.v * (bb - zn)
        rp = np.linalg.norm(bb - zn)
        rd = rho * P.v * np.linalg.norm(zn - zz)
        zz = zn
        if k + 1 < its:
            rho = O.adapt_rho(rho, rp, rd, O.RHO_ADAPT)
    np.testing.assert_allclose(bb, P.lines(b), rtol=0, atol=1e-12 * np.abs(bb).max())
    np.testing.assert_allclose(zz, P.lines(z), rtol=0, atol=1e-12 * np.abs(zz).max())
    np.testing.assert_allclose(y / (rho * P.v), P.lines(u), rtol=0,
                               atol=1e-10 * np.abs(P.lines(u)).max())


# ---------------------------------------------------------------------------------------
# Corrected images and quality measures (Section 2 model relation; Section 3 discretisation)
# ---------------------------------------------------------------------------------------
def test_corrected_images_at_zero_and_integer_shifts():
    from synth import generate
    v = generate(3, (28, 20), 1)
    P = O.make_problem(v.Ip, v.Im, v.h, 1.0)
    cp, cm = O.corrected_images(P, np.zeros((P.L, P.M + 1)))
    np.testing.assert_array_equal(cp, P.Ip)
    np.testing.assert_array_equal(cm, P.Im)
    for k in (1, 3, -2):
        cp, cm = O.corrected_images(P, np.full((P.L, P.M + 1), k * P.hp))
        ref_p, ref_m = np.zeros_like(P.Ip), np.zeros_like(P.Im)
        for c in range(P.M):
            if 0 <= c + k < P.M:
                ref_p[:, c] = P.Ip[:, c + k]
            if 0 <= c - k < P.M:
                ref_m[:, c] = P.Im[:, c - k]
        np.testing.assert_allclose(cp, ref_p, rtol=0, atol=1e-12)
        np.testing.assert_allclose(cm, ref_m, rtol=0, atol=1e-12)


def test_corrected_images_converge_to_the_true_image():
    """Noise-free pairs from a known field: at the true field both corrected images
    approximate the undistorted image, with an error that falls under refinement (linear
    interpolation of the measured samples: second order)."""
    from synth import generate
    errs = []
    for m in (32, 64, 128):
        v = generate(5, (m, m), 1, noise=0.0)
        P = O.make_problem(v.Ip, v.Im, v.h, 1.0)
        cp, cm = O.corrected_images(P, v.b_true.reshape(P.L, -1))
        It = v.I_true.reshape(P.L, -1)
        errs.append(max(np.abs(cp - It).max(), np.abs(cm - It).max()))
    assert errs[0] > 2.5 * errs[1] > 2.5 * 2.5 * errs[2], errs


def test_ncc_and_quality_consistency():
    r = np.random.default_rng(0)
    x = r.normal(size=500)
    assert abs(O.ncc(x, x) - 1.0) < 1e-14
    assert abs(O.ncc(x, 3.0 * x + 2.0) - 1.0) < 1e-14
    assert abs(O.ncc(x, -x) + 1.0) < 1e-14
    from synth import generate
    v = generate(3, (16, 12, 6), 0)
    P = O.make_problem(v.Ip, v.Im, v.h, 1.0)
    b = v.b_true.reshape(P.L, -1)
    q = O.image_quality(P, b)
    assert abs(q["D"] - O.distance(P, b)) <= 1e-14 * O.distance(P, b)


# ---------------------------------------------------------------------------------------
# Multilevel strategy (Section 4.4): level sizes, restriction, prolongation
# ---------------------------------------------------------------------------------------
def test_level_sizes_reproduce_the_papers_hierarchies():
    """Section 5 (test data): three levels of 32x32, 64x64, 128x128 in 2D and of
    50x50x33, 100x100x66, 200x200x132 in 3D."""
    assert O.level_sizes(128, 128, 1, 3) == [(32, 32, 1), (64, 64, 1), (128, 128, 1)]
    assert O.level_sizes(200, 200, 132, 3) == [(50, 50, 33), (100, 100, 66), (200, 200, 132)]
    # an odd count stays while the others are still halved
    assert O.level_sizes(240, 200, 110, 4) == [(30, 25, 55), (60, 50, 55), (120, 100, 55),
                                               (240, 200, 110)]
    assert O.level_sizes(7, 9, 5, 3) == [(7, 9, 5)]


def test_restriction_keeps_constants_and_mass():
    r = np.random.default_rng(3)
    for fine, coarse in (((16, 12, 8), (8, 6, 4)), ((16, 12, 1), (8, 6, 1)), ((16, 9, 8), (8, 9, 4))):
        M, m2, m3 = fine
        x = r.normal(size=(m3, m2, M))
        c = O.restrict_cells(x, fine, coarse)
        vf = 1.0 / (M * m2 * m3)
        vc = 1.0 / (coarse[0] * coarse[1] * coarse[2])
        assert abs(c.sum() * vc - x.sum() * vf) <= 1e-12 * np.abs(x).sum() * vf
        np.testing.assert_allclose(O.restrict_cells(np.full((m3, m2, M), 2.5), fine, coarse), 2.5)


def test_prolongation_is_exact_on_linear_fields_and_keeps_feasibility():
    r = np.random.default_rng(4)
    coarse, fine = (8, 6, 4), (16, 12, 8)
    Mc, m2c, m3c = coarse
    M, m2, m3 = fine

    def lin(Mx, my, mz, a, b_, c_):
        xp = np.arange(Mx + 1) / Mx                       # PE faces
        y = (np.arange(my) + 0.5) / my                    # cell centres across
        z = (np.arange(mz) + 0.5) / mz
        return a * xp[None, None, :] + b_ * y[None, :, None] + c_ * z[:, None, None]

    bc = lin(Mc, m2c, m3c, 0.3, -0.7, 0.2)
    bf = O.prolong_faces(bc, coarse, fine)
    ref = lin(M, m2, m3, 0.3, -0.7, 0.2)
    # exact away from the transverse ends (constant extrapolation there)
    np.testing.assert_allclose(bf[1:-1, 1:-1], ref[1:-1, 1:-1], rtol=0, atol=1e-14)
    # along PE the prolongated differences repeat the coarse ones; across it is convex
    b = np.cumsum(r.normal(size=(m3c, m2c, Mc + 1)), axis=2)
    b *= 0.9 / (np.abs(np.diff(b, axis=2)).max() * Mc)
    d1c = np.abs(np.diff(b, axis=2)).max() * Mc
    pf = O.prolong_faces(b, coarse, fine)
    d1f = np.abs(np.diff(pf, axis=2)).max() * M
    assert d1f <= d1c * (1 + 1e-12)


def test_single_level_multilevel_is_plain_gn():
    from synth import generate
    v = generate(3, (20, 16), 1)
    b1, reps, sizes = O.solve_multilevel_gnpcg(v.Ip, v.Im, v.h, 0.5, levels=1, max_iter=4,
                                               use_stopping=False)
    P = O.make_problem(v.Ip, v.Im, v.h, 0.5)
    b2, rep = O.solve_gnpcg(P, max_iter=4, use_stopping=False)
    np.testing.assert_array_equal(b1, b2)
    assert reps[0].J == rep.J and reps[0].pcg_iters == rep.pcg_iters


def test_multilevel_gn_starts_each_level_from_the_prolongated_field():
    """Section 4.4: the finer level's GN starts at P b_c, so its first objective is the
    objective of the prolongated coarse result on the finer images, and GN decreases it."""
    from synth import generate
    v = generate(4, (24, 20, 8), 0)
    b, reps, sizes = O.solve_multilevel_gnpcg(v.Ip, v.Im, v.h, 0.5, levels=2, max_iter=3,
                                              use_stopping=False)
    assert sizes == [(12, 10, 4), (24, 20, 8)]
    Pf = O.make_problem(v.Ip, v.Im, v.h, 0.5)
    Pc = O.make_problem(O.restrict_cells(v.Ip, sizes[1], sizes[0]),
                        O.restrict_cells(v.Im, sizes[1], sizes[0]),
                        tuple(2.0 * x for x in v.h), 0.5)
    coarse_b = O.solve_gnpcg(Pc, max_iter=3, use_stopping=False)[0]
    start = O.prolong_faces(coarse_b, sizes[0], sizes[1])
    assert O.feasible(Pf, start)
    assert reps[1].J[0] == pytest.approx(O.objective(Pf, start, True)["J"], rel=1e-12)
    assert reps[1].J[-1] < reps[1].J[0] and reps[0].J[-1] < reps[0].J[0]


def test_admm_restart_strategies():
    """The three restarts of Section 4.4 on a coarse state: (1) prolongates b, z and u;
    (2) b0 = z0 = P b_c, u0 = 0; (3) b0 = z0 = P((b_c + z_c)/2), u0 = 0, falling back to
    b0 = P b_c when the average leaves the feasible set. Prolongation keeps a feasible b
    feasible (the fine D1 b values are convex combinations of coarse ones)."""
    from synth import generate
    v = generate(5, (16, 12, 8), 0)
    mf, mc = (16, 12, 8), (8, 6, 4)
    Pf = O.make_problem(v.Ip, v.Im, v.h, 0.5)
    r = np.random.default_rng(6)
    shape_c = (mc[2], mc[1], mc[0] + 1)
    bc = np.cumsum(r.uniform(-0.9, 0.9, size=shape_c) * (1.0 / mc[0]), axis=2)
    zc = bc + 0.01 * r.normal(size=shape_c) / mc[0]
    uc = r.normal(size=shape_c)
    hc = 1.0 / mc[0]
    assert np.abs(np.diff(bc, axis=2)).max() / hc <= 0.9
    b1, z1, u1 = O.ml_restart(Pf, 1, bc, zc, uc, mc, mf)
    assert np.abs(np.diff(b1, axis=2)).max() / Pf.hp <= np.abs(np.diff(bc, axis=2)).max() / hc + 1e-12
    assert np.abs(u1).max() > 0 and np.all(z1 != b1)
    b2, z2, u2 = O.ml_restart(Pf, 2, bc, zc, uc, mc, mf)
    np.testing.assert_array_equal(b2, b1)
    np.testing.assert_array_equal(z2, b2)
    assert not np.any(u2)
    b3, z3, u3 = O.ml_restart(Pf, 3, bc, zc, uc, mc, mf)
    np.testing.assert_allclose(z3, 0.5 * (b1 + z1), rtol=0, atol=1e-15)
    np.testing.assert_array_equal(b3, z3)
    assert not np.any(u3)
    steep = zc.copy()
    steep[..., 1:] += np.arange(1, mc[0] + 1) * 4.0 * hc     # slopes beyond 1 in z only
    b4, z4, _ = O.ml_restart(Pf, 3, bc, steep, uc, mc, mf)
    assert not O.feasible(Pf, z4)
    np.testing.assert_array_equal(b4, b1)


def test_single_level_multilevel_is_plain_admm():
    from synth import generate
    v = generate(2, (20, 16), 1)
    b1, reps, sizes = O.solve_multilevel_admm(v.Ip, v.Im, v.h, 1.0, levels=1, rho=1e3,
                                              max_iter=12, eps_abs=0.0, eps_rel=0.0)
    P = O.make_problem(v.Ip, v.Im, v.h, 1.0)
    b2, _, _, rep = O.solve_admm(P, rho=1e3, max_iter=12, eps_abs=0.0, eps_rel=0.0)
    assert sizes == [(P.M, P.m2, P.m3)]
    np.testing.assert_array_equal(b1, b2)
    assert reps[0].r_pri == rep.r_pri
