"""Plain float64 NumPy implementation of the discretised problem and both solvers.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Layout. Every array is canonical: the phase-encoding (PE) axis is the last numpy axis and
is contiguous. Images (cells) have shape (m3, m2, M); the field b lives on the PE faces,
shape (m3, m2, M + 1) (Section 3: b is sampled on the x1-faces, here x1 = PE axis). A 2D
problem is the case m3 = 1, h3 = 1, so that the cell volume v = h_p h2 h3 is the paper's
h^3 (h^2 in 2D). Internally the solvers work on "lines" (one PE line per row):
images (L, M), faces (L, M + 1), L = m2 * m3, line index = j + m2 * k.

Readings of the paper adopted here (each one also listed in the design notes):
  * image model: linear interpolation along the PE axis of the cell-centred samples with
    zero outside the M samples; derivative from the segment chosen by floor() (the
    right-hand segment at a knot), zero outside [-1, M) in index units;
  * the gradient of the penalty is beta v D1^T phi'(D1 b) (D1^T: dimensions force it);
  * the QP gradient uses alpha v D1^T D1 b^k (gradient of (alpha v / 2)|D1 b|^2);
  * P_block = H_D + alpha v (D1^T D1 + M) + Hess(P) + gamma I with M = diag(D2^T D2 + D3^T D3);
  * P_SGS splits H_JGN into strictly lower / diagonal / strictly upper parts in the face
    order i + (M+1)(j + m2 k), the paper's x1-fastest order with x1 the PE axis;
  * gamma is used unscaled;
  * the step size of GN is chosen by Armijo backtracking (c1 = 1e-4, halving, at most
    ``ls_max`` trials) with an infeasible trial point counting as +inf;
  * PCG starts from 0, stops on the recursively updated residual, at most ``pcg_max``;
  * the ADMM b-step takes ``sqp_iters`` linearisations (default 1) of f at b^k and solves
    each QP in the step x (constraints -1 <= D1 (b^k + x) <= 1) by the primal active-set
    method with the Schur-complement KKT solve; a PE line is one "block";
  * the ADMM tolerances use the newest iterates (b^{k+1}, z^{k+1}, u^{k+1}).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

__all__ = [
    "Problem", "make_problem",
    "interp_linear", "line_eval", "distance", "reg_S", "penalty_P",
    "phi", "dphi", "d2phi",
    "objective", "gradient", "hessian_tridiag", "apply_laplacian_cross", "apply_D1tD1",
    "hessian_apply", "pblock_tridiag", "jacobi_diag", "thomas",
    "hessian_sparse", "sgs_apply",
    "pcg", "gn_direction", "armijo", "solve_gnpcg", "GNReport",
    "dct_matrix", "dct_eigs", "zstep", "qp_active_set", "bstep_line", "bstep",
    "admm_residuals", "solve_admm", "ADMMReport", "augmented_lagrangian",
    "adapt_rho", "RHO_FIXED", "RHO_ADAPT", "RHO_ADAPT_FLOOR",
    "corrected_images", "ncc", "image_quality",
    "coarse_count", "level_sizes", "restrict_cells", "prolong_faces", "feasible",
    "solve_multilevel_admm", "solve_multilevel_gnpcg", "ml_restart",
    "ML_RESTART_PROLONG_ALL", "ML_RESTART_FINE_B", "ML_RESTART_AVERAGE",
    "dense_operators",
    "bspline3", "bspline3_d1", "bspline3_d2", "spline_collocation", "spline_curvature_gram",
    "spline_coefficients", "interp_spline", "set_image_model",
]


# ---------------------------------------------------------------------------------------
# Problem data (Section 3)
# ---------------------------------------------------------------------------------------
@dataclass
class Problem:
    Ip: np.ndarray   # (L, M) image with PE direction +v, lines as rows
    Im: np.ndarray   # (L, M) image with PE direction -v
    M: int
    m2: int
    m3: int
    hp: float
    h2: float
    h3: float
    alpha: float
    beta: float = 10.0
    gamma: float = 1e-3
    # image model: "linear" (Section 3) or "spline" (the smoothed cubic B-spline model of the
    # comparison in Section 5) with smoothing weight theta and coefficients Wp, Wm (L, M)
    model: str = "linear"
    theta: float = 0.0
    Wp: Optional[np.ndarray] = None
    Wm: Optional[np.ndarray] = None

    @property
    def L(self) -> int:
        return self.m2 * self.m3

    @property
    def v(self) -> float:
        """Cell volume (the paper's h^3; h^2 in 2D)."""
        return self.hp * self.h2 * self.h3

    @property
    def n(self) -> int:
        return (self.M + 1) * self.L

    def lines(self, b: np.ndarray) -> np.ndarray:
        return np.asarray(b, dtype=np.float64).reshape(self.L, self.M + 1)

    def vol(self, b_lines: np.ndarray) -> np.ndarray:
        return np.asarray(b_lines).reshape(self.m3, self.m2, self.M + 1)


def make_problem(Ip, Im, h, alpha, beta=10.0, gamma=1e-3) -> Problem:
    """Ip, Im canonical (m3, m2, M); h = (h_p, h2, h3)."""
    Ip = np.asarray(Ip, dtype=np.float64)
    Im = np.asarray(Im, dtype=np.float64)
    if Ip.ndim == 2:
        Ip, Im = Ip[None], Im[None]
    m3, m2, M = Ip.shape
    return Problem(Ip.reshape(m2 * m3, M).copy(), Im.reshape(m2 * m3, M).copy(), M, m2, m3,
                   float(h[0]), float(h[1]), float(h[2]), float(alpha), float(beta),
                   float(gamma))


# ---------------------------------------------------------------------------------------
# Image model and residual (Section 3: the distance term and the residual Jacobian)
# ---------------------------------------------------------------------------------------
def interp_linear(T: np.ndarray, s: np.ndarray, hp: float):
    """Linear interpolation of cell-centred samples T (rows = lines) at index coordinates s.

    Sample c sits at index coordinate c. With k = floor(s), f = s - k the value is
    (1 - f) T_k + f T_{k+1}, with T_{-1} = T_M = 0, and 0 whenever k < -1 or k > M - 1.
    The derivative with respect to the physical coordinate is (T_{k+1} - T_k) / h_p on the
    same segment (0 outside)."""
    Lr, M = T.shape
    Tp = np.zeros((Lr, M + 2))
    Tp[:, 1:M + 1] = T
    k = np.floor(s)
    f = s - k
    inside = (k >= -1) & (k <= M - 1)
    ki = np.where(inside, k, -1).astype(np.int64) + 1   # column of T_k in the padded row
    rows = np.arange(Lr)[:, None]
    t0 = Tp[rows, ki]
    t1 = Tp[rows, ki + 1]
    val = np.where(inside, (1.0 - f) * t0 + f * t1, 0.0)
    der = np.where(inside, (t1 - t0) / hp, 0.0)
    return val, der


# ---------------------------------------------------------------------------------------
# Smoothed cubic B-spline image model (Section 5: the default of the comparison method,
# whose definition the paper leaves to the image-registration literature). Readings:
#   * the model is one-dimensional along PE, per line, like the linear one;
#   * I(s) = sum_k w_k beta3(s - k) in index units (sample c at s = c), coefficients on
#     the M sample positions and zero outside them (compact support, as for the linear
#     model), so I vanishes for s <= -2 and s >= M + 1;
#   * w minimises |B w - T|^2 + theta w' G w with B the collocation matrix at the samples
#     (B[c, k] = beta3(c - k)) and G the Gram matrix of the second derivatives
#     (G[k, l] = integral of beta3''(s - k) beta3''(s - l) ds), so w solves
#     (B'B + theta G) w = B'T; theta = 0 is plain spline interpolation, B w = T;
#   * I'(x) = sum_k w_k beta3'(s - k) / h_p.
# ---------------------------------------------------------------------------------------
def bspline3(t):
    """Cubic B-spline: 2/3 - t^2 + |t|^3 / 2 on |t| < 1, (2 - |t|)^3 / 6 on 1 <= |t| < 2."""
    a = np.abs(t)
    return np.where(a < 1.0, 2.0 / 3.0 - a * a + 0.5 * a ** 3,
                    np.where(a < 2.0, (2.0 - a) ** 3 / 6.0, 0.0))


def bspline3_d1(t):
    """First derivative of bspline3."""
    a = np.abs(t)
    sg = np.sign(t)
    return np.where(a < 1.0, -2.0 * t + 1.5 * t * a, np.where(a < 2.0, -0.5 * sg * (2.0 - a) ** 2, 0.0))


def bspline3_d2(t):
    """Second derivative of bspline3 (piecewise linear)."""
    a = np.abs(t)
    return np.where(a < 1.0, -2.0 + 3.0 * a, np.where(a < 2.0, 2.0 - a, 0.0))


def spline_collocation(M: int) -> np.ndarray:
    """B[c, k] = beta3(c - k) for samples and coefficients 0..M-1 (dense, for clarity)."""
    c = np.arange(M, dtype=np.float64)
    return bspline3(c[:, None] - c[None, :])


def spline_curvature_gram(M: int) -> np.ndarray:
    """G[k, l] = integral over the real line of beta3''(s - k) beta3''(s - l) ds. beta3''
    is linear on every unit interval, so Simpson's rule on each interval is exact."""
    G = np.zeros((M, M))
    for d in range(4):
        m = np.arange(-2, 2)          # the intervals [m, m + 1] that can carry both supports
        lo, mid, hi = m.astype(float), m + 0.5, m + 1.0
        f = lambda x: bspline3_d2(x) * bspline3_d2(x - d)
        val = float(np.sum((f(lo) + 4.0 * f(mid) + f(hi)) / 6.0))
        idx = np.arange(M - d)
        G[idx, idx + d] = val
        G[idx + d, idx] = val
    return G


def spline_coefficients(T: np.ndarray, theta: float) -> np.ndarray:
    """Coefficients w (rows = lines) of the smoothed fit to the samples T."""
    import scipy.linalg as sla
    L_, M = T.shape
    B = spline_collocation(M)
    if theta == 0.0:
        ab = np.zeros((3, M))
        ab[0, 1:] = np.diag(B, 1)
        ab[1] = np.diag(B)
        ab[2, :-1] = np.diag(B, -1)
        return sla.solve_banded((1, 1), ab, T.T).T
    A = B.T @ B + theta * spline_curvature_gram(M)
    ab = np.zeros((4, M))            # upper form of a symmetric band of half-width 3
    for d in range(4):
        ab[3 - d, d:] = np.diag(A, d)
    return sla.solveh_banded(ab, (T @ B).T).T


def interp_spline(W: np.ndarray, s: np.ndarray, hp: float):
    """Value and physical derivative of the spline with coefficients W (rows = lines) at
    index coordinates s: the four coefficients k - 1 .. k + 2 around k = floor(s)."""
    Lr, M = W.shape
    Wp = np.zeros((Lr, M + 6))
    Wp[:, 3:M + 3] = W                 # column of coefficient k: k + 3
    k = np.floor(s)
    f = s - k
    inside = (k >= -3) & (k <= M + 1)
    ki = np.where(inside, k, -3).astype(np.int64)
    rows = np.arange(Lr)[:, None]
    val = np.zeros_like(s)
    der = np.zeros_like(s)
    for i in range(-1, 3):
        col = np.clip(ki + i + 3, 0, M + 5)
        w = Wp[rows, col]
        val = val + w * bspline3(f - i)
        der = der + w * bspline3_d1(f - i)
    return np.where(inside, val, 0.0), np.where(inside, der / hp, 0.0)


def set_image_model(P: Problem, model: str, theta: float = 0.0) -> Problem:
    """Switch P to the linear or the smoothed cubic-spline image model (in place)."""
    if model == "linear":
        P.model, P.theta, P.Wp, P.Wm = "linear", 0.0, None, None
    elif model == "spline":
        P.model, P.theta = "spline", float(theta)
        P.Wp = spline_coefficients(P.Ip, P.theta)
        P.Wm = spline_coefficients(P.Im, P.theta)
    else:
        raise ValueError(f"unknown image model {model!r}")
    return P


def _interp(P: Problem, which: str, s: np.ndarray):
    if P.model == "spline":
        return interp_spline(P.Wp if which == "+" else P.Wm, s, P.hp)
    return interp_linear(P.Ip if which == "+" else P.Im, s, P.hp)


def line_eval(P: Problem, b: np.ndarray) -> Dict[str, np.ndarray]:
    """Per-cell quantities of the distance term at b (faces, any shape with n entries).

    a = A1 b (average of the two faces of a cell), g = D1 b (short difference),
    sample points x_c +/- a_c, i.e. index coordinates c +/- a_c / h_p,
    r = I+(x + A b)(1 + D1 b) - I-(x - A b)(1 - D1 b),
    and the two nonzeros of each row of the residual Jacobian: with
    Sd = I+'(.)(1 + g) + I-'(.)(1 - g) and Tv = I+(.) + I-(.),
    dr_c/db_c = Sd/2 - Tv/h_p and dr_c/db_{c+1} = Sd/2 + Tv/h_p."""
    bl = P.lines(b)
    a = 0.5 * (bl[:, :-1] + bl[:, 1:])
    g = (bl[:, 1:] - bl[:, :-1]) / P.hp
    c = np.arange(P.M, dtype=np.float64)[None, :]
    ipv, ipd = _interp(P, "+", c + a / P.hp)
    imv, imd = _interp(P, "-", c - a / P.hp)
    r = ipv * (1.0 + g) - imv * (1.0 - g)
    Sd = ipd * (1.0 + g) + imd * (1.0 - g)
    Tv = ipv + imv
    return dict(a=a, g=g, r=r, Jl=0.5 * Sd - Tv / P.hp, Jr=0.5 * Sd + Tv / P.hp,
                ipv=ipv, imv=imv, ipd=ipd, imd=imd)


def corrected_images(P: Problem, b):
    """The two distortion-corrected images of the model relation (Section 2, eq. (1) and
    its discretisation eq. D): I+(x + A b)(1 + D1 b) and I-(x - A b)(1 - D1 b) at the cell
    centres, each (L, M). They coincide at a perfect field; r is their difference."""
    e = line_eval(P, b)
    return e["ipv"] * (1.0 + e["g"]), e["imv"] * (1.0 - e["g"])


def ncc(x, y) -> float:
    """Normalised cross-correlation of two images (sums over all cells)."""
    x = np.asarray(x, np.float64).ravel()
    y = np.asarray(y, np.float64).ravel()
    xc, yc = x - x.mean(), y - y.mean()
    return float(np.dot(xc, yc) / math.sqrt(np.dot(xc, xc) * np.dot(yc, yc)))


def image_quality(P: Problem, b) -> Dict[str, float]:
    """SSD distance D(b) = (v/2)|I+corr - I-corr|^2 and the NCC of the corrected pair."""
    cp, cm = corrected_images(P, b)
    return dict(D=0.5 * P.v * float(np.sum((cp - cm) ** 2)), ncc=ncc(cp, cm),
                mean_plus=float(cp.mean()), mean_minus=float(cm.mean()))


def distance(P: Problem, b) -> float:
    """D(b) = (v/2) |r(b)|^2 (midpoint rule)."""
    r = line_eval(P, b)["r"]
    return 0.5 * P.v * float(np.sum(r * r))


def _diff_axes(P: Problem, b):
    bv = P.vol(P.lines(b))
    d1 = np.diff(bv, axis=2) / P.hp
    d2 = np.diff(bv, axis=1) / P.h2
    d3 = np.diff(bv, axis=0) / P.h3
    return d1, d2, d3


def reg_S(P: Problem, b) -> float:
    """S(b) = (v/2)(|D1 b|^2 + |D2 b|^2 + |D3 b|^2), short differences along each axis."""
    d1, d2, d3 = _diff_axes(P, b)
    return 0.5 * P.v * float(np.sum(d1 * d1) + np.sum(d2 * d2) + np.sum(d3 * d3))


def phi(x):
    """phi(x) = x^4 / (1 - x^2) on (-1, 1), +inf otherwise (the value at +-1 is +inf)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.full(x.shape, np.inf)
    ok = np.abs(x) < 1.0
    xo = x[ok]
    out[ok] = xo ** 4 / ((1.0 - xo) * (1.0 + xo))
    return out


def dphi(x):
    x = np.asarray(x, dtype=np.float64)
    q = (1.0 - x) * (1.0 + x)
    return (4 * x ** 3 - 2 * x ** 5) / (q * q)


def d2phi(x):
    x = np.asarray(x, dtype=np.float64)
    q = (1.0 - x) * (1.0 + x)
    return 2 * x ** 2 * (x ** 4 - 3 * x ** 2 + 6) / (q * q * q)


def penalty_P(P: Problem, b) -> float:
    """P(b) = beta v sum phi(D1 b)."""
    g = np.diff(P.lines(b), axis=1) / P.hp
    return P.beta * P.v * float(np.sum(phi(g)))


def objective(P: Problem, b, with_penalty: bool = True) -> Dict[str, float]:
    """Terms of J = D + alpha S (+ P for the penalised problem J_GN)."""
    D = distance(P, b)
    S = reg_S(P, b)
    g = np.diff(P.lines(b), axis=1) / P.hp
    feasible = bool(np.all(np.abs(g) < 1.0)) if with_penalty else bool(np.all(np.abs(g) <= 1.0))
    Pv = penalty_P(P, b) if with_penalty else 0.0
    return dict(J=D + P.alpha * S + Pv, D=D, S=S, P=Pv, feasible=feasible)


# ---------------------------------------------------------------------------------------
# Derivatives (Section 3, gradients and approximate Hessians)
# ---------------------------------------------------------------------------------------
def _D1t(w: np.ndarray, hp: float) -> np.ndarray:
    """D1^T w for per-cell w (L, M) -> faces (L, M + 1)."""
    out = np.zeros((w.shape[0], w.shape[1] + 1))
    out[:, :-1] -= w / hp
    out[:, 1:] += w / hp
    return out


def _lap_axis(x: np.ndarray, axis: int, h: float) -> np.ndarray:
    """D~^T D~ x along one axis (short differences, Neumann ends)."""
    d = np.diff(x, axis=axis) / h
    out = np.zeros_like(x)
    sl_lo = [slice(None)] * x.ndim
    sl_hi = [slice(None)] * x.ndim
    sl_lo[axis] = slice(0, -1)
    sl_hi[axis] = slice(1, None)
    out[tuple(sl_lo)] -= d / h
    out[tuple(sl_hi)] += d / h
    return out


def apply_D1tD1(P: Problem, x) -> np.ndarray:
    return _lap_axis(P.lines(x), 1, P.hp)


def apply_laplacian_cross(P: Problem, x) -> np.ndarray:
    """(D2^T D2 + D3^T D3) x as lines (L, M + 1)."""
    xv = P.vol(P.lines(x))
    out = _lap_axis(xv, 1, P.h2) + _lap_axis(xv, 0, P.h3)
    return out.reshape(P.L, P.M + 1)


def gradient(P: Problem, b, with_penalty: bool = True) -> np.ndarray:
    """grad J = v J_r^T r + alpha v (D1'D1 + D2'D2 + D3'D3) b (+ beta v D1^T phi'(D1 b))."""
    bl = P.lines(b)
    e = line_eval(P, bl)
    gD = np.zeros_like(bl)
    gD[:, :-1] += P.v * e["Jl"] * e["r"]
    gD[:, 1:] += P.v * e["Jr"] * e["r"]
    gS = P.v * (apply_D1tD1(P, bl) + apply_laplacian_cross(P, bl))
    out = gD + P.alpha * gS
    if with_penalty:
        out = out + P.beta * P.v * _D1t(dphi(e["g"]), P.hp)
    return out


def hessian_tridiag(P: Problem, b, with_penalty: bool = True, rho: float = 0.0,
                    with_gamma: bool = True):
    """Tridiagonal line blocks of H_D + alpha v D1'D1 (+ Hess P) (+ gamma I) (+ rho v I).

    Returns (diag (L, M+1), off (L, M)) where off[:, c] couples faces c and c+1."""
    bl = P.lines(b)
    e = line_eval(P, bl)
    diag = np.zeros_like(bl)
    diag[:, :-1] += P.v * e["Jl"] ** 2
    diag[:, 1:] += P.v * e["Jr"] ** 2
    off = P.v * e["Jl"] * e["Jr"]
    q = np.full_like(e["g"], P.alpha * P.v / P.hp ** 2)
    if with_penalty:
        q = q + P.beta * P.v * d2phi(e["g"]) / P.hp ** 2
    diag[:, :-1] += q
    diag[:, 1:] += q
    off = off - q
    if with_gamma:
        diag = diag + P.gamma
    if rho:
        diag = diag + rho * P.v
    return diag, off


def _cross_diag(P: Problem) -> np.ndarray:
    """diag(D2^T D2 + D3^T D3) as lines."""
    cnt2 = np.zeros(P.m2)
    if P.m2 > 1:
        cnt2[:] = 2
        cnt2[0] = cnt2[-1] = 1
    cnt3 = np.zeros(P.m3)
    if P.m3 > 1:
        cnt3[:] = 2
        cnt3[0] = cnt3[-1] = 1
    dv = cnt3[:, None] / P.h3 ** 2 + cnt2[None, :] / P.h2 ** 2      # (m3, m2)
    return np.repeat(dv.reshape(-1, 1), P.M + 1, axis=1)


def hessian_apply(P: Problem, tri, x) -> np.ndarray:
    """H_JGN x = (line tridiagonal) x + alpha v (D2'D2 + D3'D3) x."""
    diag, off = tri
    xl = P.lines(x)
    y = diag * xl
    y[:, :-1] += off * xl[:, 1:]
    y[:, 1:] += off * xl[:, :-1]
    return y + P.alpha * P.v * apply_laplacian_cross(P, xl)


def pblock_tridiag(P: Problem, tri):
    """Block-Jacobi preconditioner of Section 4.1: the cross-line coupling replaced by
    its diagonal."""
    diag, off = tri
    return diag + P.alpha * P.v * _cross_diag(P), off


def jacobi_diag(P: Problem, tri) -> np.ndarray:
    diag, _ = tri
    return diag + P.alpha * P.v * _cross_diag(P)


def hessian_sparse(P: Problem, tri):
    """H_JGN as a sparse matrix over the faces in the order i + (M+1)(j + m2 k): the line
    tridiagonal blocks ``tri`` plus alpha v (D2'D2 + D3'D3), D2 and D3 assembled from their
    Kronecker definition (eq. d2d3) as sparse matrices."""
    import scipy.sparse as sp
    diag, off = tri
    nf = P.M + 1
    o = np.zeros((P.L, nf))
    o[:, :-1] = off                         # o[l, i] couples faces i and i+1 of line l
    ov = o.reshape(-1)[:-1]
    H = sp.diags([diag.reshape(-1), ov, ov], [0, 1, -1], format="csr")

    def dt(m, h):
        if m < 2:
            return sp.csr_matrix((0, m))
        return sp.diags([-np.ones(m - 1) / h, np.ones(m - 1) / h], [0, 1], shape=(m - 1, m))

    eye = lambda k: sp.identity(k, format="csr")  # noqa: E731
    D2 = sp.kron(eye(P.m3), sp.kron(dt(P.m2, P.h2), eye(nf)))
    D3 = sp.kron(dt(P.m3, P.h3), eye(P.m2 * nf))
    return (H + P.alpha * P.v * (D2.T @ D2 + D3.T @ D3)).tocsr()


def _sgs_parts(P: Problem, tri):
    import scipy.sparse as sp
    H = hessian_sparse(P, tri)
    return sp.tril(H, 0, format="csr"), H.diagonal(), sp.triu(H, 0, format="csr")


def _sgs_solve(P: Problem, parts, r) -> np.ndarray:
    import scipy.sparse.linalg as sla
    lower, dj, upper = parts                     # L + P_Jac, diag, U + P_Jac
    y = sla.spsolve_triangular(lower, P.lines(r).reshape(-1), lower=True)
    z = sla.spsolve_triangular(upper, dj * y, lower=False)
    return z.reshape(P.L, P.M + 1)


def sgs_apply(P: Problem, tri, r) -> np.ndarray:
    """z = P_SGS^{-1} r with P_SGS = (L + P_Jac) P_Jac^{-1} (U + P_Jac) (eq. Psgs): L, U
    the strictly lower and upper parts of H_JGN, P_Jac its diagonal; a forward triangular
    solve, a diagonal scaling and a backward triangular solve."""
    return _sgs_solve(P, _sgs_parts(P, tri), r)


def thomas(diag: np.ndarray, off: np.ndarray, rhs: np.ndarray) -> np.ndarray:
    """Solve symmetric tridiagonal systems row-wise (Thomas algorithm, no pivoting).
    diag (L, N), off (L, N-1), rhs (L, N) or (L, N, K)."""
    N = diag.shape[1]
    cp = np.zeros_like(diag)
    dp = np.array(rhs, dtype=np.float64, copy=True)
    extra = dp.ndim == 3
    den = diag[:, 0].copy()
    cp[:, 0] = off[:, 0] / den if N > 1 else 0.0
    dp[:, 0] = dp[:, 0] / (den[:, None] if extra else den)
    for i in range(1, N):
        den = diag[:, i] - off[:, i - 1] * cp[:, i - 1]
        if i < N - 1:
            cp[:, i] = off[:, i] / den
        o = off[:, i - 1]
        if extra:
            dp[:, i] = (dp[:, i] - o[:, None] * dp[:, i - 1]) / den[:, None]
        else:
            dp[:, i] = (dp[:, i] - o * dp[:, i - 1]) / den
    for i in range(N - 2, -1, -1):
        if extra:
            dp[:, i] -= cp[:, i][:, None] * dp[:, i + 1]
        else:
            dp[:, i] -= cp[:, i] * dp[:, i + 1]
    return dp


# ---------------------------------------------------------------------------------------
# Gauss-Newton-PCG (Section 4.1)
# ---------------------------------------------------------------------------------------
def pcg(P: Problem, tri, rhs, precond: str = "block", tol: float = 0.1, maxit: int = 30):
    """Preconditioned CG on H x = rhs from x0 = 0; stops when |r_k| <= tol |rhs| with the
    recursively updated residual, or after maxit matrix-vector products.
    Returns (x, iterations, relative residual)."""
    rhs = P.lines(rhs)
    nb = math.sqrt(float(np.sum(rhs * rhs)))
    x = np.zeros_like(rhs)
    if nb == 0.0:
        return x, 0, 0.0
    if precond == "block":
        pd, po = pblock_tridiag(P, tri)
        apply_M = lambda r: thomas(pd, po, r)  # noqa: E731
    elif precond == "jacobi":
        jd = jacobi_diag(P, tri)
        apply_M = lambda r: r / jd  # noqa: E731
    elif precond == "sgs":
        parts = _sgs_parts(P, tri)
        apply_M = lambda r: _sgs_solve(P, parts, r)  # noqa: E731
    elif precond == "none":
        apply_M = lambda r: r.copy()  # noqa: E731
    else:
        raise ValueError(precond)
    r = rhs.copy()
    z = apply_M(r)
    p = z.copy()
    rz = float(np.sum(r * z))
    it = 0
    rel = 1.0
    while it < maxit:
        q = hessian_apply(P, tri, p)
        a = rz / float(np.sum(p * q))
        x += a * p
        r -= a * q
        it += 1
        rel = math.sqrt(float(np.sum(r * r))) / nb
        if rel <= tol:
            break
        z = apply_M(r)
        rz_new = float(np.sum(r * z))
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, rel


def gn_direction(P: Problem, b, precond="block", eta=0.1, maxit=30):
    """One inexact GN direction: PCG on H_JGN(b) d = -grad J_GN(b)."""
    g = gradient(P, b, True)
    tri = hessian_tridiag(P, b, True)
    d, it, rel = pcg(P, tri, -g, precond, eta, maxit)
    return d, g, it, rel


def armijo(P: Problem, b, d, J0: float, gTd: float, c1=1e-4, ls_max=10):
    """Backtracking on J_GN: lambda = 1, 1/2, ...; accept the first trial with
    J_GN(b + lambda d) <= J_GN(b) + c1 lambda g^T d (infeasible trials are +inf).
    Returns (lambda or 0.0 on failure, J at the accepted point, trials)."""
    bl = P.lines(b)
    lam = 1.0
    for t in range(ls_max):
        bt = bl + lam * P.lines(d)
        o = objective(P, bt, True)
        Jt = o["J"] if o["feasible"] else np.inf
        if Jt <= J0 + c1 * lam * gTd:
            return lam, Jt, t + 1
        lam *= 0.5
    return 0.0, J0, ls_max


@dataclass
class GNReport:
    J: List[float] = field(default_factory=list)
    grad_norm: List[float] = field(default_factory=list)
    pcg_iters: List[int] = field(default_factory=list)
    pcg_relres: List[float] = field(default_factory=list)
    step: List[float] = field(default_factory=list)
    iters: int = 0
    converged: bool = False
    ls_failed: bool = False


def solve_gnpcg(P: Problem, b0=None, max_iter=10, precond="block", eta=0.1, pcg_max=30,
                eps_obj=1e-3, eps_iter=1e-2, eps_grad=1e-2, use_stopping=True,
                rel_grad_tol=0.0, c1=1e-4, ls_max=10):
    """Inexact Gauss-Newton on J_GN = D + alpha S + P with Armijo steps (Section 4.1).

    Stopping: all three relative tests of Section 4.1 (with J_GN at the starting point in
    the role of J_GN(0)) when ``use_stopping``, or |grad| <= rel_grad_tol |grad_0| when
    rel_grad_tol > 0, or max_iter steps."""
    b = np.zeros((P.L, P.M + 1)) if b0 is None else P.lines(b0).copy()
    rep = GNReport()
    o = objective(P, b, True)
    if not o["feasible"]:
        raise ValueError("infeasible starting guess")
    J = o["J"]
    J0 = J
    g = gradient(P, b, True)
    gn = math.sqrt(float(np.sum(g * g)))
    g0 = gn
    rep.J.append(J)
    rep.grad_norm.append(gn)
    prev = None
    for k in range(max_iter + 1):
        if prev is not None:
            Jp, bp = prev
            if use_stopping:
                c_obj = abs(J - Jp) <= eps_obj * (1.0 + abs(J0))
                c_it = math.sqrt(float(np.sum((b - bp) ** 2))) <= eps_iter * (
                    1.0 + math.sqrt(float(np.sum(bp * bp))))
                c_gr = gn <= eps_grad * (1.0 + abs(J0))
                if c_obj and c_it and c_gr:
                    rep.converged = True
                    break
        if rel_grad_tol > 0 and gn <= rel_grad_tol * g0:
            rep.converged = True
            break
        if k == max_iter:
            break
        tri = hessian_tridiag(P, b, True)
        d, it, rel = pcg(P, tri, -g, precond, eta, pcg_max)
        gTd = float(np.sum(g * d))
        lam, Jt, _ = armijo(P, b, d, J, gTd, c1, ls_max)
        rep.pcg_iters.append(it)
        rep.pcg_relres.append(rel)
        rep.step.append(lam)
        rep.iters = k + 1
        if lam == 0.0:
            rep.ls_failed = True
            break
        prev = (J, b.copy())
        b = b + lam * d
        J = Jt
        g = gradient(P, b, True)
        gn = math.sqrt(float(np.sum(g * g)))
        rep.J.append(J)
        rep.grad_norm.append(gn)
    return P.vol(b), rep


# ---------------------------------------------------------------------------------------
# ADMM (Section 4.2)
# ---------------------------------------------------------------------------------------
def dct_matrix(m: int) -> np.ndarray:
    """Orthonormal DCT-II: C[j', j] = s_j' cos(pi j' (2 j + 1) / (2 m)),
    s_0 = sqrt(1/m), s_j' = sqrt(2/m)."""
    j = np.arange(m)
    C = np.cos(np.pi * np.outer(j, 2 * j + 1) / (2.0 * m))
    C *= math.sqrt(2.0 / m)
    C[0, :] = math.sqrt(1.0 / m)
    return C


def dct_eigs(m: int, h: float) -> np.ndarray:
    """Diagonal of Lambda(m, h) with D~(m,h)^T D~(m,h) = C^T Lambda C (eq. dctdiag)."""
    j = np.arange(m)
    return (2.0 - 2.0 * np.cos(np.pi * j / m)) / (h * h)


def zstep(P: Problem, w, rho: float) -> np.ndarray:
    """z = Gt^{-1} rho v w with Gt = alpha v (D2'D2 + D3'D3) + rho v I, diagonalised by the
    2D DCT over the two non-PE axes: z = C^T diag(rho / (rho + alpha Lambda)) C w."""
    wv = P.vol(P.lines(w))
    C2, C3 = dct_matrix(P.m2), dct_matrix(P.m3)
    lam = dct_eigs(P.m3, P.h3)[:, None] + dct_eigs(P.m2, P.h2)[None, :]   # (m3, m2)
    t = np.matmul(C2[None], wv)                                           # along j
    t = np.tensordot(C3, t, axes=(1, 0))                                  # along k
    t *= (rho / (rho + P.alpha * lam))[:, :, None]
    t = np.tensordot(C3.T, t, axes=(1, 0))
    t = np.matmul(C2.T[None], t)
    return t.reshape(P.L, P.M + 1)


def _tri_solve1(diag, off, rhs):
    return thomas(diag[None], off[None], rhs[None])[0]


def qp_active_set(Gd, Go, c, gbar, hp, tol=1e-12, max_iter=None):
    """Primal active-set method for one PE line (Section 4.2, eq. qp and eq. schurasqp):

        min_x 1/2 x^T G x + c^T x  s.t.  A x >= d,
        A = [D1; -D1],  d = -1 - A b^k  (constraints -1 <= g + D1 x <= 1, g = D1 b^k).

    G is tridiagonal SPD (diag Gd, off-diagonal Go). Constraint index 2c is D1 row c
    (lower bound on cell c), 2c + 1 is -D1 row c (upper bound). Starting point x = 0 with
    the working set of constraints active at b^k. Each iteration solves the KKT system by
    the Schur complement: lambda = -(A_W G^-1 A_W^T)^-1 (A_W G^-1 gh - hh),
    p = G^-1 (A_W^T lambda + gh), gh = -c - G x, hh = d_W - A_W x.
      * p = 0 and lambda >= 0: optimal;
      * p = 0, some lambda < 0: drop the most negative one (lowest index on ties);
      * p != 0: longest step sigma <= 1 keeping feasibility, add every blocking constraint.
    Returns (x, working set (sorted constraint indices), lambda, iterations)."""
    Mc = gbar.shape[0]
    N = Mc + 1
    if max_iter is None:
        max_iter = 4 * N

    def row(i):
        a = np.zeros(N)
        cc = i // 2
        sgn = 1.0 if i % 2 == 0 else -1.0
        a[cc] = -sgn / hp
        a[cc + 1] = sgn / hp
        return a

    dvec = np.empty(2 * Mc)
    dvec[0::2] = -1.0 - gbar
    dvec[1::2] = -1.0 + gbar
    Afull = np.array([row(i) for i in range(2 * Mc)]) if Mc > 0 else np.zeros((0, N))

    def Gmul(x):
        y = Gd * x
        y[:-1] += Go * x[1:]
        y[1:] += Go * x[:-1]
        return y

    x = np.zeros(N)
    W = [i for i in range(2 * Mc) if abs(Afull[i] @ x - dvec[i]) <= tol]
    # both bounds of one cell cannot be active together
    lam = np.zeros(0)
    its = 0
    for its in range(1, max_iter + 1):
        gh = -c - Gmul(x)
        if W:
            AW = Afull[W]
            hh = dvec[W] - AW @ x
            Y = thomas(Gd[None], Go[None], AW.T[None])[0]            # G^-1 A_W^T
            S = AW @ Y
            Gig = _tri_solve1(Gd, Go, gh)
            lam = -np.linalg.solve(S, AW @ Gig - hh)
            p = _tri_solve1(Gd, Go, AW.T @ lam + gh)
        else:
            lam = np.zeros(0)
            p = _tri_solve1(Gd, Go, gh)
        if np.max(np.abs(p)) <= tol * hp:
            if lam.size == 0 or np.all(lam >= 0):
                return x, sorted(W), lam, its
            jmin = int(np.argmin(lam))      # first occurrence = lowest index on ties
            W.pop(jmin)
            continue
        Ap = Afull @ p
        Ax = Afull @ x
        sigma = 1.0
        ratios = np.full(2 * Mc, np.inf)
        inW = np.zeros(2 * Mc, dtype=bool)
        inW[W] = True
        cand = (~inW) & (Ap < 0)
        ratios[cand] = (dvec[cand] - Ax[cand]) / Ap[cand]
        rmin = float(np.min(ratios)) if Mc > 0 else np.inf
        if rmin < 1.0:
            sigma = max(rmin, 0.0)
        x = x + sigma * p
        if rmin < 1.0:
            blocking = np.nonzero(cand & (ratios <= rmin + tol))[0]
            W = sorted(set(W) | set(int(i) for i in blocking))
    return x, sorted(W), lam, its


def _qp_data(P: Problem, bl, zl, ul, rho):
    """QP data of every line at the linearisation point b^k (Section 4.2):
    c = grad D(b^k) + alpha v D1'D1 b^k + rho v (b^k - z^k + u^k),
    G = H_D(b^k) + alpha v D1'D1 + rho v I (tridiagonal per line).
    Returns (Gd (L, M+1), Go (L, M), c (L, M+1), g = D1 b^k (L, M))."""
    e = line_eval(P, bl)
    v = P.v
    gD = np.zeros_like(bl)
    gD[:, :-1] += v * e["Jl"] * e["r"]
    gD[:, 1:] += v * e["Jr"] * e["r"]
    c = gD + P.alpha * v * apply_D1tD1(P, bl) + rho * v * (bl - zl + ul)
    Gd = np.zeros_like(bl)
    Gd[:, :-1] += v * e["Jl"] ** 2
    Gd[:, 1:] += v * e["Jr"] ** 2
    q = P.alpha * v / P.hp ** 2
    Gd[:, :-1] += q
    Gd[:, 1:] += q
    Gd += rho * v
    Go = v * e["Jl"] * e["Jr"] - q
    return Gd, Go, c, e["g"]


def bstep_line(P: Problem, bl, zl, ul, ip, im, rho, tol=1e-12):
    """The QP of one PE line (QP data at b^k, then :func:`qp_active_set`)."""
    sub = Problem(ip[None], im[None], P.M, 1, 1, P.hp, P.h2, P.h3, P.alpha, P.beta, P.gamma)
    if P.model != "linear":
        set_image_model(sub, P.model, P.theta)   # line-local fit, the same as P's row
    Gd, Go, c, g = _qp_data(sub, bl[None], zl[None], ul[None], rho)
    return qp_active_set(Gd[0], Go[0], c[0], g[0], P.hp, tol)


def bstep(P: Problem, b, z, u, rho: float, sqp_iters: int = 1, tol=1e-12):
    """b^{k+1} = argmin over C of f(b) + (rho v / 2)|b - z^k + u^k|^2, one QP per PE line
    per linearisation (eq. admmStep1).

    Evaluation order only: the first active-set iteration of every line whose initial
    working set is empty is the unconstrained step p = -G^{-1} c; when that full step is
    feasible (no ratio below 1) the method stops there with x = p, so those lines are
    solved together by one batched tridiagonal solve. Every other line runs
    :func:`qp_active_set` from x = 0. Returns (b_new (L, M+1), |W| per line, QP
    iterations per line)."""
    bl = P.lines(b).copy()
    zl, ul = P.lines(z), P.lines(u)
    nact = np.zeros(P.L, dtype=np.int64)
    qits = np.zeros(P.L, dtype=np.int64)
    for _ in range(sqp_iters):
        Gd, Go, c, g = _qp_data(P, bl, zl, ul, rho)
        x = thomas(Gd, Go, -c)
        gp = np.diff(x, axis=1) / P.hp
        w0_empty = np.all((np.abs(g + 1.0) > tol) & (np.abs(g - 1.0) > tol), axis=1)
        # ratio test at x = 0: row D1 (lower) blocks when D1 p < 0, row -D1 when D1 p > 0
        with np.errstate(divide="ignore", invalid="ignore"):
            r_lo = np.where(gp < 0, (-1.0 - g) / gp, np.inf)
            r_hi = np.where(gp > 0, (1.0 - g) / gp, np.inf)
        rmin = np.minimum(r_lo, r_hi).min(axis=1) if P.M > 0 else np.full(P.L, np.inf)
        easy = w0_empty & (rmin >= 1.0)
        bnew = bl + np.where(easy[:, None], x, 0.0)
        nact[:] = 0
        qits[:] = np.where(easy, 2, 0)
        for ln in np.nonzero(~easy)[0]:
            xl, W, _, its = qp_active_set(Gd[ln], Go[ln], c[ln], g[ln], P.hp, tol)
            bnew[ln] = bl[ln] + xl
            nact[ln] = len(W)
            qits[ln] = its
        bl = bnew
    return bl, nact, qits


def augmented_lagrangian(P: Problem, b, z, u, rho: float) -> float:
    """L_rho(b, z, y) = f(b) + g(z) + y^T (b - z) + (rho v / 2)|b - z|^2, y = rho v u
    (eq. Lp; the indicator of C is 0 for the feasible iterates produced here)."""
    bl, zl, ul = P.lines(b), P.lines(z), P.lines(u)
    d1 = np.diff(bl, axis=1) / P.hp
    f = distance(P, bl) + 0.5 * P.alpha * P.v * float(np.sum(d1 * d1))
    zv = P.vol(zl)
    d2 = np.diff(zv, axis=1) / P.h2
    d3 = np.diff(zv, axis=0) / P.h3
    gz = 0.5 * P.alpha * P.v * float(np.sum(d2 * d2) + np.sum(d3 * d3))
    y = rho * P.v * ul
    return f + gz + float(np.sum(y * (bl - zl))) + 0.5 * rho * P.v * float(np.sum((bl - zl) ** 2))


def admm_residuals(P: Problem, b_new, z_new, z_old, u_new, rho, eps_abs, eps_rel):
    """Primal/dual residuals and tolerances of eq. admmStop (newest iterates)."""
    n = P.n
    nb = math.sqrt(float(np.sum(b_new * b_new)))
    nz = math.sqrt(float(np.sum(z_new * z_new)))
    nu = math.sqrt(float(np.sum(u_new * u_new)))
    r_pri = math.sqrt(float(np.sum((b_new - z_new) ** 2)))
    r_dual = rho * P.v * math.sqrt(float(np.sum((z_new - z_old) ** 2)))
    e_pri = math.sqrt(n) * eps_abs + eps_rel * max(nb, nz)
    e_dual = math.sqrt(n) * eps_abs + eps_rel * rho * P.v * nu
    return r_pri, r_dual, e_pri, e_dual


@dataclass
class ADMMReport:
    r_pri: List[float] = field(default_factory=list)
    r_dual: List[float] = field(default_factory=list)
    eps_pri: List[float] = field(default_factory=list)
    eps_dual: List[float] = field(default_factory=list)
    max_active: List[int] = field(default_factory=list)
    lagrangian: List[float] = field(default_factory=list)
    rho: List[float] = field(default_factory=list)
    iters: int = 0
    converged: bool = False


RHO_FIXED, RHO_ADAPT, RHO_ADAPT_FLOOR = 0, 1, 2


def adapt_rho(rho, r_pri, r_dual, mode, tau=1.3, mu=10.0, rho_min=1e2):
    """Residual balancing (Section 4.3, adaptive penalty; Boyd et al. Section 3.4.1):
    rho * tau if r_pri > mu r_dual, rho / tau if r_dual > mu r_pri, else unchanged. Mode
    RHO_ADAPT_FLOOR skips a decrease that would go below rho_min. Returns the new rho; the
    caller rescales the scaled dual u by rho_old / rho_new so that y = rho v u is unchanged."""
    if mode == RHO_FIXED:
        return rho
    if r_pri > mu * r_dual:
        return rho * tau
    if r_dual > mu * r_pri:
        new = rho / tau
        if mode == RHO_ADAPT_FLOOR and new < rho_min:
            return rho
        return new
    return rho


def solve_admm(P: Problem, b0=None, z0=None, u0=None, rho=1e3, max_iter=100,
               eps_abs=0.2, eps_rel=0.2, sqp_iters=1, with_lagrangian=False, tol=1e-12,
               rho_mode=RHO_FIXED, tau=1.3, mu=10.0, rho_min=1e2):
    """Scaled ADMM of Section 4.2: b-step (SQP/active set per line), z-step (DCT solve),
    u^{k+1} = u^k + b^{k+1} - z^{k+1}; stop by eq. admmStop or after max_iter. With an
    adaptive rho_mode the penalty is updated after each non-final iteration by
    :func:`adapt_rho` and u rescaled accordingly."""
    b = np.zeros((P.L, P.M + 1)) if b0 is None else P.lines(b0).copy()
    z = b.copy() if z0 is None else P.lines(z0).copy()
    u = np.zeros_like(b) if u0 is None else P.lines(u0).copy()
    g = np.diff(b, axis=1) / P.hp
    if np.any(np.abs(g) > 1.0 + 1e-12):
        raise ValueError("starting guess violates -1 <= D1 b <= 1")
    rep = ADMMReport()
    for k in range(max_iter):
        b, nact, _ = bstep(P, b, z, u, rho, sqp_iters, tol)
        z_new = zstep(P, b + u, rho)
        u = u + b - z_new
        rp, rd, ep, ed = admm_residuals(P, b, z_new, z, u, rho, eps_abs, eps_rel)
        z = z_new
        rep.r_pri.append(rp)
        rep.r_dual.append(rd)
        rep.eps_pri.append(ep)
        rep.eps_dual.append(ed)
        rep.rho.append(rho)
        rep.max_active.append(int(nact.max()) if nact.size else 0)
        if with_lagrangian:
            rep.lagrangian.append(augmented_lagrangian(P, b, z, u, rho))
        rep.iters = k + 1
        if rp <= ep and rd <= ed:
            rep.converged = True
            break
        if k + 1 < max_iter:
            new = adapt_rho(rho, rp, rd, rho_mode, tau, mu, rho_min)
            u = u * (rho / new)
            rho = new
    return P.vol(b), P.vol(z), P.vol(u), rep


# ---------------------------------------------------------------------------------------
# Multilevel strategy (Section 4.4): coarse-to-fine levels, image restriction, field
# prolongation and the ADMM restart of the third strategy. The paper defers the transfer
# operators to the image-registration literature; the readings used here: every axis with
# an even cell count of at least 4 is halved per level; images are restricted by averaging
# the fine cells of a coarse cell; the field is prolongated linearly along PE on the faces
# (even fine faces on coarse faces, odd ones at midpoints) and with the cell-centred
# weights 3/4, 1/4 across (the nearer and the farther coarse neighbour, constant at the
# ends). Along PE the prolongated field keeps the coarse D1 b values, across it is a convex
# combination of coarse lines, so a feasible coarse field stays feasible.
# ---------------------------------------------------------------------------------------
def coarse_count(m: int) -> int:
    return m // 2 if (m % 2 == 0 and m >= 4) else m


def level_sizes(M: int, m2: int, m3: int, levels: int):
    """Cell counts (M, m2, m3) of the levels, coarse to fine (fewer levels if no axis can
    be halved any more)."""
    sizes = [(M, m2, m3)]
    while len(sizes) < levels:
        a, b, c = sizes[-1]
        nxt = (coarse_count(a), coarse_count(b), coarse_count(c) if c > 1 else 1)
        if nxt == sizes[-1]:
            break
        sizes.append(nxt)
    return sizes[::-1]


def restrict_cells(x, fine, coarse):
    """Cell array (m3, m2, M) on the fine grid -> coarse grid: mean of the fine cells of
    each coarse cell (factor 1 or 2 per axis)."""
    M, m2, m3 = fine
    Mc, m2c, m3c = coarse
    v = np.asarray(x, np.float64).reshape(m3, m2, M)
    if Mc != M:
        v = 0.5 * (v[:, :, 0::2] + v[:, :, 1::2])
    if m2c != m2:
        v = 0.5 * (v[:, 0::2, :] + v[:, 1::2, :])
    if m3c != m3:
        v = 0.5 * (v[0::2] + v[1::2])
    return v


def _prolong_cc(v, axis):
    n = v.shape[axis]
    lo = np.take(v, np.r_[0, np.arange(n - 1)], axis=axis)
    hi = np.take(v, np.r_[np.arange(1, n), n - 1], axis=axis)
    shape = list(v.shape)
    shape[axis] = 2 * n
    out = np.empty(shape)
    ev = [slice(None)] * v.ndim
    od = [slice(None)] * v.ndim
    ev[axis] = slice(0, None, 2)
    od[axis] = slice(1, None, 2)
    out[tuple(ev)] = 0.75 * v + 0.25 * lo
    out[tuple(od)] = 0.75 * v + 0.25 * hi
    return out


def prolong_faces(b, coarse, fine):
    """Face array (m3c, m2c, Mc + 1) on the coarse grid -> fine grid (m3, m2, M + 1)."""
    Mc, m2c, m3c = coarse
    M, m2, m3 = fine
    v = np.asarray(b, np.float64).reshape(m3c, m2c, Mc + 1)
    if M != Mc:
        f = np.empty((m3c, m2c, M + 1))
        f[:, :, 0::2] = v
        f[:, :, 1::2] = 0.5 * (v[:, :, :-1] + v[:, :, 1:])
        v = f
    if m2 != m2c:
        v = _prolong_cc(v, 1)
    if m3 != m3c:
        v = _prolong_cc(v, 0)
    return v


def feasible(P: Problem, b, tol=1e-5) -> bool:
    """|D1 b| <= 1 (+ tol) on every cell."""
    return bool(np.all(np.abs(np.diff(P.lines(b), axis=1)) / P.hp <= 1.0 + tol))


ML_RESTART_PROLONG_ALL, ML_RESTART_FINE_B, ML_RESTART_AVERAGE = 1, 2, 3


def ml_restart(P: Problem, strategy: int, bc, zc, uc, mc, mf):
    """Starting ADMM state (b0, z0, u0) on the finer grid mf from the coarse result
    (b_c, z_c, u_c) on mc, by the three strategies of Section 4.4:
      1: b0 = P b_c, z0 = P z_c, u0 = P u_c;
      2: b0 = z0 = P b_c, u0 = 0;
      3: b0 = z0 = P((b_c + z_c) / 2), u0 = 0 -- with b0 = P b_c instead when that average
         violates |D1 b| <= 1 (z is not constrained, so the average may be infeasible).
    P = prolong_faces; P is the fine Problem (for the feasibility test)."""
    pb = prolong_faces(bc, mc, mf)
    if strategy == ML_RESTART_PROLONG_ALL:
        return pb, prolong_faces(zc, mc, mf), prolong_faces(uc, mc, mf)
    zero = np.zeros_like(pb)
    if strategy == ML_RESTART_FINE_B:
        return pb, pb.copy(), zero
    if strategy == ML_RESTART_AVERAGE:
        avg = prolong_faces(0.5 * (bc + zc), mc, mf)
        return (avg if feasible(P, avg) else pb), avg, zero
    raise ValueError(strategy)


def _ml_problems(Ip, Im, h, alpha, levels, beta, gamma, image_model="linear", theta=0.0):
    """(sizes coarse to fine, a function level -> Problem on that level's restricted images;
    every level uses the same image model, the spline one fitted to that level's images)."""
    M, m2, m3 = Ip.shape[2], Ip.shape[1], Ip.shape[0]
    sizes = level_sizes(M, m2, m3, levels)
    imgs = {sizes[-1]: (np.asarray(Ip, np.float64), np.asarray(Im, np.float64))}
    for lf, lc in zip(sizes[::-1][:-1], sizes[::-1][1:]):
        fp, fm = imgs[lf]
        imgs[lc] = (restrict_cells(fp, lf, lc), restrict_cells(fm, lf, lc))

    def problem(li):
        sz = sizes[li]
        hl = tuple(h[a] * (M, m2, m3)[a] / sz[a] for a in range(3))
        if m3 == 1:
            hl = (hl[0], hl[1], h[2])
        P = make_problem(imgs[sz][0], imgs[sz][1], hl, alpha, beta, gamma)
        return set_image_model(P, image_model, theta)

    return sizes, problem


def solve_multilevel_admm(Ip, Im, h, alpha, levels=3, beta=10.0, gamma=1e-3, rho=1e3,
                          restart=ML_RESTART_AVERAGE, image_model="linear", theta=0.0, **admm):
    """Coarse-to-fine ADMM (Section 4.4) from b = z = u = 0 on the coarsest level, the
    finer levels started by ml_restart (the paper's experiments use strategy 3). rho carries
    over between levels (the rho of the last iteration). Returns (b on the finest grid,
    per-level ADMM reports, sizes)."""
    sizes, problem = _ml_problems(Ip, Im, h, alpha, levels, beta, gamma, image_model, theta)
    reps = []
    bc = zc = uc = None
    for li, sz in enumerate(sizes):
        P = problem(li)
        if bc is None:
            b0 = z0 = u0 = np.zeros((sz[2], sz[1], sz[0] + 1))
        else:
            b0, z0, u0 = ml_restart(P, restart, bc, zc, uc, sizes[li - 1], sz)
        b, z, u, rep = solve_admm(P, b0, z0, u0, rho=rho, **admm)
        reps.append(rep)
        rho = rep.rho[-1] if rep.rho else rho
        bc, zc, uc = b, z, u
    return bc, reps, sizes


def solve_multilevel_gnpcg(Ip, Im, h, alpha, levels=3, beta=10.0, gamma=1e-3, image_model="linear",
                           theta=0.0, **gn):
    """Coarse-to-fine GN-PCG (Section 4.4): GN from b = 0 on the coarsest level, each finer
    level started from the prolongation of the coarser result (feasible: prolongation keeps
    the coarse D1 b values along PE and mixes lines convexly across). Returns (b on the
    finest grid, per-level GN reports, sizes)."""
    sizes, problem = _ml_problems(Ip, Im, h, alpha, levels, beta, gamma, image_model, theta)
    reps = []
    bc = None
    for li, sz in enumerate(sizes):
        P = problem(li)
        b0 = None if bc is None else prolong_faces(bc, sizes[li - 1], sz)
        b, rep = solve_gnpcg(P, b0, **gn)
        reps.append(rep)
        bc = b
    return bc, reps, sizes
# ---------------------------------------------------------------------------------------
def dense_operators(M: int, m2: int, m3: int, hp: float, h2: float, h3: float):
    """A1, D1, D2, D3 as dense matrices built from eq. A, eq. D1 and eq. d2d3, generalised
    to m = (M, m2, m3) cells and anisotropic h (face index = i + (M+1)(j + m2 k))."""
    def Dt(m, h):
        D = np.zeros((max(m - 1, 0), m))
        for r in range(m - 1):
            D[r, r] = -1.0 / h
            D[r, r + 1] = 1.0 / h
        return D

    def At(m):
        A = np.zeros((m, m + 1))
        for r in range(m):
            A[r, r] = A[r, r + 1] = 0.5
        return A

    I = np.eye
    A1 = np.kron(I(m2 * m3), At(M))
    D1 = np.kron(I(m2 * m3), Dt(M + 1, hp))
    D2 = np.kron(I(m3), np.kron(Dt(m2, h2), I(M + 1)))
    D3 = np.kron(Dt(m3, h3), I(m2 * (M + 1)))
    return A1, D1, D2, D3
