"""Pins of the oracle's smoothed cubic B-spline image model (the comparison model of
Section 5; its definition is read from the image-registration literature the paper cites):
the basis and its curvature Gram matrix against brute-force quadrature, interpolation at
the samples, exact reproduction of cubic polynomials away from the ends, the derivative by
finite differences, optimality of the smoothed fit against a quadrature of its objective,
and the objective and gradient of the problem with this model by finite differences."""
import numpy as np
import pytest

import oracle as O
import oracle.epi_oracle as OE


def _quad(f, lo, hi, n=400001):
    x = np.linspace(lo, hi, n)
    y = f(x)
    return float(np.sum((y[1:] + y[:-1]) * 0.5) * (x[1] - x[0]))


def test_basis_partition_of_unity_and_support():
    t = np.linspace(-3.0, 3.0, 6001)
    assert np.all(OE.bspline3(t[np.abs(t) >= 2.0]) == 0.0)
    s = np.linspace(0.0, 1.0, 101)
    tot = sum(OE.bspline3(s - k) for k in range(-3, 5))
    np.testing.assert_allclose(tot, 1.0, rtol=0, atol=1e-15)
    # the derivatives by finite differences
    h = 1e-6
    tt = np.linspace(-2.2, 2.2, 441) + 0.0123
    np.testing.assert_allclose(OE.bspline3_d1(tt), (OE.bspline3(tt + h) - OE.bspline3(tt - h)) / (2 * h),
                               rtol=0, atol=1e-8)
    np.testing.assert_allclose(OE.bspline3_d2(tt), (OE.bspline3_d1(tt + h) - OE.bspline3_d1(tt - h)) / (2 * h),
                               rtol=0, atol=1e-6)


def test_curvature_gram_against_quadrature():
    G = OE.spline_curvature_gram(9)
    for d in range(6):
        q = _quad(lambda x: OE.bspline3_d2(x) * OE.bspline3_d2(x - d), -3.0, 3.0 + d)
        assert abs(G[2, 2 + d] - q) <= 1e-8 if 2 + d < 9 else True, (d, q)
    np.testing.assert_allclose(G, G.T)
    assert np.all(np.linalg.eigvalsh(G) >= -1e-12)      # positive semidefinite


def test_interpolation_at_the_samples():
    rng = np.random.default_rng(3)
    T = rng.normal(size=(5, 23))
    W = OE.spline_coefficients(T, 0.0)
    c = np.tile(np.arange(23, dtype=float), (5, 1))
    val, _ = OE.interp_spline(W, c, 0.1)
    np.testing.assert_allclose(val, T, rtol=0, atol=1e-12)
    # outside the support the model vanishes
    far = np.array([[-2.0, -2.5, 24.0, 30.0]] * 5)
    v2, d2 = OE.interp_spline(W, far, 0.1)
    assert np.all(v2 == 0.0) and np.all(d2 == 0.0)


def test_cubic_polynomials_are_reproduced_away_from_the_ends():
    M, hp = 90, 0.02
    c = np.arange(M, dtype=float)
    p = lambda s: 0.3 - 0.02 * s + 1.5e-3 * s ** 2 - 2.0e-5 * s ** 3
    dp = lambda s: -0.02 + 3.0e-3 * s - 6.0e-5 * s ** 2
    W = OE.spline_coefficients(p(c)[None], 0.0)
    s = np.linspace(35.0, 55.0, 203)[None] + 0.0137
    val, der = OE.interp_spline(W, s, hp)
    np.testing.assert_allclose(val, p(s), rtol=0, atol=1e-12)
    np.testing.assert_allclose(der * hp, dp(s), rtol=0, atol=1e-12)


def test_derivative_by_finite_differences():
    rng = np.random.default_rng(4)
    T = rng.uniform(0.0, 1.0, size=(3, 31))
    for theta in (0.0, 0.3):
        W = OE.spline_coefficients(T, theta)
        s = rng.uniform(-2.5, 32.5, size=(3, 200))
        hp, e = 0.05, 1e-6
        _, der = OE.interp_spline(W, s, hp)
        vp, _ = OE.interp_spline(W, s + e, hp)
        vm, _ = OE.interp_spline(W, s - e, hp)
        np.testing.assert_allclose(der, (vp - vm) / (2 * e * hp), rtol=0, atol=1e-6 * np.abs(der).max())


def _fit_objective(w, T, theta):
    """|B w - T|^2 + theta * integral (I'')^2, the integral by composite Simpson on a grid
    that contains the integers (I'' of the assembled spline is linear between them, so its
    square is integrated exactly) -- independent of the banded Gram matrix."""
    M = T.size
    c = np.arange(M, dtype=float)
    Bw = sum(w[k] * OE.bspline3(c - k) for k in range(M))
    n = 8 * (M + 3)
    x = np.linspace(-2.0, M + 1.0, n + 1)
    d2 = sum(w[k] * OE.bspline3_d2(x - k) for k in range(M))
    y = d2 * d2
    wts = np.ones(n + 1)
    wts[1:-1:2], wts[2:-1:2] = 4.0, 2.0
    integral = float(np.sum(wts * y) * (x[1] - x[0]) / 3.0)
    return float(np.sum((Bw - T) ** 2)) + theta * integral


@pytest.mark.parametrize("theta", [0.05, 1.0])
def test_smoothed_fit_minimises_its_objective(theta):
    rng = np.random.default_rng(5)
    T = rng.uniform(0.0, 1.0, size=17)
    w = OE.spline_coefficients(T[None], theta)[0]
    f0 = _fit_objective(w, T, theta)
    eps = 1e-5
    for _ in range(6):
        d = rng.normal(size=w.size)
        fp, fm = _fit_objective(w + eps * d, T, theta), _fit_objective(w - eps * d, T, theta)
        # stationarity (the central difference of a quadratic is exact up to quadrature)
        assert abs(fp - fm) / (2 * eps) <= 1e-7 * (1.0 + abs(f0)), (fp - fm) / (2 * eps)
        assert fp >= f0 and fm >= f0
    # more smoothing: less curvature, larger misfit
    w2 = OE.spline_coefficients(T[None], 10 * theta)[0]
    curv = lambda ww: _fit_objective(ww, T, 1.0) - _fit_objective(ww, T, 0.0)
    assert curv(w2) < curv(w)
    assert _fit_objective(w2, T, 0.0) > _fit_objective(w, T, 0.0)


@pytest.mark.parametrize("theta", [0.0, 0.2])
def test_objective_gradient_with_the_spline_model_by_finite_differences(theta):
    from synth import generate
    v = generate(2, (28, 9, 5), 0)
    P = O.make_problem(v.Ip, v.Im, v.h, 0.7)
    O.set_image_model(P, "spline", theta)
    rng = np.random.default_rng(6)
    b = 0.4 * v.b_true.reshape(P.L, -1) + 0.05 * P.hp * rng.normal(size=(P.L, P.M + 1))
    g = O.gradient(P, b, True)
    for _ in range(5):
        d = rng.normal(size=b.shape)
        e = 1e-6 * P.hp
        fd = (O.objective(P, b + e * d, True)["J"] - O.objective(P, b - e * d, True)["J"]) / (2 * e)
        an = float(np.sum(g * d))
        assert abs(fd - an) <= 1e-6 * (abs(an) + 1e-12 * abs(O.objective(P, b)["J"])), (fd, an)


def test_spline_model_differs_from_linear_and_fits_the_truth():
    """At the generator's true field the distance of the smoothed spline model is small,
    as for the linear model (the model relation holds up to interpolation error)."""
    from synth import generate
    v = generate(0, (64, 64), 1)
    P = O.make_problem(v.Ip, v.Im, v.h, 50.0)
    bt = v.b_true.reshape(P.L, -1)
    D0_lin, Dt_lin, Dh_lin = (O.distance(P, f * bt) for f in (0.0, 1.0, 0.5))
    O.set_image_model(P, "spline", 0.0)
    D0_spl, Dt_spl, Dh_spl = (O.distance(P, f * bt) for f in (0.0, 1.0, 0.5))
    assert Dt_lin < 0.02 * D0_lin and Dt_spl < 0.02 * D0_spl
    # at b = 0 every sample point is a knot, where the interpolating spline equals the
    # linear model; between knots they differ
    assert abs(D0_spl - D0_lin) <= 1e-12 * D0_lin
    assert abs(Dh_spl - Dh_lin) > 1e-3 * Dh_lin
