"""Checks of the synthetic generator against the distortion model it implements."""
import numpy as np
import pytest

import oracle as O
from synth import generate, to_canonical, from_canonical, batch_shapes, serving_requests


def test_canonical_round_trip():
    r = np.random.default_rng(0)
    for shape, pe in (((5, 7), 0), ((5, 7), 1), ((3, 4, 6), 0), ((3, 4, 6), 1), ((3, 4, 6), 2)):
        a = r.normal(size=shape)
        c = to_canonical(a, pe)
        assert c.shape[-1] == shape[pe] and c.ndim == 3
        np.testing.assert_array_equal(from_canonical(c, len(shape), pe), a)


@pytest.mark.parametrize("m,pe", [((48, 40), 1), ((24, 20, 16), 0), ((20, 24, 16), 2)])
def test_field_bounds_and_shapes(m, pe):
    v = generate(3, m, pe)
    M, m2, m3 = v.m
    assert v.Ip.shape == (m3, m2, M) and v.b_true.shape == (m3, m2, M + 1)
    g = np.diff(v.b_true, axis=-1) / v.h[0]
    assert np.abs(g).max() <= v.params["dmax"] + 1e-12
    assert np.abs(v.b_true).max() <= v.params["peak"] * v.h[0] * (1 + 1e-12)


def test_line_mass_is_conserved():
    """Section 1/2: the intensity modulation is the Jacobian of the 1D map, so each PE line
    of either measured image carries the mass of the undistorted line (up to quadrature)."""
    v = generate(5, (96, 64), 1, noise=0.0)
    hp = v.h[0]
    m0 = v.I_true.sum(-1) * hp
    for I in (v.Ip, v.Im):
        m1 = I.sum(-1) * hp
        assert np.abs(m1 - m0).max() <= 2e-3 * np.abs(m0).max()


def test_distance_at_truth_vanishes_under_refinement():
    """With no noise the discrete distance at the generating field is interpolation and
    quadrature error only: small against D(0) and shrinking with h."""
    ratios = []
    for m in (32, 64, 128):
        v = generate(7, (m, m), 1, noise=0.0)
        P = O.make_problem(v.Ip, v.Im, v.h, 50.0)
        ratios.append(O.distance(P, v.b_true) / O.distance(P, np.zeros(P.n)))
    assert ratios[-1] < 0.01
    assert ratios[2] < ratios[1] < ratios[0]


def test_workload_lists_are_seeded():
    a, b = batch_shapes(48), batch_shapes(48)
    assert a == b and len(a) == 48
    for _, m, pe in a:
        assert 96 <= m[0] <= 160 and 96 <= m[1] <= 160 and 48 <= m[2] <= 96 and pe in (0, 1, 2)
    s = serving_requests(20.0, 10.0)
    assert s == serving_requests(20.0, 10.0)
    assert 100 < len(s) < 320
