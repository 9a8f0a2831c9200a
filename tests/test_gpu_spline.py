"""The smoothed cubic B-spline image model (Section 5's comparison model) on the GPU against
the FP64 oracle, through the C ABI: the coefficients (via the model's values at the
samples), the objective and its gradient, the corrected images, one ADMM iteration, GN-PCG
steps and the coarse-to-fine solvers. The images handed to both sides are the same float32
values, so the only differences are the float32 rounding of the coefficients and of the
kernels' arithmetic."""
import ctypes

import numpy as np
import pytest

import oracle as O
from synth import generate
from tests.gpu_common import (T, N, J_REL, FIELD_VOX, torch_dev, oracle_precond, precond_tol,
                               gn_step_tol)

pytestmark = pytest.mark.gpu

# 1..8 faces per lane, 2D and 3D, ragged tails, m2 = 1 lines, short lines (M = 2, 9)
SHAPES = [((32, 40), 1), ((16, 20, 12), 0), ((240, 8, 6), 0), ((20, 70, 9), 1),
          ((300, 3, 2), 0), ((350, 2, 2), 0), ((420, 2, 3), 0), ((511, 4, 3), 0),
          ((2, 9, 1), 1), ((63, 5, 4), 0), ((3, 2, 5), 0)]
THETAS = [0.0, 0.5, 20.0]


def _vol(seed, shape, pe):
    """The seeded volume with its images rounded to float32 (what the GPU receives)."""
    v = generate(seed, shape, pe)
    v.Ip = v.Ip.astype(np.float32).astype(np.float64)
    v.Im = v.Im.astype(np.float32).astype(np.float64)
    return v


def _oracle(v, alpha, theta, beta=10.0):
    return O.set_image_model(O.make_problem(v.Ip, v.Im, v.h, alpha, beta), "spline", theta)


def _problem(v, alpha, theta, prec="mixed", beta=10.0):
    from paper_1607_00531_amd import Problem
    return Problem(T(v.Ip), T(v.Im), v.h, alpha, beta=beta, precision=prec,
                   image_model="spline", theta=theta)


def _smooth_field(P, seed, gmax):
    r = np.random.default_rng(seed)
    b = np.cumsum(r.normal(size=(P.L, P.M + 1)), axis=1)
    b -= b.mean(axis=1, keepdims=True)
    g = np.diff(b, axis=1) / P.hp
    return b * (gmax / np.abs(g).max())


def _scale(P):
    """Largest model value magnitude: the coefficients bound |I| by max|w|."""
    return max(np.abs(P.Wp).max(), np.abs(P.Wm).max(), np.abs(P.Ip).max(), 1e-30)


def _grad_scale(P, b):
    """Magnitude of the terms whose sum is the distance gradient, v (|J_l| + |J_r|)
    (|I+| + |I-|): float32 rounding of the residual shows on this scale, and it dominates
    where smoothing makes the two corrected images nearly equal and the gradient small."""
    e = O.line_eval(P, b)
    return P.v * np.max(np.abs(e["Jl"]) + np.abs(e["Jr"])) * np.max(np.abs(e["ipv"]) + np.abs(e["imv"]))


@pytest.mark.parametrize("shape,pe", SHAPES)
def test_interpolating_spline_reproduces_the_samples(shape, pe):
    """theta = 0: at b = 0 the corrected images are the model's values at the cell centres,
    which the interpolating spline makes equal to the samples (B w = T), independently of
    the oracle."""
    import torch
    v = _vol(5, shape, pe)
    with _problem(v, 0.5, 0.0) as pr:
        outp = torch.zeros(pr.shape_cells, device=torch_dev())
        outm = torch.zeros_like(outp)
        pr.corrected_images(T(np.zeros(pr.shape_faces)), outp, outm)
        scale = max(np.abs(v.Ip).max(), np.abs(v.Im).max())
        assert np.abs(N(outp) - v.Ip).max() <= 2e-6 * scale
        assert np.abs(N(outm) - v.Im).max() <= 2e-6 * scale


@pytest.mark.parametrize("theta", THETAS)
@pytest.mark.parametrize("shape,pe", SHAPES)
def test_spline_corrected_images(shape, pe, theta):
    import torch
    v = _vol(2, shape, pe)
    P = _oracle(v, 0.7, theta)
    with _problem(v, 0.7, theta) as pr:
        for bb in (np.zeros((P.L, P.M + 1)), v.b_true.reshape(P.L, -1), _smooth_field(P, 3, 0.6)):
            outp = torch.zeros(pr.shape_cells, device=torch_dev())
            outm = torch.zeros_like(outp)
            q = pr.corrected_images(T(bb.reshape(pr.shape_faces)), outp, outm)
            cp, cm = O.corrected_images(P, bb)
            assert np.abs(N(outp).reshape(P.L, -1) - cp).max() <= 1e-5 * _scale(P)
            assert np.abs(N(outm).reshape(P.L, -1) - cm).max() <= 1e-5 * _scale(P)
            qo = O.image_quality(P, bb)
            assert abs(q["D"] - qo["D"]) <= J_REL * qo["D"] + 1e-30
            assert abs(q["ncc"] - qo["ncc"]) <= 1e-6


@pytest.mark.parametrize("theta", THETAS)
@pytest.mark.parametrize("shape,pe", SHAPES)
def test_spline_objective_and_gradient(shape, pe, theta):
    v = _vol(2, shape, pe)
    P = _oracle(v, 0.7, theta)
    with _problem(v, 0.7, theta) as pr:
        for bb in (np.zeros((P.L, P.M + 1)), v.b_true.reshape(P.L, -1), _smooth_field(P, 3, 0.6)):
            for pen in (True, False):
                g = T(np.zeros(pr.shape_faces))
                t = pr.objective(T(bb.reshape(pr.shape_faces)), pen, grad=g)
                o = O.objective(P, bb, pen)
                for key in ("J", "D", "S", "P"):
                    assert abs(t[key] - o[key]) <= J_REL * max(abs(o["J"]), 1e-300), (key, t, o)
                assert t["feasible"] == o["feasible"]
                go = O.gradient(P, bb, pen).reshape(-1)
                err = np.abs(N(g).reshape(-1) - go).max()
                assert err <= 2e-4 * np.abs(go).max() + 1e-5 * _grad_scale(P, bb), \
                    (err / np.abs(go).max(), err / _grad_scale(P, bb))


@pytest.mark.parametrize("prec", ["fp32", "mixed"])
@pytest.mark.parametrize("shape,pe,alpha,theta", [((64, 64), 1, 50.0, 0.0), ((240, 8, 6), 0, 0.5, 0.5),
                                                  ((20, 70, 9), 1, 0.5, 20.0),
                                                  ((63, 6, 5), 0, 0.5, 0.0),
                                                  ((255, 3, 2), 0, 0.5, 0.5)])
def test_spline_admm_one_iteration_from_the_same_state(shape, pe, alpha, theta, prec):
    v = _vol(1, shape, pe)
    P = _oracle(v, alpha, theta)
    rho = 1e3
    b0, z0, u0, _ = O.solve_admm(P, rho=rho, max_iter=3, eps_abs=0, eps_rel=0)
    b0, z0, u0 = (P.lines(x) for x in (b0, z0, u0))
    bn, _, _ = O.bstep(P, b0, z0, u0, rho)
    zn = O.zstep(P, bn + u0, rho)
    un = u0 + bn - zn
    with _problem(v, alpha, theta, prec) as pr:
        sh = pr.shape_faces
        b, z, u = T(b0.reshape(sh)), T(z0.reshape(sh)), T(u0.reshape(sh))
        rep = pr.solve_admm(b, z, u, rho=rho, max_iter=1, eps_abs=0.0, eps_rel=0.0)
        assert rep["iters"] == 1
        for gpu, cpu in ((b, bn), (z, zn), (u, un)):
            err = np.abs(N(gpu).reshape(P.L, -1) - cpu).max() / P.hp
            assert err <= FIELD_VOX, err


@pytest.mark.parametrize("precond", ["block", "jacobi", "sgs"])
@pytest.mark.parametrize("theta", THETAS)
@pytest.mark.parametrize("shape,pe", [((32, 40), 1), ((16, 20, 12), 0), ((240, 8, 6), 0),
                                      ((511, 4, 3), 0), ((2, 9, 1), 1)])
def test_spline_precond_apply(shape, pe, theta, precond):
    """z = P^-1 r with the GN Hessian blocks of the spline model (its J_r^T J_r part uses
    the spline's derivative) against the oracle, at the float32 sensitivity bar of the
    linear model's test."""
    v = _vol(4, shape, pe)
    P = _oracle(v, 0.7, theta)
    b = _smooth_field(P, 5, 0.6)
    tri = O.hessian_tridiag(P, b, True)
    r = np.random.default_rng(6).normal(size=(P.L, P.M + 1))
    zo = oracle_precond(P, tri, r, precond)
    tol = precond_tol(P, tri, r, precond, zo)
    with _problem(v, 0.7, theta) as pr:
        sh = pr.shape_faces
        z = pr.precond_apply(T(b.reshape(sh)), T(r.reshape(sh)), precond)
        err = np.abs(N(z).reshape(P.L, -1) - zo).max() / np.abs(zo).max()
        assert err <= tol, (err, tol)


@pytest.mark.parametrize("shape,pe,alpha,theta", [((64, 64), 1, 5.0, 0.0), ((16, 20, 12), 0, 0.5, 0.5),
                                                  ((240, 8, 6), 0, 0.5, 20.0)])
def test_spline_gnpcg_steps(shape, pe, alpha, theta):
    """Each of four GN-PCG steps taken from the oracle's iterate: the objective after the
    step (within gn_step_tol, the float32 sensitivity of the step), the PCG iteration count
    and the new field. Steps from a common state, so that float32 differences of the
    directions do not accumulate along a trajectory."""
    v = _vol(1, shape, pe)
    P = _oracle(v, alpha, theta)
    with _problem(v, alpha, theta, "mixed") as pr:
        bk = np.zeros((P.L, P.M + 1))
        for k in range(4):
            b1, r1 = O.solve_gnpcg(P, bk, max_iter=1, use_stopping=False)
            b = T(bk.reshape(pr.shape_faces))
            rep = pr.solve_gnpcg(b, max_iter=1, use_stopping=0)
            tol = gn_step_tol(P, bk)
            assert abs(rep["J"][0] - r1.J[0]) <= J_REL * r1.J[0], (k, rep["J"], r1.J)
            assert abs(rep["J"][1] - r1.J[1]) <= tol, (k, rep["J"], r1.J, tol)
            assert rep["pcg_iters"] == r1.pcg_iters, (k, rep["pcg_iters"], r1.pcg_iters)
            assert np.abs(N(b).reshape(P.L, -1) - P.lines(b1)).max() / P.hp <= FIELD_VOX
            bk = P.lines(b1)


def test_spline_multilevel_gnpcg():
    from paper_1607_00531_amd import solve_multilevel_gnpcg
    v = _vol(3, (64, 48), 1)
    alpha, theta = 5.0, 0.5
    bo, reps, sizes = O.solve_multilevel_gnpcg(v.Ip, v.Im, v.h, alpha, levels=2,
                                               image_model="spline", theta=theta,
                                               max_iter=3, use_stopping=False)
    b = T(np.zeros((v.Ip.shape[0], v.Ip.shape[1], v.Ip.shape[2] + 1)))
    rep = solve_multilevel_gnpcg(T(v.Ip), T(v.Im), v.h, alpha, b, levels=2, precision="mixed",
                                 image_model="spline", theta=theta, max_iter=3, use_stopping=0)
    assert rep["iters"] == [r.iters for r in reps]
    for Jg, ro in zip(rep["J_last"], reps):
        assert abs(Jg - ro.J[-1]) <= J_REL * ro.J[0]
    assert np.abs(N(b) - bo.reshape(N(b).shape)).max() / v.h[0] <= FIELD_VOX


def test_spline_model_rejected_where_it_has_no_coefficients():
    """The batched engine and the allocation-free objective take the linear model only."""
    import torch
    from paper_1607_00531_amd import Batch, EpiError, EPI_EINVAL, EPI_ENOTSUP, epi
    v = _vol(4, (24, 20, 6), 0)
    st = [T(np.zeros((6, 20, 25))) for _ in range(3)]
    with Batch(max_slots=2) as bt:
        with pytest.raises(EpiError) as e:
            bt.admit(T(v.Ip), T(v.Im), v.h, 5.0, *st, image_model="spline", theta=0.5)
        assert e.value.status == EPI_ENOTSUP
    lib = epi.lib()
    g = epi._grid_struct(tuple(v.Ip.shape), v.h, 5.0, 10.0, 1e-3, "mixed", None, "spline", 0.5)
    terms = torch.zeros(5, dtype=torch.float64, device=torch_dev())
    lib.epi_objective_noalloc.argtypes = [ctypes.POINTER(epi.Grid)] + [ctypes.c_void_p] * 3 + \
        [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.epi_objective_noalloc.restype = ctypes.c_int
    Ip, Im = T(v.Ip), T(v.Im)
    assert lib.epi_objective_noalloc(ctypes.byref(g), Ip.data_ptr(), Im.data_ptr(),
                                     st[0].data_ptr(), 1, terms.data_ptr(), None,
                                     None) == EPI_ENOTSUP
    from paper_1607_00531_amd import Problem
    for bad in (dict(image_model="spline", theta=-1.0),):
        with pytest.raises(EpiError) as e:
            Problem(Ip, Im, v.h, 5.0, **bad)
        assert e.value.status == EPI_EINVAL


def test_spline_at_the_benchmark_size():
    """240 x 200 x 110 (the benchmark's workload) with the smoothed spline model: objective
    and gradient at the true field and at zero, and one ADMM iteration from the oracle's
    state after two, in the benchmark's mixed precision."""
    from synth import config_volume
    v = config_volume("3d_240x200x110", 0)
    v.Ip = v.Ip.astype(np.float32).astype(np.float64)
    v.Im = v.Im.astype(np.float32).astype(np.float64)
    P = _oracle(v, 50.0, 0.5)
    with _problem(v, 50.0, 0.5) as pr:
        for bb in (v.b_true.reshape(P.L, -1), np.zeros((P.L, P.M + 1))):
            g = T(np.zeros(pr.shape_faces))
            t = pr.objective(T(bb.reshape(pr.shape_faces)), True, grad=g)
            o = O.objective(P, bb, True)
            for key in ("J", "D", "S", "P"):
                assert abs(t[key] - o[key]) <= J_REL * abs(o["J"]), (key, t[key], o[key])
            go = O.gradient(P, bb, True).reshape(-1)
            err = np.abs(N(g).reshape(-1) - go).max()
            assert err <= 2e-4 * np.abs(go).max() + 1e-5 * _grad_scale(P, bb), err
        rho = 1e3
        b0, z0, u0, _ = O.solve_admm(P, rho=rho, max_iter=2, eps_abs=0, eps_rel=0)
        b0, z0, u0 = (P.lines(x) for x in (b0, z0, u0))
        bn, _, _ = O.bstep(P, b0, z0, u0, rho)
        zn = O.zstep(P, bn + u0, rho)
        un = u0 + bn - zn
        sh = pr.shape_faces
        b, z, u = T(b0.reshape(sh)), T(z0.reshape(sh)), T(u0.reshape(sh))
        rep = pr.solve_admm(b, z, u, rho=rho, max_iter=1, eps_abs=0.0, eps_rel=0.0)
        assert rep["iters"] == 1
        for gpu, cpu in ((b, bn), (z, zn), (u, un)):
            err = np.abs(N(gpu).reshape(P.L, -1) - cpu).max() / P.hp
            print(f"one spline ADMM step at 240x200x110: {err:.2e} voxel")
            assert err <= FIELD_VOX, err
