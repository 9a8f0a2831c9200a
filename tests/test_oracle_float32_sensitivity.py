"""How the ADMM iteration responds to float32 rounding, shown on the CPU with the oracle
(no GPU code is involved; the float32 roundings are planted into the oracle's arithmetic
here). Two effects decide what a float32 implementation can match at the full sizes:

1. The b-step matrix G = H_D + alpha v D1'D1 + rho v I (Section 4.2, the QP data) has a
   diagonal of about 2 alpha v / h^2 + rho v, and alpha v / h^2 exceeds rho v by 800 at
   128 x 128 x 64 (2900 at 240 x 200 x 110). Rounding that diagonal to float32 perturbs
   the small eigenvalues of G, which are those of the fields that are smooth along a line,
   by about 1e-4 relative; one b-step moves by ~1e-6 voxel, and the ADMM map amplifies it
   to ~1e-4..1e-3 voxel within a few iterations. One step of iterative refinement whose
   residual is formed as v J'(J x) + alpha v D1'(D1 x) + rho v x (differences first)
   removes the effect. The b-step kernels do exactly that.
2. The derivative of the linear image model (Section 3) jumps at the knots, so the b-step
   is discontinuous in b wherever a cell's displacement crosses a sample position: a
   change of the state far below one float32 rounding moves the next iterate by many
   orders of magnitude more when it carries a displacement across a knot. At full size
   some of the ~1e7 interpolated samples sit that close to a knot every few iterations,
   so two correct implementations whose states differ by float32 rounding separate by up
   to ~1e-3..1e-2 voxel at such an iteration (locally; the smoothed z and the residual
   norms hardly move) and then contract back. Whole-trajectory field comparisons at the
   full sizes therefore bound the iterate after a knot event only loosely, while single
   steps from the same state, residual histories and converged solutions are compared at
   the tight bars."""
import numpy as np
import pytest

import oracle as O
import oracle.epi_oracle as OE
from synth import generate, config_volume

F32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)


def _bstep_unconstrained(P, b, z, u, rho, mode):
    """b-step of lines without active constraints, with the matrix G in three forms:
    'exact' (float64), 'f32' (diagonal and off-diagonal rounded to float32), 'refined'
    (the float32-rounded G plus one refinement step with the structured residual)."""
    Gd, Go, c, g = OE._qp_data(P, b, z, u, rho)
    if mode == "exact":
        x = OE.thomas(Gd, Go, -c)
    else:
        x = OE.thomas(F32(Gd), F32(Go), -c)
        if mode == "refined":
            e = OE.line_eval(P, b)
            Jx = e["Jl"] * x[:, :-1] + e["Jr"] * x[:, 1:]
            JtJx = np.zeros_like(x)
            JtJx[:, :-1] += e["Jl"] * Jx
            JtJx[:, 1:] += e["Jr"] * Jx
            res = -c - (P.v * JtJx + P.alpha * P.v * OE.apply_D1tD1(P, x) + rho * P.v * x)
            x = x + OE.thomas(F32(Gd), F32(Go), res)
    gn = g + np.diff(x, axis=1) / P.hp
    assert np.abs(gn).max() < 1.0      # no line reaches the bound on this workload
    return b + x


def _admm(P, iters, mode, rho=1e3):
    b = np.zeros((P.L, P.M + 1))
    z, u = b.copy(), b.copy()
    out = []
    for _ in range(iters):
        b = _bstep_unconstrained(P, b, z, u, rho, mode)
        zn = O.zstep(P, b + u, rho)
        u = u + b - zn
        z = zn
        out.append(b)
    return out


def test_float32_diagonal_of_G_is_amplified_and_refinement_removes_it():
    v = config_volume("3d_128x128x64", 0)
    P = O.make_problem(v.Ip, v.Im, v.h, 50.0)
    assert P.alpha / P.hp ** 2 / 1e3 > 500          # alpha v / h^2 over rho v
    iters = 5
    ref = _admm(P, iters, "exact")
    err = {m: [np.abs(a - r).max() / P.hp for a, r in zip(_admm(P, iters, m), ref)]
           for m in ("f32", "refined")}
    assert max(err["f32"]) >= 1e-4, err["f32"]              # ~5e-4 voxel at iteration 2
    assert max(err["refined"]) <= 1e-8, err["refined"]
    # the unrefined error grows through the iteration: the first step is far below it
    assert err["f32"][0] < 0.1 * max(err["f32"])


def _knot_state(P, b, line, cell, offset):
    """b with the displacement of one cell placed at a sample position plus `offset`
    (index units): both faces of the cell shift by the same amount, so g = D1 b is
    unchanged there."""
    bl = b.copy()
    a = 0.5 * (bl[line, cell] + bl[line, cell + 1]) / P.hp
    shift = (np.round(a) + offset - a) * P.hp
    bl[line, cell] += shift
    bl[line, cell + 1] += shift
    return bl


def test_bstep_is_discontinuous_where_a_displacement_crosses_a_knot():
    v = generate(0, (64, 64), 1)
    P = O.make_problem(v.Ip, v.Im, v.h, 50.0)
    b, z, u, _ = O.solve_admm(P, rho=1e3, max_iter=3, eps_abs=0.0, eps_rel=0.0)
    b, z, u = (P.lines(x) for x in (b, z, u))
    # the cell whose image pair has the largest jump of the interpolation derivative
    I2 = np.abs(np.diff(P.Ip, 2, axis=1)) + np.abs(np.diff(P.Im, 2, axis=1))
    line, cell = np.unravel_index(int(np.argmax(I2)), I2.shape)
    cell += 1
    eps = 1e-9                        # index units: far below one float32 rounding of b
    resp = {}
    for where, off in (("knot", 0.0), ("between", 0.37)):
        lo = _knot_state(P, b, line, cell, off - eps)
        hi = _knot_state(P, b, line, cell, off + eps)
        bl, _, _ = OE.bstep(P, lo, z, u, 1e3)
        bh, _, _ = OE.bstep(P, hi, z, u, 1e3)
        # change of the step (the inputs differ by 2 eps h on two faces)
        resp[where] = np.abs((bh - hi) - (bl - lo)).max() / P.hp
    assert resp["between"] <= 1e-6, resp            # continuous: of the order of eps
    assert resp["knot"] >= 1e3 * max(resp["between"], 1e-12), resp
    assert resp["knot"] >= 1e-5, resp
