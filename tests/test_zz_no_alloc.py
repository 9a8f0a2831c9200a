"""epi_objective_noalloc (the entry point for callers that cannot allocate device memory)
against epi_objective on the same inputs: two calls in a row on one GPU, the second with a
smaller grid, through the C ABI. Both evaluate the same kernels with the same reduction
order, so the terms agree to the objective bar (1e-5 relative; equal in practice) and the
gradients element by element."""
import ctypes

import numpy as np
import pytest

from synth import generate
from tests.gpu_common import T, N, J_REL

pytestmark = pytest.mark.gpu


def _call_noalloc(lib, epi, v, alpha, b, with_pen, grad):
    import torch
    g = epi._grid_struct(tuple(v.Ip.shape), v.h, alpha, 10.0, 1e-3, "mixed")
    Ip, Im = T(v.Ip), T(v.Im)
    terms = torch.full((5,), float("nan"), dtype=torch.float64, device=b.device)
    lib.epi_objective_noalloc.argtypes = [ctypes.POINTER(epi.Grid)] + [ctypes.c_void_p] * 3 + \
        [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.epi_objective_noalloc.restype = ctypes.c_int
    st = lib.epi_objective_noalloc(ctypes.byref(g), Ip.data_ptr(), Im.data_ptr(), b.data_ptr(),
                                   1 if with_pen else 0, terms.data_ptr(),
                                   grad.data_ptr() if grad is not None else None, None)
    assert st == 0, lib.epi_last_error()
    torch.cuda.synchronize()
    return terms.cpu().numpy()


@pytest.mark.parametrize("with_pen", [True, False])
def test_noalloc_objective_matches_epi_objective_on_two_calls(with_pen):
    import torch
    from paper_1607_00531_amd import Problem, epi
    lib = epi.lib()
    lib.epi_last_error.restype = ctypes.c_char_p
    # the second call has the smaller grid
    for seed, m, pe, alpha in ((21, (96, 80, 40), 0, 5.0), (22, (40, 36, 10), 1, 50.0)):
        v = generate(seed, m, pe)
        b = T(0.5 * v.b_true)
        g_ref = T(np.zeros(v.b_true.shape))
        g_new = T(np.full(v.b_true.shape, np.nan))
        with Problem(T(v.Ip), T(v.Im), v.h, alpha, precision="mixed") as pr:
            ref = pr.objective(b, with_pen, grad=g_ref)
        got = _call_noalloc(lib, epi, v, alpha, b, with_pen, g_new)
        for k, key in enumerate(("J", "D", "S", "P")):
            assert abs(got[k] - ref[key]) <= J_REL * abs(ref["J"]), (key, got[k], ref[key])
        assert got[4] == (1.0 if ref["feasible"] else 0.0)
        np.testing.assert_array_equal(N(g_new), N(g_ref))


def test_noalloc_rejects_a_grid_beyond_its_scratch():
    """51,200 PE lines need more partial sums than the static scratch holds (43,688 lines):
    EPI_EINVAL with a message, decided on the host before anything is launched (the
    pointers are never dereferenced)."""
    from paper_1607_00531_amd import epi
    lib = epi.lib()
    lib.epi_last_error.restype = ctypes.c_char_p
    lib.epi_objective_noalloc.restype = ctypes.c_int
    g = epi.Grid()
    g.ndim = 3
    g.m[0], g.m[1], g.m[2] = 8, 256, 200
    for a in range(3):
        g.h[a] = 0.01
    g.alpha, g.beta, g.gamma, g.precision = 1.0, 10.0, 1e-3, 1
    p = ctypes.c_void_p(256)
    st = lib.epi_objective_noalloc(ctypes.byref(g), p, p, p, 0, p, None, None)
    assert st == epi.EPI_EINVAL
    assert b"static scratch" in lib.epi_last_error()
