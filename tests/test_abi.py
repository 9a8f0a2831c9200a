"""The C ABI library: builds for gfx950, loads without a GPU, exports what include/epi.h
declares, and the binding's structs match the header (no device call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "epi.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(epi_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("epi_setup", "epi_objective", "epi_smooth_solve", "epi_solve_gnpcg",
              "epi_solve_admm", "epi_destroy", "epi_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1607_00531_amd import epi
    lib = epi.lib()
    for n in declared_functions():
        assert hasattr(lib, n), n
    import re
    hdr = open(os.path.join(ROOT, "include", "epi.h")).read()
    declared = int(re.search(r"#define EPI_ABI_VERSION (\d+)", hdr).group(1))
    assert lib.epi_abi_version() == declared == epi.ABI_VERSION


def test_default_options_are_the_papers():
    from paper_1607_00531_amd import gn_default_opts, admm_default_opts
    g = gn_default_opts()
    assert g["max_iter"] == 10 and g["pcg_max"] == 30 and g["precond"] == "block"
    assert g["eta"] == 0.1 and g["eps_obj"] == 1e-3 and g["eps_iter"] == 1e-2 and g["eps_grad"] == 1e-2
    a = admm_default_opts()
    assert a["eps_abs"] == 0.2 and a["eps_rel"] == 0.2 and a["sqp_iters"] == 1
    # adaptive penalty constants (tau, mu, rho_min of the paper's 3D experiments)
    assert a["rho_mode"] == 0 and a["tau"] == 1.3 and a["mu"] == 10.0 and a["rho_min"] == 1e2
    # active-set cap 4 (M + 1) (0), no Lagrangian monitoring by default
    assert a["qp_max_iter"] == 0 and a["with_lagrangian"] == 0


@pytest.mark.parametrize("m,max_iter", [((240, 200, 110), 2000), ((64, 64, 1), 20),
                                        ((128, 96, 48), 40), ((17, 5, 3), 1)])
def test_batch_footprint_covers_one_slot(m, max_iter):
    """epi_batch_footprint (host arithmetic, no device call) is at least what one resident
    request occupies: its images and state (caller-owned) and the three n-float work
    arrays, the six float64 history rows and the two DCT matrices per axis that admission
    allocates."""
    from paper_1607_00531_amd import epi
    lib = epi.lib()
    lib.epi_batch_footprint.restype = ctypes.c_int64
    lib.epi_batch_footprint.argtypes = [ctypes.POINTER(epi.Grid), ctypes.c_int32]
    g = epi.Grid()
    g.ndim = 3 if m[2] > 1 else 2
    for a in range(3):
        g.m[a] = m[a]
        g.h[a] = 1.0 / m[a] if m[a] > 1 else 1.0
    g.alpha, g.beta, g.gamma, g.precision = 50.0, 10.0, 1e-3, 1
    M, m2, m3 = m
    n, N = (M + 1) * m2 * m3, M * m2 * m3
    def packed(m):
        # forward + inverse split matrices: split-bfloat16 fragments (hi and lo, steps of
        # 32 per half) or float32 fragments (4 RTh steps of 4 per half)
        ce = (m + 1) // 2
        rth = (ce + 15) // 16
        return 2 * max(2 * (2 * rth) * ((ce + 31) // 32) * 64 * 8 * 2, (2 * rth) * (4 * rth) * 64 * 4)

    need = 4 * (2 * N + 3 * n) + 3 * 4 * n + 6 * 8 * max_iter + packed(m2) + packed(m3)
    assert lib.epi_batch_footprint(ctypes.byref(g), max_iter) >= need


def test_ctypes_structs_match_header_field_order():
    from paper_1607_00531_amd import epi
    src = open(HEADER).read()
    for cname, py in (("epi_grid", epi.Grid), ("epi_terms", epi.Terms), ("epi_gn_opts", epi.GNOpts),
                      ("epi_gn_report", epi.GNReport), ("epi_admm_opts", epi.ADMMOpts),
                      ("epi_admm_report", epi.ADMMReport)):
        body = re.search(r"typedef struct \{([^{}]*)\}\s*" + cname + ";", src).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            for part in decl.split(","):
                m = re.findall(r"\*?\s*(\w+)\s*(?:\[\d+\])?\s*$", part.strip())
                fields.append(m[-1])
        assert fields == [f for f, _ in py._fields_], (cname, fields)


def test_build_flags():
    from paper_1607_00531_amd import build
    cmd = build.build_command("/tmp/x.so")
    assert "--offload-arch=gfx950" in cmd
    i = cmd.index("-packed-fp32-ops")
    assert cmd[i - 1] == "-Xclang" and cmd[i - 2] == "-target-feature"


def test_binding_rejects_host_tensors_and_layout_helpers():
    import numpy as np
    import torch
    from paper_1607_00531_amd import Problem, to_canonical, from_canonical
    from synth import to_canonical as np_canon
    a = torch.arange(5 * 7 * 3, dtype=torch.float32).reshape(5, 7, 3)
    for pe in range(3):
        c = to_canonical(a, pe)
        np.testing.assert_array_equal(c.numpy(), np_canon(a.numpy(), pe))
        assert torch.equal(from_canonical(c, 3, pe), a)
    a2 = torch.arange(20, dtype=torch.float32).reshape(4, 5)
    for pe in range(2):
        np.testing.assert_array_equal(to_canonical(a2, pe).numpy(), np_canon(a2.numpy(), pe))
    with pytest.raises(TypeError):
        Problem(torch.zeros(1, 4, 6), torch.zeros(1, 4, 6), (1.0, 1.0, 1.0), 1.0)
