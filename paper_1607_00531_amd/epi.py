"""Python binding of libepi.so (ctypes): argument marshalling only.

Every step of the solvers runs in the HIP kernels of the library; this module turns torch
tensors into device pointers, option dictionaries into the C structs of ``include/epi.h``
and report arrays back into Python lists. PyTorch supplies device memory and streams.
Missing library -> ImportError; a failing call -> EpiError with the library's message.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libepi.so")

EPI_OK, EPI_EINVAL, EPI_ENOMEM, EPI_EINFEASIBLE, EPI_ENUMERIC, EPI_EHIP, EPI_ENOTSUP = range(7)
STATUS_NAMES = {0: "EPI_OK", 1: "EPI_EINVAL", 2: "EPI_ENOMEM", 3: "EPI_EINFEASIBLE",
                4: "EPI_ENUMERIC", 5: "EPI_EHIP", 6: "EPI_ENOTSUP"}
PREC = {"fp32": 0, "mixed": 1}
PRECOND = {"block": 0, "jacobi": 1, "none": 2, "sgs": 3}


class EpiError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Grid(C.Structure):
    _fields_ = [("ndim", C.c_int32), ("m", C.c_int32 * 3), ("h", C.c_double * 3),
                ("alpha", C.c_double), ("beta", C.c_double), ("gamma", C.c_double),
                ("precision", C.c_int32), ("image_model", C.c_int32), ("theta", C.c_double)]


IMAGE_MODELS = {"linear": 0, "spline": 1}


class Terms(C.Structure):
    _fields_ = [("J", C.c_double), ("D", C.c_double), ("S", C.c_double), ("P", C.c_double),
                ("feasible", C.c_int32)]


class GNOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("pcg_max", C.c_int32), ("precond", C.c_int32),
                ("ls_max", C.c_int32), ("use_stopping", C.c_int32), ("eta", C.c_double),
                ("eps_obj", C.c_double), ("eps_iter", C.c_double), ("eps_grad", C.c_double),
                ("ls_c1", C.c_double), ("rel_grad_tol", C.c_double)]


class GNReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("status", C.c_int32),
                ("ls_failed", C.c_int32), ("J", C.POINTER(C.c_double)),
                ("grad_norm", C.POINTER(C.c_double)), ("pcg_relres", C.POINTER(C.c_double)),
                ("step", C.POINTER(C.c_double)), ("pcg_iters", C.POINTER(C.c_int32))]


# penalty strategies of epi_admm_opts.rho_mode
RHO_MODES = {"fixed": 0, "adapt": 1, "adapt_floor": 2}
ABI_VERSION = 6


class ADMMOpts(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("sqp_iters", C.c_int32), ("check_every", C.c_int32),
                ("rho", C.c_double), ("eps_abs", C.c_double), ("eps_rel", C.c_double),
                ("rho_mode", C.c_int32), ("tau", C.c_double), ("mu", C.c_double),
                ("rho_min", C.c_double), ("qp_max_iter", C.c_int32),
                ("with_lagrangian", C.c_int32)]


class ADMMReport(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("status", C.c_int32),
                ("max_active", C.c_int32), ("hard_lines", C.c_int64),
                ("r_pri", C.POINTER(C.c_double)), ("r_dual", C.POINTER(C.c_double)),
                ("eps_pri", C.POINTER(C.c_double)), ("eps_dual", C.POINTER(C.c_double)),
                ("rho", C.POINTER(C.c_double)), ("lagrangian", C.POINTER(C.c_double))]


class Quality(C.Structure):
    _fields_ = [("D", C.c_double), ("ncc", C.c_double), ("mean_plus", C.c_double),
                ("mean_minus", C.c_double)]


class KernelProfile(C.Structure):
    _fields_ = [("ms", C.c_double * 8), ("launches", C.c_int64 * 8),
                ("us_isolated", C.c_double * 8), ("isolated_reps", C.c_int32)]


KERNEL_NAMES = ["bstep", "bstep_hard", "dct_axis3", "dct_axis2_fused", "dct_last_epilogue",
                "finalize"]

_lib = None


def lib():
    """Load libepi.so once (ImportError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1607_00531_amd.build")
        # torch's HIP runtime is loaded first so that libepi.so binds to that same runtime
        # (a second copy of libamdhip64 in the process sees no device).
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, st = C.c_void_p, C.c_int
        L.epi_abi_version.restype = C.c_int32
        if L.epi_abi_version() != ABI_VERSION:
            raise ImportError(f"{LIB_PATH} has ABI version {L.epi_abi_version()}, "
                              f"this binding expects {ABI_VERSION}: rebuild the library")
        L.epi_last_error.restype = C.c_char_p
        L.epi_setup.argtypes = [C.POINTER(Grid), vp, vp, vp, C.POINTER(vp)]
        L.epi_setup.restype = st
        L.epi_objective.argtypes = [vp, vp, C.c_int32, C.POINTER(Terms), vp]
        L.epi_objective.restype = st
        L.epi_smooth_solve.argtypes = [vp, vp, C.c_double, vp]
        L.epi_smooth_solve.restype = st
        L.epi_solve_gnpcg.argtypes = [vp, vp, C.POINTER(GNOpts), C.POINTER(GNReport)]
        L.epi_solve_gnpcg.restype = st
        L.epi_solve_admm.argtypes = [vp, vp, vp, vp, C.POINTER(ADMMOpts), C.POINTER(ADMMReport)]
        L.epi_solve_admm.restype = st
        L.epi_profile_admm.argtypes = [vp, vp, vp, vp, C.POINTER(ADMMOpts), C.POINTER(ADMMReport),
                                       C.POINTER(KernelProfile)]
        L.epi_profile_admm.restype = st
        L.epi_corrected_images.argtypes = [vp, vp, vp, vp, C.POINTER(Quality)]
        L.epi_corrected_images.restype = st
        L.epi_precond_apply.argtypes = [vp, vp, C.c_int32, vp, vp]
        L.epi_precond_apply.restype = st
        L.epi_destroy.argtypes = [vp]
        L.epi_destroy.restype = None
        L.epi_gn_default_opts.argtypes = [C.POINTER(GNOpts)]
        L.epi_admm_default_opts.argtypes = [C.POINTER(ADMMOpts)]
        _lib = L
    return _lib


def _check(status: int):
    if status != EPI_OK:
        raise EpiError(status, lib().epi_last_error().decode(errors="replace"))


def _ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
        raise TypeError("expected a float32 CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous (canonical layout)")
    return t.data_ptr()


def _stream_handle(stream) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def to_canonical(t, pe_axis: int):
    """Caller-order tensor (2D or 3D, cells or PE faces) -> canonical contiguous layout
    (m3, m2, M[+1]): PE axis last (contiguous), the other axes in order, m3 = 1 in 2D."""
    nd = t.dim()
    rest = [a for a in range(nd) if a != pe_axis]
    if nd == 2:
        return t.permute(rest[0], pe_axis).unsqueeze(0).contiguous()
    if nd == 3:
        return t.permute(rest[1], rest[0], pe_axis).contiguous()
    raise ValueError("2D or 3D tensors only")


def from_canonical(t, ndim: int, pe_axis: int):
    rest = [a for a in range(ndim) if a != pe_axis]
    if ndim == 2:
        order = [rest[0], pe_axis]
        inv = [order.index(a) for a in range(2)]
        return t[0].permute(*inv).contiguous()
    order = [rest[1], rest[0], pe_axis]
    inv = [order.index(a) for a in range(3)]
    return t.permute(*inv).contiguous()


def gn_default_opts() -> dict:
    o = GNOpts()
    lib().epi_gn_default_opts(C.byref(o))
    d = {k: getattr(o, k) for k, _ in GNOpts._fields_}
    d["precond"] = {v: k for k, v in PRECOND.items()}[d["precond"]]
    return d


def admm_default_opts() -> dict:
    o = ADMMOpts()
    lib().epi_admm_default_opts(C.byref(o))
    return {k: getattr(o, k) for k, _ in ADMMOpts._fields_}


class Problem:
    """A problem handle (epi_setup). Ip, Im: float32 CUDA tensors of shape (m3, m2, M) in
    canonical layout; h = (h_p, h2, h3) with h3 = 1 in 2D. The images are borrowed: they
    are kept referenced here for the lifetime of the handle."""

    def __init__(self, Ip, Im, h, alpha: float, beta: float = 10.0, gamma: float = 1e-3,
                 precision: str = "mixed", ndim: Optional[int] = None, stream=None,
                 image_model: str = "linear", theta: float = 0.0):
        if Ip.dim() != 3 or Ip.shape != Im.shape:
            raise ValueError("Ip and Im must have the same canonical shape (m3, m2, M)")
        m3, m2, M = (int(s) for s in Ip.shape)
        self.shape_cells = (m3, m2, M)
        self.shape_faces = (m3, m2, M + 1)
        self.ndim = ndim if ndim is not None else (2 if m3 == 1 else 3)
        self.h = tuple(float(x) for x in h)
        self.alpha, self.beta, self.gamma = float(alpha), float(beta), float(gamma)
        self.precision = precision
        self._Ip, self._Im = Ip, Im
        self._stream = stream
        g = Grid()
        g.ndim = self.ndim
        g.m[0], g.m[1], g.m[2] = M, m2, m3
        for a in range(3):
            g.h[a] = self.h[a]
        g.alpha, g.beta, g.gamma = self.alpha, self.beta, self.gamma
        g.precision = PREC[precision]
        self.image_model, self.theta = image_model, float(theta)
        g.image_model = IMAGE_MODELS[image_model]
        g.theta = self.theta
        self._h = C.c_void_p()
        _check(lib().epi_setup(C.byref(g), _ptr(Ip), _ptr(Im), _stream_handle(stream),
                               C.byref(self._h)))

    @property
    def n(self) -> int:
        m3, m2, M = self.shape_cells
        return (M + 1) * m2 * m3

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().epi_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _faces(self, t):
        if tuple(t.shape) != self.shape_faces:
            raise ValueError(f"expected face array of shape {self.shape_faces}, got {tuple(t.shape)}")
        return _ptr(t)

    def objective(self, b, with_penalty: bool = True, grad=None) -> dict:
        t = Terms()
        gp = self._faces(grad) if grad is not None else None
        _check(lib().epi_objective(self._h, self._faces(b), 1 if with_penalty else 0,
                                   C.byref(t), gp))
        return dict(J=t.J, D=t.D, S=t.S, P=t.P, feasible=bool(t.feasible))

    def smooth_solve(self, w, rho: float, out=None):
        import torch
        z = torch.empty_like(w) if out is None else out
        _check(lib().epi_smooth_solve(self._h, self._faces(w), float(rho), self._faces(z)))
        return z

    def precond_apply(self, b, r, precond="block", out=None):
        """z = P^-1 r with the GN-PCG preconditioner built from H_JGN(b) (block, jacobi,
        none or sgs); out must not overlap r or b."""
        import torch
        z = torch.empty_like(r) if out is None else out
        pc = PRECOND[precond] if isinstance(precond, str) else int(precond)
        _check(lib().epi_precond_apply(self._h, self._faces(b), pc, self._faces(r), self._faces(z)))
        return z

    def solve_gnpcg(self, b, **kw) -> dict:
        o = GNOpts()
        lib().epi_gn_default_opts(C.byref(o))
        for k, v in kw.items():
            if k == "precond":
                v = PRECOND[v] if isinstance(v, str) else int(v)
            setattr(o, k, v)
        n1 = max(o.max_iter, 0) + 1
        arrs = {k: (C.c_double * n1)() for k in ("J", "grad_norm", "pcg_relres", "step")}
        its = (C.c_int32 * n1)()
        rep = GNReport()
        for k, a in arrs.items():
            setattr(rep, k, C.cast(a, C.POINTER(C.c_double)))
        rep.pcg_iters = C.cast(its, C.POINTER(C.c_int32))
        _check(lib().epi_solve_gnpcg(self._h, self._faces(b), C.byref(o), C.byref(rep)))
        k = rep.iters
        return dict(iters=k, converged=bool(rep.converged), ls_failed=bool(rep.ls_failed),
                    J=list(arrs["J"][:k + 1]), grad_norm=list(arrs["grad_norm"][:k + 1]),
                    pcg_relres=list(arrs["pcg_relres"][:k]), step=list(arrs["step"][:k]),
                    pcg_iters=list(its[:k]))

    def corrected_images(self, b, out_plus=None, out_minus=None) -> dict:
        """Corrected images at the field b into out_plus / out_minus (canonical cell
        tensors, both or neither) and the quality measures {D, ncc, mean_plus, mean_minus}."""
        q = Quality()
        for t in (out_plus, out_minus):
            if t is not None and tuple(t.shape) != self.shape_cells:
                raise ValueError(f"expected cell tensors of shape {self.shape_cells}")
        op = _ptr(out_plus) if out_plus is not None else None
        om = _ptr(out_minus) if out_minus is not None else None
        _check(lib().epi_corrected_images(self._h, self._faces(b), op, om, C.byref(q)))
        return dict(D=q.D, ncc=q.ncc, mean_plus=q.mean_plus, mean_minus=q.mean_minus)

    def solve_admm(self, b, z, u, profile: bool = False, isolated_reps: int = 0, **kw) -> dict:
        """ADMM from the state (b, z, u), updated in place. With profile=True the solve runs
        through epi_profile_admm and the result carries per-kernel device times; with
        isolated_reps > 0 also the back-to-back launch time of each kernel family
        (microseconds per launch, kernel_us_isolated)."""
        o = ADMMOpts()
        lib().epi_admm_default_opts(C.byref(o))
        for k, v in kw.items():
            setattr(o, k, RHO_MODES[v] if k == "rho_mode" and isinstance(v, str) else v)
        n1 = max(o.max_iter, 1)
        keys = ["r_pri", "r_dual", "eps_pri", "eps_dual", "rho"]
        if o.with_lagrangian:
            keys.append("lagrangian")
        arrs = {k: (C.c_double * n1)() for k in keys}
        rep = ADMMReport()
        for k, a in arrs.items():
            setattr(rep, k, C.cast(a, C.POINTER(C.c_double)))
        if profile:
            prof = KernelProfile()
            prof.isolated_reps = int(isolated_reps)
            _check(lib().epi_profile_admm(self._h, self._faces(b), self._faces(z),
                                          self._faces(u), C.byref(o), C.byref(rep),
                                          C.byref(prof)))
        else:
            _check(lib().epi_solve_admm(self._h, self._faces(b), self._faces(z), self._faces(u),
                                        C.byref(o), C.byref(rep)))
        k = rep.iters
        out = dict(iters=k, converged=bool(rep.converged), max_active=rep.max_active,
                   hard_lines=int(rep.hard_lines))
        for key, a in arrs.items():
            out[key] = list(a[:k])
        if profile:
            out["kernel_ms"] = {n: prof.ms[i] for i, n in enumerate(KERNEL_NAMES)}
            out["kernel_launches"] = {n: int(prof.launches[i]) for i, n in enumerate(KERNEL_NAMES)}
            if isolated_reps > 0:
                out["kernel_us_isolated"] = {n: prof.us_isolated[i]
                                             for i, n in enumerate(KERNEL_NAMES)}
        return out


ML_MAX_LEVELS = 8


class MLReport(C.Structure):
    _fields_ = [("levels", C.c_int32), ("m", (C.c_int32 * 3) * ML_MAX_LEVELS),
                ("iters", C.c_int32 * ML_MAX_LEVELS), ("converged", C.c_int32 * ML_MAX_LEVELS),
                ("fallback", C.c_int32 * ML_MAX_LEVELS), ("rho_last", C.c_double * ML_MAX_LEVELS),
                ("J_last", C.c_double * ML_MAX_LEVELS)]


ML_RESTARTS = {"prolong_all": 1, "fine_b": 2, "average": 3}


def _ml_sigs(L):
    if getattr(L, "_ml_sigs", False):
        return L
    vp, i3 = C.c_void_p, C.c_int32 * 3
    L.epi_restrict_cells.argtypes = [i3, i3, vp, vp, vp]
    L.epi_restrict_cells.restype = C.c_int
    L.epi_prolong_faces.argtypes = [i3, i3, vp, vp, vp]
    L.epi_prolong_faces.restype = C.c_int
    L.epi_solve_multilevel_admm.argtypes = [C.POINTER(Grid), vp, vp, C.c_int32, C.c_int32,
                                            C.POINTER(ADMMOpts), vp, vp, C.POINTER(MLReport)]
    L.epi_solve_multilevel_admm.restype = C.c_int
    L.epi_solve_multilevel_gnpcg.argtypes = [C.POINTER(Grid), vp, vp, C.c_int32,
                                             C.POINTER(GNOpts), vp, vp, C.POINTER(MLReport)]
    L.epi_solve_multilevel_gnpcg.restype = C.c_int
    L._ml_sigs = True
    return L


def _counts(shape_cells):
    m3, m2, M = (int(x) for x in shape_cells)
    return (C.c_int32 * 3)(M, m2, m3)


def restrict_cells(fine, coarse, stream=None):
    """Coarse cell tensor = mean of the fine cells (canonical shapes (m3, m2, M), factors 1
    or 2 per axis); asynchronous on the stream."""
    L = _ml_sigs(lib())
    _check(L.epi_restrict_cells(_counts(fine.shape), _counts(coarse.shape), _ptr(fine),
                                _ptr(coarse), _stream_handle(stream)))


def prolong_faces(coarse, fine, stream=None):
    """Fine PE-face tensor from the coarse one (canonical shapes (m3, m2, M + 1))."""
    L = _ml_sigs(lib())
    mc = (coarse.shape[0], coarse.shape[1], coarse.shape[2] - 1)
    mf = (fine.shape[0], fine.shape[1], fine.shape[2] - 1)
    _check(L.epi_prolong_faces(_counts(mc), _counts(mf), _ptr(coarse), _ptr(fine),
                               _stream_handle(stream)))


def solve_multilevel_admm(Ip, Im, h, alpha, b, levels=3, beta=10.0, gamma=1e-3,
                          precision="mixed", ndim=None, stream=None, restart="average",
                          image_model="linear", theta=0.0, **opts) -> dict:
    """Coarse-to-fine ADMM (epi_solve_multilevel_admm); writes the finest field into b.
    restart: "prolong_all", "fine_b" or "average" (the three strategies of Section 4.4)."""
    L = _ml_sigs(lib())
    g = _grid_struct(tuple(Ip.shape), h, alpha, beta, gamma, precision, ndim, image_model, theta)
    o = ADMMOpts()
    L.epi_admm_default_opts(C.byref(o))
    for k, v in opts.items():
        setattr(o, k, RHO_MODES[v] if k == "rho_mode" and isinstance(v, str) else v)
    if tuple(b.shape) != (Ip.shape[0], Ip.shape[1], Ip.shape[2] + 1):
        raise ValueError("b must have the PE-face shape of the images")
    rs = ML_RESTARTS[restart] if isinstance(restart, str) else int(restart)
    rep = MLReport()
    _check(L.epi_solve_multilevel_admm(C.byref(g), _ptr(Ip), _ptr(Im), int(levels), rs,
                                       C.byref(o), _stream_handle(stream), _ptr(b),
                                       C.byref(rep)))
    n = rep.levels
    return dict(levels=n, sizes=[tuple(rep.m[l]) for l in range(n)],
                iters=list(rep.iters[:n]), converged=[bool(x) for x in rep.converged[:n]],
                fallback=[bool(x) for x in rep.fallback[:n]], rho_last=list(rep.rho_last[:n]))


def solve_multilevel_gnpcg(Ip, Im, h, alpha, b, levels=3, beta=10.0, gamma=1e-3,
                           precision="mixed", ndim=None, stream=None, image_model="linear",
                           theta=0.0, **opts) -> dict:
    """Coarse-to-fine GN-PCG (epi_solve_multilevel_gnpcg); writes the finest field into b."""
    L = _ml_sigs(lib())
    g = _grid_struct(tuple(Ip.shape), h, alpha, beta, gamma, precision, ndim, image_model, theta)
    o = GNOpts()
    L.epi_gn_default_opts(C.byref(o))
    for k, v in opts.items():
        if k == "precond":
            v = PRECOND[v] if isinstance(v, str) else int(v)
        setattr(o, k, v)
    if tuple(b.shape) != (Ip.shape[0], Ip.shape[1], Ip.shape[2] + 1):
        raise ValueError("b must have the PE-face shape of the images")
    rep = MLReport()
    _check(L.epi_solve_multilevel_gnpcg(C.byref(g), _ptr(Ip), _ptr(Im), int(levels), C.byref(o),
                                        _stream_handle(stream), _ptr(b), C.byref(rep)))
    n = rep.levels
    return dict(levels=n, sizes=[tuple(rep.m[l]) for l in range(n)],
                iters=list(rep.iters[:n]), converged=[bool(x) for x in rep.converged[:n]],
                J_last=list(rep.J_last[:n]))


EPI_EBUSY = 7
STATUS_NAMES[EPI_EBUSY] = "EPI_EBUSY"


def _batch_sigs(L):
    vp = C.c_void_p
    if getattr(L, "_batch_sigs", False):
        return L
    L.epi_batch_create.argtypes = [C.c_int32, C.c_int64, C.c_int32, C.c_int32, vp, C.POINTER(vp)]
    L.epi_batch_create.restype = C.c_int
    L.epi_batch_footprint.argtypes = [C.POINTER(Grid), C.c_int32]
    L.epi_batch_footprint.restype = C.c_int64
    L.epi_batch_admit.argtypes = [vp, C.POINTER(Grid), vp, vp, vp, vp, vp, C.POINTER(ADMMOpts),
                                  C.POINTER(C.c_int32)]
    L.epi_batch_admit.restype = C.c_int
    L.epi_batch_step.argtypes = [vp, C.POINTER(C.c_int32)]
    L.epi_batch_step.restype = C.c_int
    L.epi_batch_poll.argtypes = [vp, C.c_int32, C.POINTER(C.c_int32), C.POINTER(ADMMReport)]
    L.epi_batch_poll.restype = C.c_int
    L.epi_batch_release.argtypes = [vp, C.c_int32]
    L.epi_batch_release.restype = C.c_int
    L.epi_batch_destroy.argtypes = [vp]
    L.epi_batch_destroy.restype = None
    L.epi_batch_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                  C.POINTER(C.c_int64)]
    L.epi_batch_stats.restype = C.c_int
    L._batch_sigs = True
    return L


def _grid_struct(shape_cells, h, alpha, beta, gamma, precision, ndim=None, image_model="linear",
                 theta=0.0):
    m3, m2, M = (int(s) for s in shape_cells)
    g = Grid()
    g.ndim = ndim if ndim is not None else (2 if m3 == 1 else 3)
    g.m[0], g.m[1], g.m[2] = M, m2, m3
    for a in range(3):
        g.h[a] = float(h[a])
    g.alpha, g.beta, g.gamma = float(alpha), float(beta), float(gamma)
    g.precision = PREC[precision]
    g.image_model = IMAGE_MODELS[image_model]
    g.theta = float(theta)
    return g


class Batch:
    """Continuous-batching ADMM engine (epi_batch_*): admit volumes of different sizes, step
    all running ones together, poll and release finished ones. Tensors handed to `admit`
    are kept referenced until the slot is released."""

    def __init__(self, max_slots: int = 16, hbm_budget_bytes: int = 64 << 30,
                 precision: str = "mixed", iters_per_step: int = 8, stream=None):
        L = _batch_sigs(lib())
        self._h = C.c_void_p()
        self.precision = precision
        _check(L.epi_batch_create(int(max_slots), int(hbm_budget_bytes), PREC[precision],
                                  int(iters_per_step), _stream_handle(stream), C.byref(self._h)))
        self._keep = {}
        self._maxit = {}

    @staticmethod
    def footprint(shape_cells, h, alpha=50.0, max_iter=2000) -> int:
        g = _grid_struct(shape_cells, h, alpha, 10.0, 1e-3, "mixed")
        return int(_batch_sigs(lib()).epi_batch_footprint(C.byref(g), int(max_iter)))

    def admit(self, Ip, Im, h, alpha, b, z, u, beta=10.0, gamma=1e-3, ndim=None,
              image_model="linear", theta=0.0, **opts):
        """Returns the slot index, or None when the engine is busy (EPI_EBUSY). The engine
        takes the linear image model only (EPI_ENOTSUP otherwise)."""
        L = _batch_sigs(lib())
        g = _grid_struct(tuple(Ip.shape), h, alpha, beta, gamma, self.precision, ndim,
                         image_model, theta)
        o = ADMMOpts()
        L.epi_admm_default_opts(C.byref(o))
        for k, v in opts.items():
            setattr(o, k, RHO_MODES[v] if k == "rho_mode" and isinstance(v, str) else v)
        slot = C.c_int32(-1)
        st = L.epi_batch_admit(self._h, C.byref(g), _ptr(Ip), _ptr(Im), _ptr(b), _ptr(z),
                               _ptr(u), C.byref(o), C.byref(slot))
        if st == EPI_EBUSY:
            return None
        _check(st)
        self._keep[slot.value] = (Ip, Im, b, z, u)
        self._maxit[slot.value] = max(o.max_iter, 1)
        return slot.value

    def step(self) -> int:
        n = C.c_int32(0)
        _check(_batch_sigs(lib()).epi_batch_step(self._h, C.byref(n)))
        return n.value

    def poll(self, slot: int):
        """None while running, else the report dict (as Problem.solve_admm returns)."""
        L = _batch_sigs(lib())
        fin = C.c_int32(0)
        _check(L.epi_batch_poll(self._h, int(slot), C.byref(fin), None))
        if not fin.value:
            return None
        n1 = self._maxit[slot]
        arrs = {k: (C.c_double * n1)() for k in ("r_pri", "r_dual", "eps_pri", "eps_dual", "rho")}
        rep = ADMMReport()
        for k, a in arrs.items():
            setattr(rep, k, C.cast(a, C.POINTER(C.c_double)))
        _check(L.epi_batch_poll(self._h, int(slot), C.byref(fin), C.byref(rep)))
        if not fin.value:
            return None
        k = rep.iters
        out = dict(iters=k, converged=bool(rep.converged), max_active=rep.max_active,
                   hard_lines=int(rep.hard_lines))
        for key, a in arrs.items():
            out[key] = list(a[:k])
        return out

    def stats(self) -> dict:
        """Admissions, admissions that allocated a workspace, graph captures so far."""
        a, b, c = C.c_int64(), C.c_int64(), C.c_int64()
        _check(_batch_sigs(lib()).epi_batch_stats(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return dict(admissions=a.value, admissions_allocating=b.value, graph_captures=c.value)

    def release(self, slot: int):
        _check(_batch_sigs(lib()).epi_batch_release(self._h, int(slot)))
        self._keep.pop(slot, None)
        self._maxit.pop(slot, None)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _batch_sigs(lib()).epi_batch_destroy(self._h)
            self._h = C.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _server_sigs(L):
    vp = C.c_void_p
    if getattr(L, "_server_sigs", False):
        return L
    L.epi_server_clock.argtypes = []
    L.epi_server_clock.restype = C.c_double
    L.epi_server_create.argtypes = [C.c_int32, C.c_int64, C.c_int32, C.c_int32, vp, C.POINTER(vp)]
    L.epi_server_create.restype = C.c_int
    L.epi_server_submit.argtypes = [vp, C.c_int64, C.c_double, C.POINTER(Grid), vp, vp, vp, vp,
                                    vp, C.POINTER(ADMMOpts)]
    L.epi_server_submit.restype = C.c_int
    L.epi_server_progress.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32)]
    L.epi_server_progress.restype = C.c_int
    L.epi_server_take.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                  C.POINTER(ADMMReport)]
    L.epi_server_take.restype = C.c_int
    L.epi_server_destroy.argtypes = [vp]
    L.epi_server_destroy.restype = None
    L._server_sigs = True
    return L


class Server:
    """The request loop of the served solver (epi_server_*): submit requests as they
    arrive, call progress() repeatedly, take() finished ones. Tensors handed to submit are
    kept referenced until the request is taken."""

    def __init__(self, max_slots: int = 16, hbm_budget_bytes: int = 64 << 30,
                 precision: str = "mixed", iters_per_step: int = 8, stream=None):
        L = _server_sigs(lib())
        self._h = C.c_void_p()
        self.precision = precision
        _check(L.epi_server_create(int(max_slots), int(hbm_budget_bytes), PREC[precision],
                                   int(iters_per_step), _stream_handle(stream),
                                   C.byref(self._h)))
        self._keep = {}

    @staticmethod
    def clock() -> float:
        """Seconds on the server's monotonic clock (arrival times use it)."""
        return float(_server_sigs(lib()).epi_server_clock())

    def submit(self, request_id: int, Ip, Im, h, alpha, b, z, u, arrival=None, beta=10.0,
               gamma=1e-3, ndim=None, **opts):
        L = _server_sigs(lib())
        g = _grid_struct(tuple(Ip.shape), h, alpha, beta, gamma, self.precision, ndim)
        o = ADMMOpts()
        L.epi_admm_default_opts(C.byref(o))
        for k, v in opts.items():
            setattr(o, k, RHO_MODES[v] if k == "rho_mode" and isinstance(v, str) else v)
        t = self.clock() if arrival is None else float(arrival)
        _check(L.epi_server_submit(self._h, int(request_id), t, C.byref(g), _ptr(Ip), _ptr(Im),
                                   _ptr(b), _ptr(z), _ptr(u), C.byref(o)))
        self._keep[int(request_id)] = ((Ip, Im, b, z, u), max(o.max_iter, 1))

    def progress(self):
        """(queued, running, ready) after one round of admission, engine step and polling."""
        q, r, d = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        _check(_server_sigs(lib()).epi_server_progress(self._h, C.byref(q), C.byref(r),
                                                       C.byref(d)))
        return q.value, r.value, d.value

    def take(self):
        """The oldest finished request as a dict (id, latency_s, report fields), or None."""
        L = _server_sigs(lib())
        if not self._keep:
            return None
        cap = max(m for _, m in self._keep.values())
        arrs = {k: (C.c_double * cap)() for k in ("r_pri", "r_dual", "eps_pri", "eps_dual", "rho")}
        rep = ADMMReport()
        for k, a in arrs.items():
            setattr(rep, k, C.cast(a, C.POINTER(C.c_double)))
        rid, lat = C.c_int64(0), C.c_double(0.0)
        st = L.epi_server_take(self._h, C.byref(rid), C.byref(lat), C.byref(rep))
        if st == EPI_EBUSY:
            return None
        _check(st)
        self._keep.pop(rid.value, None)
        k = rep.iters
        out = dict(id=rid.value, latency_s=lat.value, iters=k, converged=bool(rep.converged),
                   status=rep.status, max_active=rep.max_active, hard_lines=int(rep.hard_lines))
        for key, a in arrs.items():
            out[key] = list(a[:k])
        return out

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _server_sigs(lib()).epi_server_destroy(self._h)
            self._h = C.c_void_p()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
