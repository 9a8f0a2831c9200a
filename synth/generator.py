"""Synthetic volume pairs from a known field, following the continuous distortion model.

The undistorted image I and the field b are smooth analytic functions on the unit box.
The two measured images are produced by the reversed-gradient identity of Section 2:

    I(x) = I_plus(x + b(x) v) (1 + d_v b(x)) = I_minus(x - b(x) v) (1 - d_v b(x)),

evaluated exactly at the cell centres y of each phase-encoding (PE) line by inverting
y = x +/- b(x) per sample (safeguarded Newton), so that the discrete distance at the true
field vanishes up to interpolation and quadrature error (plus the added noise).

Recipe (seeded with ``numpy.random.default_rng(seed)``; draws in this order: image
parameters, field parameters, noise for I_plus, noise for I_minus):

* image: Q Gaussian blobs (Q = 12 in 2D, 64 in 3D), centres U[0.2, 0.8]^d, widths
  U[0.03, 0.15], amplitudes U[0.2, 1]; in 3D plus an ellipsoidal shell
  0.8 exp(-(r_e - 1)^2 / (2 * 0.03^2)), r_e = |(x - 0.5) / R|, R = (0.40, 0.36, 0.42) in
  the caller's axis order; the sum is multiplied by a C1 raised-cosine window along the
  PE axis (0 on [0, 0.08] and [0.92, 1], 1 on [0.18, 0.82]) so that the support stays
  inside the domain after the distortion;
* field: B Gaussian bumps (B = 4 in 2D, 8 in 3D), centres U[0.2, 0.8]^d, widths
  U[0.08, 0.2], signs +/-1, scaled so that max |b| over the faces is ``peak`` PE voxels
  (3 in 2D, 4 in 3D) and then reduced, if needed, until max |D1 b| <= ``dmax``
  (0.8 in 2D, 0.85 in 3D);
* noise: N(0, sigma^2) with sigma = 0.01 added to each measured image.

Arrays come back in the canonical layout used everywhere else in this repository: a 3D
C-order array of shape (m3, m2, M) for cells and (m3, m2, M + 1) for PE faces, where axis
-1 is the PE axis and (m2, m3) are the other axes in the caller's order (m3 = 1 in 2D).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

SHELL_R = (0.40, 0.36, 0.42)
SHELL_W = 0.03
WIN_LO, WIN_HI = 0.08, 0.18  # raised-cosine ramp of the PE window


@dataclass
class Volume:
    """One synthetic pair in canonical layout (PE axis last in numpy order)."""

    Ip: np.ndarray          # (m3, m2, M) image measured with PE direction +v
    Im: np.ndarray          # (m3, m2, M) image measured with PE direction -v
    b_true: np.ndarray      # (m3, m2, M+1) field on the PE faces
    I_true: np.ndarray      # (m3, m2, M) undistorted image at cell centres
    m: Tuple[int, int, int]         # canonical cell counts (M, m2, m3)
    h: Tuple[float, float, float]   # canonical voxel edges (h_p, h2, h3); h3 = 1 in 2D
    ndim: int
    pe_axis: int                    # 0-based PE axis in the caller's order
    m_user: Tuple[int, ...]
    seed: int
    params: dict = field(default_factory=dict)


def _perm(ndim: int, pe_axis: int) -> List[int]:
    return [pe_axis] + [a for a in range(ndim) if a != pe_axis]


def to_canonical(arr: np.ndarray, pe_axis: int) -> np.ndarray:
    """Caller-order array (cells or PE faces) -> canonical (m3, m2, M[+1]) C-order copy."""
    nd = arr.ndim
    p = _perm(nd, pe_axis)
    if nd == 2:
        out = np.transpose(arr, (p[1], p[0]))[None]
    elif nd == 3:
        out = np.transpose(arr, (p[2], p[1], p[0]))
    else:
        raise ValueError("ndim must be 2 or 3")
    return np.ascontiguousarray(out)


def from_canonical(arr: np.ndarray, ndim: int, pe_axis: int) -> np.ndarray:
    """Inverse of :func:`to_canonical`."""
    p = _perm(ndim, pe_axis)
    if ndim == 2:
        a2 = arr[0]                       # (m2, M) with axes (p1, p0)
        inv = np.argsort([p[1], p[0]])
        return np.ascontiguousarray(np.transpose(a2, inv))
    inv = np.argsort([p[2], p[1], p[0]])
    return np.ascontiguousarray(np.transpose(arr, inv))


def _window(t: np.ndarray) -> np.ndarray:
    w = np.zeros_like(t)
    mid = (t >= WIN_HI) & (t <= 1.0 - WIN_HI)
    w[mid] = 1.0
    lo = (t > WIN_LO) & (t < WIN_HI)
    w[lo] = 0.5 * (1.0 - np.cos(np.pi * (t[lo] - WIN_LO) / (WIN_HI - WIN_LO)))
    hi = (t > 1.0 - WIN_HI) & (t < 1.0 - WIN_LO)
    w[hi] = 0.5 * (1.0 - np.cos(np.pi * ((1.0 - WIN_LO) - t[hi]) / (WIN_HI - WIN_LO)))
    return w


class _Field:
    """b(x) = s * sum_q eps_q exp(-|x - nu_q|^2 / (2 tau_q^2)) in canonical coordinates."""

    def __init__(self, nu_c, tau, eps, x2, x3):
        self.nu = nu_c            # (B, 3) canonical centres (PE first)
        self.tau = tau
        self.eps = eps
        # per-line transverse factor F[q, line] with line = j + m2 * k
        f2 = np.exp(-((x2[None, :] - nu_c[:, 1:2]) ** 2) / (2 * tau[:, None] ** 2))   # (B, m2)
        f3 = np.exp(-((x3[None, :] - nu_c[:, 2:3]) ** 2) / (2 * tau[:, None] ** 2))   # (B, m3)
        self.F = (f3[:, :, None] * f2[:, None, :]).reshape(len(tau), -1)            # (B, L)
        self.s = 1.0

    def eval(self, xp: np.ndarray, deriv: bool = False):
        """xp: (L, K) PE coordinates for every line; returns b (and d b / d x_p)."""
        val = np.zeros_like(xp)
        der = np.zeros_like(xp) if deriv else None
        for q in range(len(self.tau)):
            idx = np.nonzero(np.abs(self.F[q]) > 1e-17)[0]
            if idx.size == 0:
                continue
            d = xp[idx] - self.nu[q, 0]
            e = np.exp(-d * d / (2 * self.tau[q] ** 2)) * (self.eps[q] * self.F[q, idx])[:, None]
            val[idx] += e
            if deriv:
                der[idx] -= e * d / self.tau[q] ** 2
        val *= self.s
        if deriv:
            der *= self.s
            return val, der
        return val


def _image_lines(xp, x2l, x3l, mu_c, sig, amp, shell_R_c, three_d):
    """Undistorted image at PE coordinates xp (L, K); x2l, x3l are the transverse cell
    centres of each of the L lines."""
    out = np.zeros_like(xp)
    for q in range(len(sig)):
        G = amp[q] * np.exp(-((x2l - mu_c[q, 1]) ** 2 + (x3l - mu_c[q, 2]) ** 2)
                            / (2 * sig[q] ** 2))
        idx = np.nonzero(G > 1e-14)[0]
        if idx.size == 0:
            continue
        d = xp[idx] - mu_c[q, 0]
        out[idx] += np.exp(-d * d / (2 * sig[q] ** 2)) * G[idx, None]
    if three_d:
        T = ((x2l - 0.5) / shell_R_c[1]) ** 2 + ((x3l - 0.5) / shell_R_c[2]) ** 2
        re = np.sqrt(((xp - 0.5) / shell_R_c[0]) ** 2 + T[:, None])
        out += 0.8 * np.exp(-((re - 1.0) ** 2) / (2 * SHELL_W ** 2))
    return out * _window(xp)


def _threads() -> int:
    import os
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _invert(fld: _Field, y: np.ndarray, sign: float, bmax: float) -> np.ndarray:
    """Solve x + sign * b(x) = y per sample (monotone since 1 +/- d b > 0): Newton steps
    kept inside a shrinking bracket, iterating only on samples not yet converged."""
    x = y.copy()
    lo = y - bmax - 1e-12
    hi = y + bmax + 1e-12
    act = np.ones(y.shape, dtype=bool)
    for _ in range(100):
        li = np.nonzero(act.any(axis=1))[0]
        if li.size == 0:
            break
        sub = _Field.__new__(_Field)
        sub.nu, sub.tau, sub.eps, sub.s = fld.nu, fld.tau, fld.eps, fld.s
        sub.F = fld.F[:, li]
        xs, ys, ls, hs = x[li], y[li], lo[li], hi[li]
        bv, db = sub.eval(xs, deriv=True)
        F = xs + sign * bv - ys
        pos = F > 0
        hs = np.where(pos, np.minimum(hs, xs), hs)
        ls = np.where(~pos, np.maximum(ls, xs), ls)
        xn = xs - F / (1.0 + sign * db)
        bad = (xn <= ls) | (xn >= hs) | ~np.isfinite(xn)
        xn = np.where(bad, 0.5 * (ls + hs), xn)
        done = np.abs(F) <= 1e-15
        x[li] = np.where(done, xs, xn)
        lo[li], hi[li] = ls, hs
        act[li] = ~done
    return x


def _lines_chunk(args):
    """Undistorted and measured images of a contiguous range of PE lines (elementwise per
    line, so the result does not depend on how the lines are split)."""
    (nu, tau, eps, s, F, xx2, xx3, xcc, mu_c, sig, amp, shell_c, three_d, bmax) = args
    sub = _Field.__new__(_Field)
    sub.nu, sub.tau, sub.eps, sub.s, sub.F = nu, tau, eps, s, F
    it = _image_lines(xcc, xx2, xx3, mu_c, sig, amp, shell_c, three_d)
    res = [it]
    for sign in (+1.0, -1.0):
        xs = _invert(sub, xcc, sign, bmax)
        _, db = sub.eval(xs, deriv=True)
        res.append(_image_lines(xs, xx2, xx3, mu_c, sig, amp, shell_c, three_d)
                   / (1.0 + sign * db))
    return res


_POOL = None
_POOL_MIN_CELLS = 400_000     # smaller volumes are generated in-process


def _pool_usable() -> bool:
    """Spawned workers re-import the main module: only possible when it is a real file
    (or absent, as under ``python -c``). EPI_SYNTH_SERIAL=1 keeps generation in-process
    (for runs under a profiler, which would follow every worker)."""
    import os
    import sys
    if os.environ.get("EPI_SYNTH_SERIAL", "0") not in ("", "0"):
        return False
    f = getattr(sys.modules.get("__main__"), "__file__", None)
    return _threads() > 1 and (f is None or os.path.exists(f))


def _pool():
    """Worker processes (spawned: they import numpy and this module only) for large
    volumes; numpy's many small temporaries keep threads from scaling."""
    global _POOL
    if _POOL is None:
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor
        import atexit
        _POOL = ProcessPoolExecutor(max_workers=_threads(), mp_context=mp.get_context("spawn"))
        atexit.register(_POOL.shutdown, wait=True)
    return _POOL


def shutdown_pool() -> None:
    """Stop the worker processes now (they are otherwise stopped at interpreter exit);
    a later large volume starts a new pool."""
    global _POOL
    if _POOL is not None:
        _POOL.shutdown(wait=True)
        _POOL = None


def _run_chunks(jobs, parallel: bool):
    global _POOL
    if parallel:
        from concurrent.futures.process import BrokenProcessPool
        try:
            return list(_pool().map(_lines_chunk, jobs))
        except BrokenProcessPool:
            _POOL.shutdown(wait=False, cancel_futures=True)
            _POOL = None
    return [_lines_chunk(j) for j in jobs]


def generate(seed: int, m_user: Sequence[int], pe_axis: int, *, noise: float = 0.01,
             n_blobs: int | None = None, n_bumps: int | None = None,
             peak_vox: float | None = None, dmax: float | None = None) -> Volume:
    """Generate one pair. ``m_user`` are cell counts in the caller's axis order, ``pe_axis``
    is 0-based. Domain [0, 1]^d, h_a = 1 / m_a."""
    m_user = tuple(int(v) for v in m_user)
    d = len(m_user)
    if d not in (2, 3):
        raise ValueError("2D or 3D only")
    three_d = d == 3
    Q = n_blobs if n_blobs is not None else (64 if three_d else 12)
    B = n_bumps if n_bumps is not None else (8 if three_d else 4)
    peak = peak_vox if peak_vox is not None else (4.0 if three_d else 3.0)
    gmax = dmax if dmax is not None else (0.85 if three_d else 0.8)

    rng = np.random.default_rng(seed)
    # image parameters
    mu = rng.uniform(0.2, 0.8, size=(Q, d))
    sig = rng.uniform(0.03, 0.15, size=Q)
    amp = rng.uniform(0.2, 1.0, size=Q)
    # field parameters
    nu = rng.uniform(0.2, 0.8, size=(B, d))
    tau = rng.uniform(0.08, 0.2, size=B)
    eps = rng.choice(np.array([-1.0, 1.0]), size=B)

    p = _perm(d, pe_axis)
    M = m_user[p[0]]
    m2 = m_user[p[1]]
    m3 = m_user[p[2]] if three_d else 1
    hp, h2 = 1.0 / M, 1.0 / m2
    h3 = 1.0 / m3 if three_d else 1.0

    def canon_pts(P):
        c = np.zeros((P.shape[0], 3))
        c[:, 0] = P[:, p[0]]
        c[:, 1] = P[:, p[1]]
        c[:, 2] = P[:, p[2]] if three_d else 0.5
        return c

    mu_c, nu_c = canon_pts(mu), canon_pts(nu)
    R_user = SHELL_R[:d]
    shell_c = np.array([R_user[p[0]], R_user[p[1]], R_user[p[2]] if three_d else 1.0])

    x2 = (np.arange(m2) + 0.5) * h2
    x3 = (np.arange(m3) + 0.5) * h3 if three_d else np.array([0.5])
    L = m2 * m3
    xc = np.broadcast_to((np.arange(M) + 0.5) * hp, (L, M)).copy()        # cell centres
    xf = np.broadcast_to(np.arange(M + 1) * hp, (L, M + 1)).copy()         # PE faces

    fld = _Field(nu_c, tau, eps, x2, x3)
    bf = fld.eval(xf)
    s = peak * hp / max(np.max(np.abs(bf)), 1e-300)
    g = np.diff(bf * s, axis=1) / hp
    gm = np.max(np.abs(g))
    if gm > gmax:
        s *= gmax / gm
    fld.s = s
    b_faces = fld.eval(xf)
    bmax = float(s * np.sum(np.max(np.abs(fld.F), axis=1)))   # bound on |b| anywhere

    # Everything below is elementwise per PE line, so lines are processed in chunks (on
    # worker processes for large volumes); the result does not depend on the chunking.
    x3_of_line = np.repeat(np.arange(m3), m2)
    x2_of_line = np.tile(np.arange(m2), m3)
    par = L * M >= _POOL_MIN_CELLS and _pool_usable()
    bounds = np.linspace(0, L, min(L, 4 * _threads() if par else 1) + 1).astype(int)
    chunks = [(int(a), int(b)) for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    jobs = [(fld.nu, fld.tau, fld.eps, fld.s, fld.F[:, a:b_], x2[x2_of_line[a:b_]],
             x3[x3_of_line[a:b_]], xc[a:b_], mu_c, sig, amp, shell_c, three_d, bmax)
            for a, b_ in chunks]
    parts = _run_chunks(jobs, par)
    I_true = np.concatenate([p_[0] for p_ in parts], axis=0)
    Ip = np.concatenate([p_[1] for p_ in parts], axis=0)
    Im = np.concatenate([p_[2] for p_ in parts], axis=0)
    if noise > 0:
        Ip = Ip + rng.normal(0.0, noise, size=Ip.shape)
        Im = Im + rng.normal(0.0, noise, size=Im.shape)

    shp_c = (m3, m2, M)
    return Volume(
        Ip=Ip.reshape(shp_c), Im=Im.reshape(shp_c),
        b_true=b_faces.reshape(m3, m2, M + 1), I_true=I_true.reshape(shp_c),
        m=(M, m2, m3), h=(hp, h2, h3), ndim=d, pe_axis=pe_axis, m_user=m_user, seed=seed,
        params=dict(Q=Q, B=B, peak=peak, dmax=gmax, scale=s, noise=noise),
    )


# --------------------------------------------------------------------------------------
# The five workload configurations (sizes, PE axis, solver parameters)
# --------------------------------------------------------------------------------------
CONFIGS = {
    "2d_64x64": dict(m_user=(64, 64), pe_axis=1, alpha=50.0, beta=10.0, rho=1e3, iters=20),
    "3d_128x128x64": dict(m_user=(128, 128, 64), pe_axis=1, alpha=50.0, beta=10.0,
                             rho=1e3, iters=30),
    "3d_240x200x110": dict(m_user=(240, 200, 110), pe_axis=0, alpha=50.0, beta=10.0,
                              rho=1e3, iters=30),
}


def config_volume(name: str, seed: int = 0, **kw) -> Volume:
    c = CONFIGS[name]
    return generate(seed, c["m_user"], c["pe_axis"], **kw)


def batch_shapes(n: int = 48, lo=(96, 96, 48), hi=(160, 160, 96)):
    """Uneven batch: per seed s, sizes uniform per axis in [lo, hi] and a PE axis in {0,1,2},
    both drawn from ``default_rng(s)`` before the volume's own parameters (which then use
    seed s as well)."""
    out = []
    for s in range(n):
        r = np.random.default_rng(10_000 + s)
        m = tuple(int(r.integers(lo[a], hi[a] + 1)) for a in range(3))
        pe = int(r.integers(0, 3))
        out.append((s, m, pe))
    return out


def serving_requests(rate: float = 20.0, duration: float = 120.0, seed: int = 12345,
                     frac_2d: float = 0.3):
    """Poisson arrivals: list of (t_arrival, request_seed, m_user, pe_axis)."""
    r = np.random.default_rng(seed)
    t, q, out = 0.0, 0, []
    while True:
        t += r.exponential(1.0 / rate)
        if t > duration:
            break
        if r.random() < frac_2d:
            side = (int(r.integers(128, 257)), int(r.integers(128, 257)))
            out.append((t, q, side, 1))
        else:
            m = (int(r.integers(64, 241)), int(r.integers(64, 201)), int(r.integers(64, 111)))
            out.append((t, q, m, 0))
        q += 1
    return out
