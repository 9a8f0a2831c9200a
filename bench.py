#!/usr/bin/env python3
"""Throughput of the ADMM solver on synthetic volumes shaped like the paper's
high-resolution 3D data: 240 x 200 x 110 cells, PE along the first axis (5,302,000 PE-face
unknowns), alpha = 50, rho = 1e3, solved from b = z = u = 0 to the relative residual 1e-3
(eq. admmStop with eps_abs = 0, eps_rel = 1e-3), on one MI355X.

One step = one volume solved to that tolerance. The mixed-precision solver (split-bf16
MFMA DCT) gives `value`; the plain float32 solver is timed beside it. Inputs are resident in
HBM and the problem handles exist before the timed region (slot preallocation); each step
clears the state and runs the whole solve.

Two more legs time the continuous-batching engine (epi_batch_*) against the plain float32
single-volume solver:
  * batched: 48 volumes, each axis uniform in [96,160] x [96,160] x [48,96], PE axis drawn
    per volume, 40 ADMM iterations each, admitted together (setup inside the timed region);
  * served: a Poisson request stream (20 req/s; 30% 2D slices 128..256 per side, 70% 3D
    volumes 64..240 x 64..200 x 64..110), each request solved from zero to the relative
    residual 1e-3; latency = completion - arrival. Requests draw their images from a pool
    of volumes generated from the stream's first requests (generation is far slower than
    the arrival rate), uploaded to HBM before the stream starts.
Prints one JSON line on stdout.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

M_USER = (240, 200, 110)
PE_AXIS = 0
ALPHA, BETA, RHO = 50.0, 10.0, 1e3
TOL = 1e-3
# ADMM iterations per graph replay between host checks of the stopping flag (results do not
# depend on it; 32 measured 0.7 % faster than 16 and than 64 on the four 240x200x110 solves)
CHECK_EVERY = 32
MAX_ITER = 2000


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def mfma_flops(M, m2, m3, precision, fixed_rho=True):
    """Matrix-core flops each DCT pass executes over the unpadded transform lengths. The
    split-bf16 path runs the even/odd halves of each transform (2c^2 + 2f^2 per column of
    length m, c = ceil(m/2), f = floor(m/2)) with three products per multiply-add; the
    float32 path runs full products (2m^2 per column). The j-axis pass applies forward and
    inverse (two products), except in split-bf16 with a fixed rho, where it is one product
    with the per-slice operator of the same half-block shape."""
    n = (M + 1) * m2 * m3

    def per_face(m):
        if precision == "mixed":
            c, f = (m + 1) // 2, m // 2
            return 3 * (2 * c * c + 2 * f * f) / m
        return 2 * m

    j = 1 if (precision == "mixed" and fixed_rho) else 2
    return {"dct_axis3": per_face(m3) * n, "dct_axis2_fused": j * per_face(m2) * n,
            "dct_last_epilogue": per_face(m3) * n}


def zop_bytes(m2, m3):
    """Bytes of the split-bf16 per-slice operators of the j-axis pass (fixed rho): hi and lo
    bfloat16 fragments of both even/odd halves, padded to 16-row tiles and 32-wide steps."""
    ce = (m2 + 1) // 2
    rt, ks = 2 * ((ce + 15) // 16), (ce + 31) // 32
    return m3 * 2 * rt * ks * 64 * 8 * 2


def method_bytes(M, m2, m3):
    """HBM bytes the method itself must move (float32, each line or tile staged on chip
    once): the b-step reads I+, I- (8 bytes per cell) and b, z, u and writes b (16 bytes
    per face); the z- and u-step read b, u and the old z and write z, u (20 bytes per
    face). One ADMM iteration: 8 N + 36 n bytes (44 bytes per face)."""
    n = (M + 1) * m2 * m3
    N = M * m2 * m3
    return {"bstep": 8 * N + 16 * n, "zu_step": 20 * n, "iteration": 8 * N + 36 * n}


def algorithmic_bytes(M, m2, m3, zop=True):
    """HBM bytes each kernel family of this implementation moves per launch (float32
    arrays): the method's bytes plus the intermediates of the three-pass z-step and the
    fused w = b + u. zop: the j-axis pass also reads its per-slice operators (split-bf16
    solver with a fixed rho)."""
    n = (M + 1) * m2 * m3
    N = M * m2 * m3
    last = 24 * n                                  # read T, b, u, z_old; write z, u
    return {
        "bstep": 4 * (2 * N + 5 * n),              # read I+, I-, b, z, u; write b, w
        "dct_axis3": 8 * n,                        # read w, write T1
        # read T1, write T2 (3D) / epilogue (2D); + the operators
        "dct_axis2_fused": 8 * n + (zop_bytes(m2, m3) if zop else 0),
        "dct_last_epilogue": last,
        "bstep_hard": 0, "finalize": 0,
    }


def _profile_blob(fname):
    """The machine-readable block of a committed profile summary, or None when it is missing
    or the kernel sources changed since its counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", fname)
    try:
        txt = open(path).read()
        blob = json.loads(re.search(r"```json\n(.*?)\n```", txt, re.S).group(1))
    except (OSError, AttributeError, ValueError):
        return None
    csrc = os.path.join(ROOT, "paper_1607_00531_amd", "csrc")
    for src, h in blob["sources_sha256_16"].items():
        try:
            cur = hashlib.sha256(open(os.path.join(csrc, src), "rb").read()).hexdigest()[:16]
        except OSError:
            return None
        if cur != h:
            return None
    return blob


def counter_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE / WRITE_SIZE summary,
    or None when the kernel sources changed since those counters were taken."""
    blob = _profile_blob("admm_gnpcg_240x200x110_hbm_counters.md")
    rec = blob["per_launch"].get(kernel) if blob else None
    return rec["traffic_bytes"] if rec else None


def counter_valu(kernel, launch_us):
    """VALU issue rate of `kernel`: wave64 VALU instructions per launch (SQ_INSTS_VALU, from
    the committed SQ-counter summary) over the launch time measured here, against the VALU
    issue peak; None when the sources changed since the counters were taken."""
    blob = _profile_blob("admm_gnpcg_240x200x110_sq_counters.md")
    rec = blob["per_launch"].get(kernel) if blob else None
    if not rec or not launch_us:
        return None
    peak = blob["peak_valu_wave_instructions_per_s"] / 1e9
    ach = rec["valu_wave_instructions"] / (launch_us * 1e-6) / 1e9
    return {"wave_instructions_per_launch": rec["valu_wave_instructions"],
            "per_wave": rec["valu_per_wave"], "achieved": round(ach, 1), "peak": peak,
            "unit": "G wave64 VALU instructions/s", "frac": round(ach / peak, 4),
            "peak_rule": blob["peak_rule"], "source": "SQ_INSTS_VALU, profiles/"
            "admm_gnpcg_240x200x110_sq_counters.md"}


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    f, c = int(np.floor(k)), int(np.ceil(k))
    return xs[f] + (xs[c] - xs[f]) * (k - f)


def host_cpu():
    """CPU model and the number of CPUs this process may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    return model, ncpu


def _oracle_admm_iters(O, P, iters):
    """`iters` FP64 ADMM iterations from zero; seconds per iteration, the last two iterates
    and the residual histories."""
    b = np.zeros((P.L, P.M + 1))
    z, u = b.copy(), b.copy()
    hist = {"r_pri": [], "r_dual": []}
    prev = None
    t0 = time.perf_counter()
    for _ in range(iters):
        prev = (b, z, u)
        bn, _, _ = O.bstep(P, b, z, u, RHO)
        zn = O.zstep(P, bn + u, RHO)
        u = u + bn - zn
        rp, rd, _, _ = O.admm_residuals(P, bn, zn, z, u, RHO, 0.0, 0.0)
        hist["r_pri"].append(rp)
        hist["r_dual"].append(rd)
        b, z = bn, zn
    return (time.perf_counter() - t0) / iters, prev, (b, z, u), hist


def cpu_baseline(vol, gpu_iters_mean, iters, iters_1thread=3):
    """The FP64 oracle on this host: `iters` ADMM iterations of one 240 x 200 x 110 volume
    with every thread the BLAS library uses, scaled by the GPU's mean iteration count to
    one solve; the same with one thread (`iters_1thread` iterations); and per-iteration
    times of the 2D 64 x 64 and 3D 128 x 128 x 64 workloads. Also returns the oracle's
    last two iterates and histories of the 240 x 200 x 110 sample."""
    import oracle as O
    from synth import config_volume
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        blas = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    except Exception:
        threadpool_limits, blas = None, 1
    model, ncpu = host_cpu()
    P = O.make_problem(vol.Ip, vol.Im, vol.h, ALPHA, BETA)
    dt, prev, last, hist = _oracle_admm_iters(O, P, iters)
    dt1 = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            dt1 = _oracle_admm_iters(O, P, iters_1thread)[0]
    small = {}
    for name, k in (("2d_64x64", 20), ("3d_128x128x64", 4)):
        v = config_volume(name, 0)
        Pk = O.make_problem(v.Ip, v.Im, v.h, ALPHA, BETA)
        small[name] = {"s_per_iteration": round(_oracle_admm_iters(O, Pk, k)[0], 5),
                       "iterations_timed": k}
    base = {"value": 1.0 / (dt * gpu_iters_mean), "unit": "volumes/s", "cores": int(blas),
            "kind": "oracle",
            "sample": f"{iters} FP64 ADMM iterations of one 240x200x110 volume "
                      f"({dt:.2f} s/iteration, {dt * iters:.1f} s) x {gpu_iters_mean:.1f} "
                      f"iterations per solve (mean of the GPU solves), extrapolated; BLAS "
                      f"threads {blas}, numpy's elementwise work on one thread",
            "host_cpu": model, "host_cpus_available": ncpu,
            "one_thread": None if dt1 is None else {
                "value": 1.0 / (dt1 * gpu_iters_mean), "unit": "volumes/s",
                "s_per_iteration": round(dt1, 4), "iterations_timed": iters_1thread},
            "s_per_iteration": round(dt, 4), "other_workloads": small}
    ref = {"P": P, "prev": prev, "last": last, "hist": hist, "J": O.objective(P, last[0])["J"]}
    return base, ref


def oracle_error(prob, ref, iters, shape):
    """Error of the GPU (mixed precision, the timed configuration) against the oracle on
    the cpu_baseline sample: one iteration from the oracle's iterate iters - 1 (the
    per-step criterion, 1e-3 voxel), and the whole trajectory of `iters` iterations from
    zero (histories at 1e-4 relative; fields reported with the share of faces beyond
    1e-3 voxel, since the iterate after a knot crossing of the linear image model is
    discontinuous in the state)."""
    import torch
    P = ref["P"]
    dev = torch.device("cuda:0")
    T = lambda a: torch.tensor(np.ascontiguousarray(a).reshape(shape), dtype=torch.float32, device=dev)

    def field(g, c):
        e = np.abs(g.cpu().numpy().reshape(P.L, -1) - c) / P.hp
        return {"max_vox": float(e.max()), "faces_beyond_1e-3_vox": float(np.mean(e > 1e-3))}

    b, z, u = (torch.zeros(shape, device=dev) for _ in range(3))
    rep = prob.solve_admm(b, z, u, rho=RHO, max_iter=iters, eps_abs=0.0, eps_rel=0.0,
                          check_every=CHECK_EVERY)
    J = prob.objective(b, True)["J"]
    hrel = max(abs(a - c) / abs(c) for key in ("r_pri", "r_dual")
               for a, c in zip(rep[key], ref["hist"][key]))
    traj = {"iters": iters, "b": field(b, ref["last"][0]), "z": field(z, ref["last"][1]),
            "u": field(u, ref["last"][2]), "J_rel": abs(J - ref["J"]) / abs(ref["J"]),
            "hist_rel_max": hrel}
    b, z, u = (T(x) for x in ref["prev"])
    rep = prob.solve_admm(b, z, u, rho=RHO, max_iter=1, eps_abs=0.0, eps_rel=0.0, check_every=16)
    step = {"b_vox": field(b, ref["last"][0])["max_vox"], "z_vox": field(z, ref["last"][1])["max_vox"],
            "u_vox": field(u, ref["last"][2])["max_vox"],
            "r_pri_rel": abs(rep["r_pri"][0] - ref["hist"]["r_pri"][-1]) / ref["hist"]["r_pri"][-1],
            "r_dual_rel": abs(rep["r_dual"][0] - ref["hist"]["r_dual"][-1]) / ref["hist"]["r_dual"][-1]}
    return {"one_step_from_oracle_iterate": step, "trajectory": traj}


def converged_error(prob, shape, seed):
    """The timed solve of one volume against the stored oracle solve of the same volume to
    the relative residual 1e-3 (tests/oracle_samples/, written by the oracle alone): the
    iteration counts and b, z, u at the stored faces."""
    import torch
    path = os.path.join(ROOT, "tests", "oracle_samples", f"admm_240x200x110_seed{seed}.npz")
    if not os.path.exists(path):
        return None
    ref = np.load(path)
    dev = torch.device("cuda:0")
    b, z, u = (torch.zeros(shape, device=dev) for _ in range(3))
    rep = prob.solve_admm(b, z, u, rho=RHO, max_iter=MAX_ITER, eps_abs=0.0, eps_rel=TOL,
                          check_every=CHECK_EVERY)
    hp = 1.0 / M_USER[PE_AXIS]
    out = {"seed": seed, "gpu_iters": rep["iters"], "oracle_iters": int(ref["iters"]),
           "faces_compared": int(ref["idx"].size)}
    for name, t in zip("bzu", (b, z, u)):
        g = t.cpu().numpy().reshape(-1)[ref["idx"]].astype(np.float64)
        out[f"{name}_vox"] = float(np.abs(g - ref[name]).max() / hp)
    return out


def engine_same_volumes(imgs, vols, m3, m2, M, steps, max_iter, iters_per_step=16):
    """The batching engine (mixed precision) on the headline volumes: all of them admitted
    together, each solved from zero to the relative residual 1e-3; `steps` volumes in
    total after one warm-up round. Admission is inside the timed region."""
    import torch
    from paper_1607_00531_amd import Batch
    dev = imgs[0][0].device
    states = [[torch.zeros((m3, m2, M + 1), device=dev) for _ in range(3)] for _ in imgs]
    opts = dict(rho=RHO, max_iter=max_iter, eps_abs=0.0, eps_rel=TOL)

    def one_round(bt, k):
        for st in states[:k]:
            for t in st:
                t.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        slots = [bt.admit(Ip, Im, v.h, ALPHA, *st, beta=BETA, **opts)
                 for (Ip, Im), v, st in zip(imgs[:k], vols[:k], states[:k])]
        while bt.step() > 0:
            pass
        reps = [bt.poll(x) for x in slots]
        for x in slots:
            bt.release(x)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, reps

    with Batch(max_slots=len(imgs), precision="mixed", iters_per_step=iters_per_step) as bt:
        one_round(bt, len(imgs))
        done, total, iters, conv = 0, 0.0, [], []
        while done < steps:
            k = min(len(imgs), steps - done)
            dt, reps = one_round(bt, k)
            total += dt
            done += k
            iters += [r["iters"] for r in reps]
            conv += [r["converged"] for r in reps]
    return {"value": round(done / total, 3), "unit": "volumes/s", "volumes": done,
            "resident": len(imgs), "iters": iters, "converged": all(conv),
            "iters_per_step": iters_per_step}


def batched_leg(dev, n_vol, iters, log_every=8):
    """48 uneven volumes, a fixed number of ADMM iterations each: the batching engine in
    mixed precision (all admitted together) against the float32 and mixed single-volume
    solvers one after another. Setup (admission / problem creation) is timed in all three."""
    import torch
    from synth import generate, batch_shapes
    from paper_1607_00531_amd import Batch, Problem

    items = []
    t0 = time.perf_counter()
    for s, m, pe in batch_shapes(n_vol):
        v = generate(s, m, pe)
        items.append((v, torch.tensor(v.Ip, dtype=torch.float32, device=dev),
                      torch.tensor(v.Im, dtype=torch.float32, device=dev)))
        if (s + 1) % log_every == 0:
            log(f"batched leg: generated {s + 1}/{n_vol} volumes ({time.perf_counter() - t0:.0f} s)")
    faces = sum((v.m[0] + 1) * v.m[1] * v.m[2] for v, _, _ in items)
    states = [[torch.zeros((v.m[2], v.m[1], v.m[0] + 1), device=dev) for _ in range(3)]
              for v, _, _ in items]
    opts = dict(rho=RHO, max_iter=iters, eps_abs=0.0, eps_rel=0.0)

    def clear():
        for st in states:
            for t in st:
                t.zero_()
        torch.cuda.synchronize()

    def run_batch(iters_per_step):
        clear()
        t0 = time.perf_counter()
        with Batch(max_slots=n_vol, precision="mixed", iters_per_step=iters_per_step) as bt:
            slots = [bt.admit(Ip, Im, v.h, ALPHA, *st, beta=BETA, **opts)
                     for (v, Ip, Im), st in zip(items, states)]
            if any(x is None for x in slots):
                raise RuntimeError("batched leg: admission refused")
            while bt.step() > 0:
                pass
            reps = [bt.poll(x) for x in slots]
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
        assert all(r is not None and r["iters"] == iters for r in reps)
        return dt

    def run_single(precision):
        clear()
        t0 = time.perf_counter()
        for (v, Ip, Im), st in zip(items, states):
            with Problem(Ip, Im, v.h, ALPHA, BETA, precision=precision) as pr:
                r = pr.solve_admm(*st, check_every=iters, **opts)
                assert r["iters"] == iters
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    run_batch(8)                       # warm-up (code objects, graph instantiation)
    run_single("fp32")
    t_batch = run_batch(8)
    log(f"batched leg: engine {n_vol / t_batch:.2f} volumes/s")
    t_fp32 = run_single("fp32")
    log(f"batched leg: plain fp32 {n_vol / t_fp32:.2f} volumes/s")
    t_mixed = run_single("mixed")
    log(f"batched leg: single-volume mixed {n_vol / t_mixed:.2f} volumes/s")
    return {"workload": f"{n_vol} volumes, axes uniform in [96,160]x[96,160]x[48,96], PE axis "
                        f"per volume, {iters} ADMM iterations each, alpha=50 rho=1e3",
            "faces_total": faces,
            "engine_mixed": {"value": round(n_vol / t_batch, 3), "unit": "volumes/s",
                             "s_total": round(t_batch, 4)},
            "plain_fp32": {"value": round(n_vol / t_fp32, 3), "unit": "volumes/s",
                           "s_total": round(t_fp32, 4)},
            "single_volume_mixed": {"value": round(n_vol / t_mixed, 3), "unit": "volumes/s",
                                    "s_total": round(t_mixed, 4)},
            "speedup_vs_plain_fp32": round(t_fp32 / t_batch, 3)}


def served_leg(dev, seconds, rate, bases_per_class, max_iter):
    """Open-loop Poisson stream (synth.serving_requests: arrival times, request seeds, sizes
    and PE axes) served by the native request loop (epi_server_*, mixed precision) and by the
    plain float32 single-volume solver in arrival order; p50/p99 of completion - arrival.

    Every request gets its own image pair of exactly its size: a window of a large synthetic
    pair of its class (3D with its PE axis, or 2D), at an offset drawn from the request's
    seed. Generating each request's pair from scratch costs 10-20 CPU-seconds per 3D volume,
    about 20,000 CPU-seconds for a 120 s stream, so the large pairs are generated once
    (bases_per_class per class) and the windows are cut on the device before the stream
    starts (inputs resident in HBM, as for the headline)."""
    import torch
    from synth import generate, serving_requests
    from paper_1607_00531_amd import Problem, Server

    reqs = serving_requests(rate=rate, duration=seconds)
    t0 = time.perf_counter()
    bases = {}
    for cls, (m_user, pe) in {"3d0": ((240, 200, 110), 0), "3d1": ((240, 200, 110), 1),
                              "3d2": ((240, 200, 110), 2), "2d": ((256, 256), 1)}.items():
        for k in range(bases_per_class):
            v = generate(50_000 + 100 * len(bases) + k, m_user, pe)
            bases.setdefault(cls, []).append(
                (v, torch.tensor(v.Ip, dtype=torch.float32, device=dev),
                 torch.tensor(v.Im, dtype=torch.float32, device=dev)))
        log(f"served leg: {bases_per_class} base pair(s) of class {cls} "
            f"({time.perf_counter() - t0:.0f} s)")
    items = []
    for t_a, q, m_user, pe in reqs:
        cls = "2d" if len(m_user) == 2 else f"3d{pe}"
        v, Ip, Im = bases[cls][q % len(bases[cls])]
        oth = [a for a in range(len(m_user)) if a != pe]
        c = (m_user[oth[1]] if len(m_user) == 3 else 1, m_user[oth[0]], m_user[pe])   # (m3, m2, M)
        r = np.random.default_rng(q)
        o = [int(r.integers(0, Ip.shape[a] - c[a] + 1)) for a in range(3)]
        win = (slice(o[0], o[0] + c[0]), slice(o[1], o[1] + c[1]), slice(o[2], o[2] + c[2]))
        items.append((t_a, Ip[win].contiguous(), Im[win].contiguous(), v.h, len(m_user)))
    states = [[torch.zeros((Ip.shape[0], Ip.shape[1], Ip.shape[2] + 1), device=dev)
               for _ in range(3)] for _, Ip, _, _, _ in items]
    torch.cuda.synchronize()
    log(f"served leg: {len(items)} request windows on the device ({time.perf_counter() - t0:.0f} s)")

    def clear():
        for st in states:
            for t in st:
                t.zero_()
        torch.cuda.synchronize()

    def serve_engine(sel, rho_mode="fixed", rho0=RHO, iters_per_step=8, max_slots=32):
        opts = dict(rho=rho0, max_iter=max_iter, eps_abs=0.0, eps_rel=TOL, rho_mode=rho_mode)
        reps = {}
        with Server(max_slots=max_slots, precision="mixed", iters_per_step=iters_per_step) as sv:
            start = sv.clock()
            k = 0
            while len(reps) < len(sel):
                now = sv.clock() - start
                while k < len(sel) and items[sel[k]][0] <= now:
                    t_a, Ip, Im, h, nd = items[sel[k]]
                    sv.submit(sel[k], Ip, Im, h, ALPHA, *states[sel[k]], arrival=start + t_a,
                              beta=BETA, ndim=nd, **opts)
                    k += 1
                q, r, d = sv.progress()
                rep = sv.take()
                while rep is not None:
                    reps[rep["id"]] = rep
                    if len(reps) % 250 == 0:
                        log(f"served leg: {len(reps)}/{len(sel)} requests done "
                            f"({sv.clock() - start:.0f} s)")
                    rep = sv.take()
                if q == 0 and r == 0 and k < len(sel):
                    time.sleep(max(0.0, min(items[sel[k]][0] - (sv.clock() - start), 0.005)))
            total = sv.clock() - start
        lat = [x["latency_s"] for x in reps.values()]
        iters = [x["iters"] for x in reps.values()]
        return lat, iters, [x["converged"] for x in reps.values()], total

    def serve_single(sel, precision="fp32"):
        opts = dict(rho=RHO, max_iter=max_iter, eps_abs=0.0, eps_rel=TOL)
        lat, iters, conv = [], [], []
        torch.cuda.synchronize()
        start = time.perf_counter()
        for i in sel:
            t_a, Ip, Im, h, nd = items[i]
            now = time.perf_counter() - start
            if now < t_a:
                time.sleep(t_a - now)
            with Problem(Ip, Im, h, ALPHA, BETA, precision=precision, ndim=nd) as pr:
                r = pr.solve_admm(*states[i], check_every=16, **opts)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - start - t_a)
            iters.append(r["iters"])
            conv.append(r["converged"])
            if len(lat) % 250 == 0:
                log(f"served leg: {len(lat)}/{len(sel)} requests done one at a time "
                    f"({time.perf_counter() - start:.0f} s)")
        return lat, iters, conv, time.perf_counter() - start

    serve_engine(list(range(min(8, len(items)))))      # warm-up
    clear()
    out = {"workload": f"Poisson stream {rate:g} req/s for {seconds:g} s ({len(items)} "
                       f"requests), 30% 2D 128..256^2, 70% 3D 64..240x64..200x64..110, "
                       f"each request a window of its own size and seeded offset in one of "
                       f"{bases_per_class} large synthetic pair(s) per class, solve to rel. "
                       f"residual 1e-3 from zero (cap {max_iter} iterations)",
           "requests": len(items)}
    everything = list(range(len(items)))
    for name, fn in (("engine_mixed", lambda: serve_engine(everything)),
                     # residual balancing from rho = 1e6 down to the floor 1e2, as in the
                     # paper's adaptive-rho experiment (Section 4.3, Figure 7)
                     ("engine_mixed_adaptive_rho", lambda: serve_engine(everything, "adapt_floor", 1e6)),
                     ("plain_fp32", lambda: serve_single(everything))):
        lat, iters, conv, total = fn()
        clear()
        out[name] = {"volumes_per_s": round(len(lat) / total, 3),
                     "p50_ms": round(1e3 * percentile(lat, 50), 2),
                     "p99_ms": round(1e3 * percentile(lat, 99), 2),
                     "completed": len(lat), "converged": int(sum(conv)),
                     "capped": int(sum(1 for x in iters if x >= max_iter)),
                     "mean_iters": round(float(np.mean(iters)), 1), "s_total": round(total, 3)}
        log(f"served leg: {name} {json.dumps(out[name])}")
    return out


def precond_leg(dev, gn_steps=3, applies=5):
    """The preconditioner comparison of Section 5 on the 128 x 128 x 64 synthetic volume
    (PE axis 2): for each preconditioner, GN-PCG from b = 0 for a fixed number of steps
    (PCG iterations and final relative residual per step, wall time) and the device time of
    one application at the field reached (HIP events around epi_precond_apply, which also
    evaluates H_JGN). Two weights: the volume's alpha, where the transverse smoothness
    coupling dominates H_JGN, and a data-dominated alpha = 0.5."""
    import torch
    from synth import config_volume, CONFIGS
    from paper_1607_00531_amd import Problem
    cfg = CONFIGS["3d_128x128x64"]
    v = config_volume("3d_128x128x64", 0)
    Ip = torch.tensor(v.Ip, dtype=torch.float32, device=dev)
    Im = torch.tensor(v.Im, dtype=torch.float32, device=dev)
    M, m2, m3 = v.m
    out = {"workload": f"GN-PCG, {m3}x{m2}x{M} cells (canonical), {gn_steps} GN steps from "
                       f"b=0, eta=0.1, at most 30 PCG iterations per step"}
    for alpha in (cfg["alpha"], 0.5):
        res = {}
        with Problem(Ip, Im, v.h, alpha, cfg["beta"], precision="mixed") as pr:
            r = torch.randn(pr.shape_faces, device=dev)
            z = torch.empty_like(r)
            for pc in ("block", "jacobi", "sgs", "none"):
                b = torch.zeros(pr.shape_faces, device=dev)
                pr.solve_gnpcg(b.clone(), max_iter=1, use_stopping=0, precond=pc)   # warm-up
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rep = pr.solve_gnpcg(b, max_iter=gn_steps, use_stopping=0, precond=pc)
                torch.cuda.synchronize()
                wall = time.perf_counter() - t0
                pr.precond_apply(b, r, pc, out=z)
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
                torch.cuda.synchronize()
                ev[0].record()
                for _ in range(applies):
                    pr.precond_apply(b, r, pc, out=z)
                ev[1].record()
                torch.cuda.synchronize()
                npcg = sum(rep["pcg_iters"])
                res[pc] = {"pcg_iters": rep["pcg_iters"],
                           "pcg_relres": [round(x, 4) for x in rep["pcg_relres"]],
                           "J": [round(x, 6) for x in rep["J"]],
                           "gn_wall_s": round(wall, 4),
                           "ms_per_pcg_iter_incl_gn_overhead": round(1e3 * wall / max(npcg, 1), 3),
                           "apply_ms_incl_hessian_eval": round(ev[0].elapsed_time(ev[1]) / applies, 3)}
                log(f"precond alpha={alpha} {pc}: {json.dumps(res[pc])}")
        out[f"alpha={alpha}"] = res
    return out


def quality_leg(probs, vols, k=4):
    """The user-visible result on the first k headline volumes (Section 5's quality columns,
    synthetic truth only): SSD distance and normalised cross-correlation of the corrected
    pair before (b = 0) and after the ADMM solve, and the field's error against the
    synthetic truth in voxels (RMS and max over the PE faces)."""
    import torch
    out = []
    for pr, v in list(zip(probs, vols))[:k]:
        st = [torch.zeros(pr.shape_faces, device="cuda") for _ in range(3)]
        q0 = pr.corrected_images(st[0])
        rep = pr.solve_admm(*st, rho=RHO, max_iter=MAX_ITER, eps_abs=0.0, eps_rel=TOL,
                            check_every=CHECK_EVERY)
        q1 = pr.corrected_images(st[0])
        err = (st[0].double().cpu().numpy() - v.b_true) / v.h[0]
        out.append({"seed": v.seed, "iters": rep["iters"],
                    "D": [round(q0["D"], 6), round(q1["D"], 6)],
                    "ncc": [round(q0["ncc"], 5), round(q1["ncc"], 5)],
                    "field_error_vox": {"rms": round(float(np.sqrt(np.mean(err ** 2))), 4),
                                        "max": round(float(np.abs(err).max()), 4)},
                    "true_field_max_vox": round(float(np.abs(v.b_true).max() / v.h[0]), 3)})
    log(f"quality leg: {json.dumps(out)}")
    return {"workload": f"first {k} headline volumes, ADMM to rel. residual {TOL:g}; corrected "
                        "pair at b = 0 and at the solution, field against the synthetic truth",
            "volumes": out}


def multilevel_leg(imgs, vols, steps, levels=3):
    """The coarse-to-fine strategy of Section 4.4 (restart from the average of the coarser
    level's b and z, the paper's third strategy) on the headline volumes: every level
    solved to the headline's relative residual, set-up of every level (handles, tables)
    inside the timed region. Two penalty schedules: the headline's fixed rho = 1e3, and the
    paper's adaptive one (residual balancing from rho = 1e6 with the floor 1e2, Section 4.3).
    Reported beside the single-level headline, which solves the finest grid from zero."""
    import torch
    from paper_1607_00531_amd import solve_multilevel_admm
    m3, m2, M = imgs[0][0].shape
    b = torch.zeros((m3, m2, M + 1), device=imgs[0][0].device)
    out = {}
    for name, rho0, mode in (("fixed_rho", RHO, "fixed"), ("adaptive_rho_from_1e6", 1e6, "adapt_floor")):
        per, lat = [], []
        for i in range(steps):
            (Ip, Im), v = imgs[i % len(imgs)], vols[i % len(vols)]
            b.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = solve_multilevel_admm(Ip, Im, v.h, ALPHA, b, levels=levels, beta=BETA,
                                      restart="average", rho=rho0, rho_mode=mode,
                                      max_iter=MAX_ITER, eps_abs=0.0, eps_rel=TOL,
                                      check_every=CHECK_EVERY)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
            per.append(r)
        fine = [r["iters"][-1] for r in per]
        out["levels"] = " -> ".join("x".join(map(str, s)) for s in per[0]["sizes"])
        out[name] = {"volumes_per_s": round(len(lat) / sum(lat), 3),
                     "p50_ms": round(1e3 * percentile(lat, 50), 2),
                     "p99_ms": round(1e3 * percentile(lat, 99), 2),
                     "iters_per_level": [r["iters"] for r in per],
                     "finest_converged": int(sum(r["converged"][-1] for r in per)),
                     "finest_at_iteration_cap": int(sum(1 for x in fine if x >= MAX_ITER))}
        log(f"multilevel leg {name}: {json.dumps(out[name])}")
    out["workload"] = (f"coarse-to-fine ADMM, {levels} levels, restart from the average of b "
                       f"and z, every level to rel. residual {TOL:g}")
    return out


def spline_leg(imgs, vols, steps, isolated_reps, thetas=(0.0, 0.5)):
    """The smoothed cubic-spline image model (Section 5's comparison model) on the headline
    volumes, beside the linear model: set-up time of a problem (which computes both images'
    coefficients), ADMM solves to the same tolerance, and the b-step kernel launched back to
    back. The b-step moves the same bytes under both models (the coefficients replace the
    samples), so its time ratio is the cost of the four-tap evaluation."""
    import torch
    from paper_1607_00531_amd import Problem
    m3, m2, M = imgs[0][0].shape
    state = [torch.zeros((m3, m2, M + 1), device=imgs[0][0].device) for _ in range(3)]
    out = {"workload": f"ADMM to rel. residual {TOL:g}, the first {steps} headline volumes, "
                       f"mixed precision; theta in grid units"}
    for model, theta in [("linear", 0.0)] + [("spline", t) for t in thetas]:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        probs = [Problem(Ip, Im, v.h, ALPHA, BETA, precision="mixed", image_model=model,
                         theta=theta) for (Ip, Im), v in list(zip(imgs, vols))[:steps]]
        torch.cuda.synchronize()
        setup = (time.perf_counter() - t0) / len(probs)
        iters = []
        t0 = time.perf_counter()
        for pr in probs:
            for t in state:
                t.zero_()
            iters.append(pr.solve_admm(*state, rho=RHO, max_iter=MAX_ITER, eps_abs=0.0,
                                       eps_rel=TOL, check_every=CHECK_EVERY)["iters"])
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        for t in state:
            t.zero_()
        prof = probs[0].solve_admm(*state, profile=True, isolated_reps=isolated_reps, rho=RHO,
                                   max_iter=40, eps_abs=0.0, eps_rel=0.0)
        key = model if model == "linear" else f"spline theta={theta:g}"
        out[key] = {"setup_s_per_volume": round(setup, 4), "admm_iters": iters,
                    "volumes_per_s": round(len(probs) / total, 3),
                    "us_per_iteration": round(1e6 * total / max(sum(iters), 1), 2),
                    "bstep_us_back_to_back": round(prof.get("kernel_us_isolated", {}).get("bstep", 0.0), 3)}
        log(f"spline leg {key}: {json.dumps(out[key])}")
        for pr in probs:
            pr.close()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--volumes", type=int, default=20,
                    help="distinct seeds 0..volumes-1, cycled over the steps")
    ap.add_argument("--isolated-reps", type=int, default=20,
                    help="back-to-back launches per kernel family for the roofline timing")
    ap.add_argument("--cpu-iters", type=int, default=24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gn", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--max-iter", type=int, default=MAX_ITER,
                    help="ADMM iteration cap per solve (short profiling runs)")
    ap.add_argument("--no-batched", action="store_true", help="skip the 48-volume batched leg")
    ap.add_argument("--batch-volumes", type=int, default=48)
    ap.add_argument("--batch-iters", type=int, default=40)
    ap.add_argument("--no-served", action="store_true", help="skip the request-stream leg")
    ap.add_argument("--no-spline", action="store_true", help="skip the spline image model leg")
    ap.add_argument("--no-multilevel", action="store_true", help="skip the coarse-to-fine leg")
    ap.add_argument("--no-quality", action="store_true",
                    help="skip the corrected-image / field-error report")
    ap.add_argument("--no-precond", action="store_true",
                    help="skip the preconditioner comparison on the 128x128x64 volume")
    ap.add_argument("--serve-seconds", type=float, default=20.0)
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-bases", type=int, default=1,
                    help="large synthetic pairs per request class that the served requests "
                         "are cut from")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 512 MiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "decomposition is described in the design notes and not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from synth import generate, shutdown_pool
    from paper_1607_00531_amd import Problem

    dev = torch.device("cuda:0")
    vols = []
    for s in range(args.volumes):
        t0 = time.perf_counter()
        vols.append(generate(s, M_USER, PE_AXIS))
        log(f"generated volume seed {s} in {time.perf_counter() - t0:.1f} s")
    shutdown_pool()
    M, m2, m3 = vols[0].m
    n = (M + 1) * m2 * m3

    def T(a):
        return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev)

    imgs = [(T(v.Ip), T(v.Im)) for v in vols]
    state = [torch.zeros((m3, m2, M + 1), device=dev) for _ in range(3)]

    def run(precision, steps, warmup):
        probs = [Problem(Ip, Im, v.h, ALPHA, BETA, precision=precision)
                 for (Ip, Im), v in zip(imgs, vols)]
        lat, iters, conv = [], [], []

        def one(i):
            for t in state:
                t.zero_()
            return probs[i % len(probs)].solve_admm(*state, rho=RHO, max_iter=args.max_iter,
                                                    eps_abs=0.0, eps_rel=TOL,
                                                    check_every=CHECK_EVERY)

        for i in range(warmup):
            one(i)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for i in range(steps):
            t0 = time.perf_counter()
            r = one(i)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
            iters.append(r["iters"])
            conv.append(r["converged"])
        torch.cuda.synchronize()
        total = time.perf_counter() - t_start
        return probs, total, lat, iters, conv

    if args.copy_calibration:
        src = torch.ones(128 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 536870912 bytes read and written by one copy kernel")

    log("timing the mixed-precision solver")
    probs, total, lat, iters, conv = run("mixed", args.steps, args.warmup)
    value = args.steps / total
    log(f"mixed: {value:.2f} volumes/s, iterations {iters}, converged {conv}")

    engine = None
    if not args.no_served:
        log("timing the batching engine on the same volumes (all resident together)")
        engine = engine_same_volumes(imgs, vols, m3, m2, M, args.steps, args.max_iter)
        log(f"engine: {json.dumps(engine)}")

    # per-kernel device time of one profiled solve (HIP events on the library stream around
    # every launch) and, on a copy of its final state, each kernel family launched
    # back to back (one event pair per family): the latter is the roofline's kernel time
    for t in state:
        t.zero_()
    prof = probs[0].solve_admm(*state, profile=True, isolated_reps=args.isolated_reps, rho=RHO,
                               max_iter=args.max_iter, eps_abs=0.0, eps_rel=TOL,
                               check_every=CHECK_EVERY)
    nbytes = algorithmic_bytes(M, m2, m3)
    mbytes = method_bytes(M, m2, m3)
    kernels = {}
    for name, ms in prof["kernel_ms"].items():
        cnt = prof["kernel_launches"][name]
        if cnt == 0:
            continue
        avg_ms = ms / cnt
        iso_us = prof.get("kernel_us_isolated", {}).get(name, 0.0)
        gbs = nbytes[name] / (iso_us * 1e-6) / 1e9 if nbytes[name] and iso_us > 0 else None
        kernels[name] = {"avg_us_events_per_launch": round(avg_ms * 1e3, 3),
                         "avg_us_back_to_back": round(iso_us, 3), "launches": cnt,
                         "total_ms": ms, "bytes_per_launch": nbytes[name],
                         "GB_s": round(gbs, 1) if gbs else None}
        fl = mfma_flops(M, m2, m3, "mixed").get(name)
        if fl and iso_us > 0:
            tf = fl / (iso_us * 1e-6) / 1e12
            kernels[name].update({"mfma_flops_per_launch": fl, "mfma_TFLOP_s": round(tf, 1),
                                  "mfma_frac_of_bf16_peak": round(tf / 2500.0, 4)})
    peak = 8000.0
    dom = "bstep"
    t_dom = kernels[dom]["avg_us_back_to_back"] or kernels[dom]["avg_us_events_per_launch"]
    ach = mbytes[dom] / (t_dom * 1e-6) / 1e9
    traffic = counter_traffic(dom)
    iter_s = total / max(sum(iters), 1)
    roofline = {"bound": "hbm", "kernel": "bstep (k_admm_bstep<4>)", "achieved": round(ach, 1),
                "peak": peak, "unit": "GB/s", "frac": round(ach / peak, 4), "traffic": traffic,
                "bytes_per_launch": mbytes[dom],
                "bytes_rule": "8 B per cell (I+, I-) + 16 B per face (read b, z, u; write b)",
                "avg_launch_us": round(t_dom, 2),
                "timing": (f"HIP events around {args.isolated_reps} back-to-back launches on "
                           f"the library stream" if args.isolated_reps > 0 else
                           "HIP events around each launch of a profiled solve"),
                "with_fused_w_write": {
                    "bytes_per_launch": nbytes[dom],
                    "frac": round(nbytes[dom] / (t_dom * 1e-6) / 1e9 / peak, 4)},
                "whole_iteration": {
                    "bytes_per_iteration": mbytes["iteration"],
                    "bytes_rule": "8 B per cell + 36 B per face (44 B per face)",
                    "us_per_iteration": round(iter_s * 1e6, 2),
                    "frac": round(mbytes["iteration"] / iter_s / 1e9 / peak, 4),
                    "timing": "timed region / ADMM iterations (set-up and host polls included)"},
                # what limits the kernel: vector-ALU issue, from the committed SQ counters
                "valu": counter_valu(dom, t_dom)}
    iter_us = 1e3 * sum(k["total_ms"] for k in kernels.values()) / max(prof["iters"], 1)
    log(f"profile: {json.dumps(kernels)}")

    plain = None
    if not args.no_fp32:
        log("timing the plain float32 solver")
        # the same volumes in the same order as the headline, so the two differ only in
        # the z-step arithmetic
        pprobs, ptotal, plat, piters, pconv = run("fp32", args.steps, 1)
        plain = {"value": round(len(plat) / ptotal, 3), "unit": "volumes/s",
                 "p50_ms": round(1e3 * percentile(plat, 50), 2),
                 "p99_ms": round(1e3 * percentile(plat, 99), 2),
                 "us_per_iteration": round(1e6 * ptotal / max(sum(piters), 1), 2),
                 "iters": piters, "converged": all(pconv)}
        for p in pprobs:
            p.close()

    gn = None
    if not args.no_gn:
        log("timing one GN-PCG solve")
        b = torch.zeros((m3, m2, M + 1), device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = probs[0].solve_gnpcg(b, max_iter=30, use_stopping=0, rel_grad_tol=TOL)
        torch.cuda.synchronize()
        gn = {"s_per_volume": round(time.perf_counter() - t0, 4), "gn_iters": r["iters"],
              "pcg_iters": r["pcg_iters"], "converged": r["converged"],
              "stop": "|grad J_GN| <= 1e-3 |grad J_GN(0)| or 30 GN steps"}

    batched = None
    if not args.no_batched:
        log("batched leg")
        batched = batched_leg(dev, args.batch_volumes, args.batch_iters)

    served = None
    if not args.no_served:
        log("served leg")
        served = served_leg(dev, args.serve_seconds, args.serve_rate, args.serve_bases, MAX_ITER)

    quality = quality_leg(probs, vols) if not args.no_quality else None

    multilevel = None
    if not args.no_multilevel:
        log("multilevel leg")
        multilevel = multilevel_leg(imgs, vols, args.steps)

    spline = None
    if not args.no_spline:
        log("spline image model leg")
        spline = spline_leg(imgs, vols, min(4, len(vols)), args.isolated_reps)

    precond = None
    if not args.no_precond:
        log("preconditioner leg")
        precond = precond_leg(dev)

    base = None
    err = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        base, ref = cpu_baseline(vols[0], float(np.mean(iters)), args.cpu_iters)
        log(f"cpu baseline: {json.dumps(base)}")
        err = oracle_error(probs[0], ref, args.cpu_iters, (m3, m2, M + 1))
        if len(probs) > 3:
            err["converged_solve"] = converged_error(probs[3], (m3, m2, M + 1), 3)
        log(f"error vs oracle: {json.dumps(err)}")

    for p in probs:
        p.close()
    out = {
        "metric": "volumes/s at ~5M DOF to rel. residual 1e-3 vs plain FP32; p50/p99 latency",
        "value": round(value, 3),
        "unit": "volumes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * total / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (z-step DCT: 3-term split-bf16 MFMA, f32 accumulate; f64 norms)",
        "data": "synthetic",
        "config": {"workload": "ADMM, 240x200x110 cells, PE axis 1, 5302000 PE faces, "
                               "alpha=50 rho=1e3, from b=z=u=0 to rel. residual 1e-3",
                   "volumes": args.volumes, "precision": "mixed", "n_faces": n},
        "p50_ms": round(1e3 * percentile(lat, 50), 2),
        "p99_ms": round(1e3 * percentile(lat, 99), 2),
        "admm_iters": iters,
        "converged": all(conv),
        "volumes_converged": int(sum(conv)),
        "volumes_at_iteration_cap": int(sum(1 for x in iters if x >= args.max_iter)),
        "us_per_iteration_profiled": round(iter_us, 2),
        "us_per_iteration": round(1e6 * total / max(sum(iters), 1), 2),
        "roofline": roofline,
        "kernels": kernels,
        "plain_fp32": plain,
        "engine_same_volumes": engine,
        "gnpcg": gn,
        "batched": batched,
        "served": served,
        "preconditioners": precond,
        "spline_image_model": spline,
        "multilevel": multilevel,
        "quality": quality,
        "cpu_baseline": base,
        "error_vs_oracle": err,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
