"""Helpers shared by the GPU parity tests (inputs, tolerances)."""
import numpy as np

# Tolerances of the GPU path against the FP64 oracle.
#  * objective: relative 1e-5 (float32 per-cell arithmetic, float64 sums);
#  * field: 1e-3 voxel (max abs difference / h_p);
#  * residual histories: relative 1e-4, or an absolute floor of EPS_HIST[prec] * scale where
#    scale = max(|b|, |z|) of the oracle (the float32 / split-bfloat16 rounding of b and z
#    bounds how small a difference |b - z| can be resolved).
J_REL = 1e-5
FIELD_VOX = 1e-3
HIST_REL = 1e-4
EPS_HIST = {"fp32": 2e-6, "mixed": 4e-5}


def torch_dev():
    import torch
    return torch.device("cuda:0")


def T(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=torch_dev())


def N(t):
    return t.detach().cpu().numpy().astype(np.float64)


def hist_ok(gpu, cpu, scale, prec):
    gpu, cpu = np.asarray(gpu), np.asarray(cpu)
    if gpu.shape != cpu.shape:
        return False, f"length {gpu.shape} vs {cpu.shape}"
    err = np.abs(gpu - cpu)
    lim = np.maximum(HIST_REL * np.abs(cpu), EPS_HIST[prec] * scale)
    bad = np.nonzero(err > lim)[0]
    if bad.size:
        i = bad[0]
        return False, f"iteration {i}: gpu {gpu[i]:.6e} cpu {cpu[i]:.6e} limit {lim[i]:.2e}"
    return True, ""
