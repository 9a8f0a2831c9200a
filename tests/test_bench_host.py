"""Host-side parts of bench.py (no GPU): the one-GPU guard, the byte and flop accounting,
and the counter-summary lookup that keys on the kernel sources."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_algorithmic_bytes_of_the_admm_kernels():
    import bench
    M, m2, m3 = 240, 200, 110
    n, N = (M + 1) * m2 * m3, M * m2 * m3
    b = bench.algorithmic_bytes(M, m2, m3)
    assert b["bstep"] == 4 * (2 * N + 5 * n) == 148_280_000
    assert b["dct_axis3"] == 8 * n
    # 110 slices x (hi, lo) x 14 row tiles (both halves) x 4 contraction steps x 1 KiB
    assert b["dct_axis2_fused"] - 8 * n == bench.zop_bytes(m2, m3) == 110 * 2 * 14 * 4 * 1024
    assert bench.algorithmic_bytes(M, m2, m3, zop=False)["dct_axis2_fused"] == 8 * n
    assert b["dct_last_epilogue"] == 24 * n


def test_method_bytes_are_44_per_face():
    """What the ADMM iteration must move with every line and tile staged on chip once:
    the b-step reads both images (8 B per cell) and b, z, u and writes b (16 B per face);
    the z- and u-step read b, u and the old z and write z, u (20 B per face)."""
    import bench
    M, m2, m3 = 240, 200, 110
    n, N = (M + 1) * m2 * m3, M * m2 * m3
    b = bench.method_bytes(M, m2, m3)
    assert b["bstep"] == 8 * N + 16 * n == 127_072_000
    assert b["zu_step"] == 20 * n
    assert b["iteration"] == b["bstep"] + b["zu_step"] == 233_112_000


def test_host_cpu_is_reported():
    import bench
    model, ncpu = bench.host_cpu()
    assert isinstance(model, str) and model and ncpu >= 1


def test_mfma_flops_of_the_split_transform():
    """Even/odd halves: 2c^2 + 2f^2 per column of length m (c, f the half lengths), three
    products per multiply-add in mixed precision; full 2m^2 per column in float32. The j-axis
    pass is one product with a fixed rho in mixed precision (per-slice operator), two
    otherwise."""
    import bench
    M, m2, m3 = 240, 200, 110
    n = (M + 1) * m2 * m3
    mixed, fp32 = bench.mfma_flops(M, m2, m3, "mixed"), bench.mfma_flops(M, m2, m3, "fp32")
    assert mixed["dct_axis3"] == 3 * (2 * 55 * 55 * 2) / 110 * n
    assert mixed["dct_axis2_fused"] == 3 * (2 * 100 * 100 * 2) / 200 * n
    adaptive = bench.mfma_flops(M, m2, m3, "mixed", fixed_rho=False)
    assert adaptive["dct_axis2_fused"] == 2 * mixed["dct_axis2_fused"]
    assert fp32["dct_axis2_fused"] == 2 * 2 * m2 * n
    odd = bench.mfma_flops(10, 7, 5, "mixed")        # odd lengths: c = 4, f = 3 for m = 7
    assert odd["dct_axis2_fused"] == 3 * (2 * 16 + 2 * 9) / 7 * (11 * 7 * 5)


def test_counter_traffic_keys_on_the_kernel_sources():
    import bench
    t = bench.counter_traffic("bstep")
    assert t is None or t > bench.algorithmic_bytes(240, 200, 110)["bstep"] * 0.9
    assert bench.counter_traffic("no_such_kernel") is None


def test_counter_valu_keys_on_the_kernel_sources():
    import bench
    v = bench.counter_valu("bstep", 33.0)
    if v is not None:
        # one b-step launch: 22,000 wavefronts (one per PE line) of some hundreds of VALU
        # instructions each; the issue peak is 1024 SIMDs x 2.4 GHz / 4 cycles
        assert v["peak"] == 1024 * 2.4 / 4
        assert 22000 * 100 < v["wave_instructions_per_launch"] < 22000 * 2000
        assert abs(v["frac"] - v["achieved"] / v["peak"]) < 1e-3
    assert bench.counter_valu("no_such_kernel", 33.0) is None
    assert bench.counter_valu("bstep", 0.0) is None
