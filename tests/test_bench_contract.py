"""The benchmark's host-side contract, on the CPU: one GPU only, and the
roofline helpers' arithmetic (algorithmic bytes, ALU figures)."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_algorithmic_bytes():
    n, nnz = 1000, 6000
    # forward: row pointers, column indices, x and phi (2 D floats), out
    assert bench.alg_bytes_fwd(n, nnz, 2) == 4 * (n + 1) + 4 * nnz + 16 * n + 4 * n
    # adjoint: x, phi and the gradient (3 D floats), and g
    assert bench.alg_bytes_bwd(n, nnz, 3) == 4 * (n + 1) + 4 * nnz + 36 * n + 4 * n
    # binary16 flow map: 2 bytes per component instead of 4
    assert bench.alg_bytes_fwd(n, nnz, 2) - bench.alg_bytes_fwd_f16(n, nnz, 2) == 4 * n
    # the paper's fixed-width list: 2 D indices, x and phi, out
    assert bench.alg_bytes_ell(n, 3) == n * (4 * 6 + 6 * 4 + 4)


def test_rooflines():
    r = bench.roofline(8e9, 1.0)     # 8 GB in 1 ms: 8000 GB/s, the HBM peak
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and abs(r["achieved"] - 8000.0) < 1e-9
    assert abs(r["frac"] - 1.0) < 1e-12
    a = bench.alu_roofline({"flops": 78.6e12 * 1e-3, "valu": bench.VALU_ISSUE_PEAK * 1e-3}, 1.0)
    assert a["bound"] == "alu" and a["frac"] == 1.0 and a["valu_issue_frac"] == 1.0
    assert bench.alu_roofline({}, 1.0)["achieved"] is None
