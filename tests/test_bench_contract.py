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


def test_profiling_runs_need_a_filled_cache(tmp_path):
    """Under --require-cache a workload missing from --cache ends the run before
    any GPU work (profilers must not see the workload generator's kernels)."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--require-cache", "--cache", str(tmp_path),
                        "--only", "fwd3d,batched"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 3
    assert "--fill-cache" in r.stderr and "abc_3d" in r.stderr and "batched_2d" in r.stderr
    loads = bench.Workloads(str(tmp_path), "cpu", require=True)
    (tmp_path / "scale_2d.npz").write_bytes(b"")
    loads.check(["scale_2d"])
    try:
        loads.check(["scale_2d", "diff_3d"])
    except bench.MissingWorkload as e:
        assert "diff_3d" in str(e)
    else:
        raise AssertionError("missing workload not reported")
    assert bench.needed_workloads(False, ["axis"]) == ["scale_2d", "abc_3d"]


def test_profile_summaries_from_rocprof_csv(tmp_path):
    """The kernel-trace and counter summarizers on rocprofv3-shaped CSV files:
    durations per kernel, and counters scaled so that the first copy-probe
    dispatch reads exactly its size."""
    kt = tmp_path / "kt" / "host" / "1"
    kt.mkdir(parents=True)
    with open(kt / "kt_kernel_trace.csv", "w") as f:
        f.write('"Kind","Kernel_Name","Start_Timestamp","End_Timestamp"\n')
        f.write('"KERNEL_DISPATCH","fwd_kernel<2, float, true, 0, 256, false>","1000","33000"\n')
        f.write('"KERNEL_DISPATCH","fwd_kernel<2, float, true, 0, 256, false>","50000","80000"\n')
        f.write('"KERNEL_DISPATCH","void at::native::neg_kernel","90000","99000"\n')
    lines = bench.summarize_trace(str(tmp_path / "kt"), "main")
    assert len(lines) == 1 and "avg_us: 31.00" in lines[0] and "calls: 2" in lines[0]
    for counter, probe, val in (("FETCH_SIZE", 131072.0, 50000.0), ("WRITE_SIZE", 262144.0, 16384.0)):
        d = tmp_path / counter / "h" / "2"
        d.mkdir(parents=True)
        with open(d / "pmc_counter_collection.csv", "w") as f:
            f.write('"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n')
            f.write(f'"1","at::native::neg_kernel","{counter}","{probe}"\n')
            f.write(f'"2","fwd_kernel<2, float, true, 0, 256, false>","{counter}","{val}"\n')
            f.write(f'"3","fwd_kernel<2, float, true, 0, 256, false>","{counter}","{val}"\n')
    lines = bench.summarize_counters(str(tmp_path / "FETCH_SIZE"), str(tmp_path / "WRITE_SIZE"), "main")
    assert len(lines) == 1
    row = dict(p.split(": ", 1) for p in lines[0].split(" | "))
    assert float(row["fetch_factor"]) == 2.0 and float(row["write_factor"]) == 1.0
    assert row["dispatches"] == "2" and float(row["fetch_kib"]) == 50000.0


def test_advect_profile_from_rocprof_csv(tmp_path, monkeypatch):
    """The RK4 flow-map profile: median SQ counters per dispatch become FLOPs
    and VALU instructions per launch (64 per wave-level count), which
    advect_counts reads back only while the kernel source hashes match."""
    kname = bench.ADVECT_KERNELS["grid_dg"][0]
    kt = tmp_path / "kt" / "h" / "1"
    kt.mkdir(parents=True)
    with open(kt / "kt_kernel_trace.csv", "w") as f:
        f.write('"Kind","Kernel_Name","Start_Timestamp","End_Timestamp"\n')
        f.write(f'"KERNEL_DISPATCH","void ftle::(anonymous namespace)::{kname}(ftle::GridField)","0","2000000"\n')
        f.write(f'"KERNEL_DISPATCH","void ftle::(anonymous namespace)::{kname}(ftle::GridField)","0","4000000"\n')
    pm = tmp_path / "pmc" / "h" / "2"
    pm.mkdir(parents=True)
    with open(pm / "pmc_counter_collection.csv", "w") as f:
        f.write('"Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n')
        for disp, scale in ((1, 1.0), (2, 3.0), (3, 2.0)):
            for c in bench.ADVECT_COUNTERS:
                f.write(f'"{disp}","{kname}","{c}","{100.0 * scale}"\n')
    lines = bench.summarize_advect(str(tmp_path / "kt"), str(tmp_path / "pmc"))
    text = "\n".join(lines)
    assert "grid_dg_fp64_flops_per_launch = 12800" in text      # 64 x median 200
    assert "grid_dg_valu_insts_per_launch = 200" in text
    assert f"{kname:<40}     2     3.000     2.000     4.000" in text
    prof = tmp_path / "advect.txt"
    prof.write_text(text + "\n")
    monkeypatch.setattr(bench, "ADVECT_PROFILE", str(prof))
    assert bench.advect_counts("grid_dg") == {"flops": 12800.0, "valu": 200.0}
    assert bench.advect_counts("dg") == {}          # no counters for that kernel in the summary
    prof.write_text(text.replace("sha256 ftle_advect_grid.hip = ", "sha256 ftle_advect_grid.hip = 0") + "\n")
    assert bench.advect_counts("grid_dg") == {}     # taken from another source
