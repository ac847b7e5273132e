"""Benchmark of the FTLE hot path on one MI355X.

Headline: forward FTLE on the 2048x2048 jittered triangulated double-gyre
mesh (4,194,304 points, float32), points/s.  Also measured in the same run
and reported under "variants": the 160^3 ABC tetrahedral forward, the 96^3
forward+adjoint, the 48-mesh batched forward, the headline with its flow map
held as binary16 displacements, the axis stencil on the 2048^2 and 160^3
meshes, the one-ring stencil built on the GPU from those meshes' cells, and
the RK4 flow map of the 2048^2 mesh.

Every timed step reads inputs already resident in HBM.  Each workload is held
in several independent copies (mesh records, coordinates, flow map, output)
and consecutive steps rotate through them, so a step never finds its inputs
in the 256 MB Infinity Cache left there by the previous step.

Algorithmic bytes per launch (each array touched once, 32-bit CSR):
  forward  B = 4 (N + 1) + 4 nnz + 2 D s N + s N
  adjoint  B = 4 (N + 1) + 4 nnz + 3 D s N + s N     (x, flow, grad; g)
with s the storage bytes (4).  "format_bytes" is what this library's own
layout (compressed tile records with 10-bit local indices) holds for the
same launch.  The RK4 flow map is bound by float64 arithmetic: its roofline
is its float64 FLOPs per launch (hardware counters, committed summary) over
the launch time, against the float64 vector peak.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0   # MI355X HBM3E, published
FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X float64 vector, published (256 CUs x 128 FLOP/clk x 2.4 GHz)
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4   # wave64 VALU instructions/s: 4 SIMDs per CU, 4 cycles each


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def paper_bits_per_point(dim):
    """Input per point of the paper's FPGA core (Section 2.1, Table 1): 12 (2D) or
    18 (3D) double-precision values and 4 or 6 32-bit neighbour indices."""
    values, indices = (12, 4) if dim == 2 else (18, 6)
    return 64 * values, 32 * indices


def paper_required_gbps(dim, mhz):
    """Bandwidth the II=1 core needs at clock `mhz`: (fp, index) GB/s."""
    fp, idx = paper_bits_per_point(dim)
    return fp / 8 * mhz * 1e6 / 1e9, idx / 8 * mhz * 1e6 / 1e9


def alg_bytes_fwd(n, nnz, dim, s=4):
    return 4 * (n + 1) + 4 * nnz + 2 * dim * s * n + s * n


def alg_bytes_fwd_f16(n, nnz, dim):
    """As alg_bytes_fwd with the flow map held as binary16 displacements."""
    return 4 * (n + 1) + 4 * nnz + dim * 4 * n + dim * 2 * n + 4 * n


def alg_bytes_bwd(n, nnz, dim, s=4):
    return 4 * (n + 1) + 4 * nnz + 3 * dim * s * n + s * n


def alg_bytes_ell(n, dim, s=4):
    """The paper's own layout for its axis stencil (Section 2.2, Table 1): a
    fixed-width list of 2*dim 32-bit neighbour indices per point (-1 where a
    side has none), no row pointers, then x and phi read and FTLE written."""
    return n * (4 * 2 * dim + 2 * dim * s + s)


def format_bytes_fwd(mesh, dim, s=4):
    st = mesh.tile_stats()
    return st["record_bytes"] + 2 * dim * s * mesh.n + s * mesh.n


def cached(name, make, cache_dir, dev):
    """Generate a workload, or load it from cache_dir (written by an earlier run).

    Profiling runs use the cache so that the profiler sees the FTLE kernels and
    not the generator's RK4 kernels.
    """
    import numpy as np
    import torch

    from workloads import configs
    if not cache_dir:
        return make()
    path = os.path.join(cache_dir, name + ".npz")
    if os.path.exists(path):
        z = np.load(path)
        ws = []
        for k in range(int(z["count"])):
            extra = {"weights": z[f"w{k}"]} if f"w{k}" in z else {}
            ws.append(configs.Workload(str(z[f"name{k}"]), int(z[f"dim{k}"]), z[f"x{k}"], z[f"c{k}"],
                                       torch.as_tensor(z[f"f{k}"], device=dev), float(z[f"T{k}"]),
                                       str(z[f"dt{k}"]), extra))
        return ws if bool(z["is_list"]) else ws[0]
    w = make()
    ws = w if isinstance(w, list) else [w]
    arrays = {"count": len(ws), "is_list": isinstance(w, list)}
    for k, x in enumerate(ws):
        arrays.update({f"name{k}": x.name, f"dim{k}": x.dim, f"x{k}": x.coords, f"c{k}": x.cells,
                       f"f{k}": x.flow_numpy(), f"T{k}": x.T, f"dt{k}": x.dtype})
        if "weights" in x.extra:
            arrays[f"w{k}"] = x.extra["weights"]
    os.makedirs(cache_dir, exist_ok=True)
    np.savez(path, **arrays)
    return w


def time_steps(fns, steps, warmup, torch):
    """Run warmup untimed steps, then exactly `steps` timed ones; ms per step."""
    for i in range(warmup):
        fns[i % len(fns)]()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        fns[i % len(fns)]()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


COUNTERS = os.path.join(ROOT, "profiles", "ftle_counters_fetch_write.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2408_02758_amd", "csrc", "ftle_kernels.hip")


def kernel_source_sha256():
    import hashlib
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def measured_traffic():
    """HBM bytes per dispatch by kernel name, from the committed rocprofv3 summary
    (FETCH_SIZE and WRITE_SIZE scaled by the copy-probe factors), or {} when the
    summary was taken from another version of the kernel source."""
    if not os.path.exists(COUNTERS):
        return {}
    meta, per_kernel = {}, {}
    with open(COUNTERS) as f:
        for ln in f:
            ln = ln.strip()
            if not ln or ln.startswith("#"):
                continue
            if ln.startswith("kernel:"):
                fields = dict(part.strip().split(": ", 1) for part in ln.split(" | "))
                per_kernel[fields["kernel"]] = (float(fields["fetch_kib"]), float(fields["write_kib"]))
            elif "=" in ln:
                k, v = ln.split("=", 1)
                meta[k.strip()] = v.strip()
    if meta.get("kernel_source_sha256") != kernel_source_sha256():
        return {}
    ff, wf = float(meta["fetch_factor"]), float(meta["write_factor"])
    return {k: round((fe * ff + wr * wf) * 1024) for k, (fe, wr) in per_kernel.items()}


ADVECT_PROFILE = os.path.join(ROOT, "profiles", "ftle_advect_rk4.txt")
ADVECT_SRC = os.path.join(ROOT, "paper_2408_02758_amd", "csrc", "ftle_advect.hip")


def advect_counts(flow="double_gyre"):
    """Float64 FLOPs and VALU instructions per launch of the measured flow map
    ("double_gyre": the 2048^2 grid; "abc": the 160^3 grid), from the committed
    rocprofv3 summary, or {} when that summary was taken from another version
    of the kernel source."""
    import hashlib
    if not os.path.exists(ADVECT_PROFILE):
        return {}
    meta = {}
    with open(ADVECT_PROFILE) as f:
        for ln in f:
            ln = ln.strip()
            if ln and not ln.startswith("#") and "=" in ln:
                k, v = ln.split("=", 1)
                meta[k.strip()] = v.strip()
    with open(ADVECT_SRC, "rb") as f:
        if meta.get("advect_source_sha256") != hashlib.sha256(f.read()).hexdigest():
            return {}
    key = "dg" if flow == "double_gyre" else "abc"
    if f"{key}_fp64_flops_per_launch" not in meta:
        return {}
    return {"flops": float(meta[f"{key}_fp64_flops_per_launch"]), "valu": float(meta[f"{key}_valu_insts_per_launch"])}


def alu_roofline(counts, ms):
    """Float64 ALU roofline of one launch from its counted FLOPs and VALU instructions."""
    if not counts:
        return {"bound": "alu", "achieved": None, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": None,
                "traffic": None}
    tf = counts["flops"] / (ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(tf, 2), "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tf / FP64_VECTOR_PEAK_TFLOPS, 4), "traffic": None,
            "fp64_flops_per_launch": counts["flops"],
            "valu_issue_frac": round(counts["valu"] / (ms * 1e-3) / VALU_ISSUE_PEAK, 4)}


def traffic_for(traffic, *names):
    """Sum of the per-dispatch traffic of the named kernels, or None if any is missing."""
    try:
        return sum(traffic[n] for n in names)
    except KeyError:
        return None


def roofline(alg_bytes, ms):
    gbps = alg_bytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(gbps / HBM_PEAK_GBPS, 4), "traffic": None}


def cpu_baseline(w, threads):
    """The FP64 oracle, as it stands, on the headline workload (per-point loop only)."""
    import numpy as np

    import oracle
    oracle.set_threads(threads)
    st = oracle.ring1(w.dim, w.n, w.cells)
    x = w.coords.astype(np.float64)
    phi = w.flow_numpy().astype(np.float64)
    t0 = time.perf_counter()
    reps = 0
    while True:
        oracle.ftle(w.dim, x, phi, st, w.T)
        reps += 1
        el = time.perf_counter() - t0
        if el >= 2.0 or reps >= 20:
            break
    return {"value": round(w.n * reps / el, 1), "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": f"all {w.n} points of the 2048^2 workload x{reps} passes, per-point loop only "
                      f"(stencil built beforehand), float64, OpenMP {threads} threads"}


def stencil_vs_oracle(w, row_ptr, col):
    """The GPU-built one-ring stencil against the oracle's, entry for entry."""
    import numpy as np

    import oracle
    ref = oracle.ring1(w.dim, w.n, w.cells)
    return {"row_ptr_equal": bool(np.array_equal(row_ptr, ref.row_ptr)),
            "col_equal": bool(np.array_equal(col, ref.col)), "nnz": int(ref.col.size)}


def error_vs_oracle(w, got, sel=None, stencil="ring1"):
    """Error of a float32 GPU FTLE field against the FP64 oracle on the same
    (float32-rounded) inputs: max |error| over finite points, and the relative
    error where the top eigenvalue is separated (gap >= 1e-3) and |ln lambda|
    >= 0.05, the mask the parity tests use."""
    import numpy as np

    import oracle
    st = oracle.ring1(w.dim, w.n, w.cells)
    if stencil == "axis":
        st = oracle.axis(w.dim, w.coords.astype(np.float64), st)
    ref, gap, _ = oracle.ftle(w.dim, w.coords.astype(np.float64), w.flow_numpy().astype(np.float64), st, w.T,
                              sel=sel, diagnostics=True)
    g = np.asarray(got, dtype=np.float64)
    if sel is not None:
        g = g[sel]
    fin = np.isfinite(ref)
    mask = fin & (gap >= 1e-3) & (2 * abs(w.T) * np.abs(ref) >= 0.05)
    rel = np.abs(g[mask] - ref[mask]) / np.abs(ref[mask])
    return {"points": int(ref.size), "max_abs_err": float(np.abs(g[fin] - ref[fin]).max(initial=0)),
            "masked_max_rel_err": float(rel.max(initial=0)), "masked_p99_rel_err": float(np.percentile(rel, 99)) if rel.size else 0.0,
            "mask_fraction": round(float(mask.mean()), 4), "nan_masks_equal": bool(np.array_equal(np.isnan(g), np.isnan(ref)))}


def grad_error_vs_oracle(w, g_in, grad):
    """Max |error| of the GPU adjoint over the max |gradient| of the FP64 oracle,
    leaving out points next to a nearly repeated top eigenvalue (gap < 1e-6),
    whose eigenvector is ill-defined (as the parity tests do)."""
    import numpy as np

    import oracle
    st = oracle.ring1(w.dim, w.n, w.cells)
    x, phi = w.coords.astype(np.float64), w.flow_numpy().astype(np.float64)
    ref = oracle.ftle_grad(w.dim, x, phi, st, w.T, np.asarray(g_in, dtype=np.float64))
    _, gap, _ = oracle.ftle(w.dim, x, phi, st, w.T, diagnostics=True)
    bad = np.zeros(w.n, bool)
    for i in np.nonzero(~(gap >= 1e-6))[0]:
        bad[i] = True
        bad[st.col[st.row_ptr[i]:st.row_ptr[i + 1]]] = True
    got = np.asarray(grad, dtype=np.float64).reshape(ref.shape)
    return {"points": int(w.n), "excluded_near_repeated_eigenvalue": int(bad.sum()),
            "max_err_over_max_grad": float(np.abs(got - ref)[~bad].max() / np.abs(ref).max())}


def oracle_advect(x0, t0, T, flow="double_gyre", dt=0.01):
    """The FP64 oracle's RK4 flow map of the given particles."""
    import oracle
    return oracle.advect_rk4(flow, x0, t0, T, dt)


def copy_probe_gbps(torch, dev, mib=1024, reps=10):
    """Bandwidth of a plain elementwise kernel (torch.neg: mib MiB read + mib MiB written)."""
    src = torch.ones(mib << 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(2):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.neg(src, out=dst)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return round(2 * (mib << 20) / t / 1e9, 1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--copies", type=int, default=3, help="input copies rotated between steps")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", default="",
                    help="comma list of: f16,fwd3d,fwdbwd,batched,axis,neighbours,advect (the 2D headline always runs)")
    ap.add_argument("--cache", default="", help="directory to keep generated workloads in (npz)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one plain elementwise copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the FTLE hot path is "
              "built and measured on a single MI355X (meshes would be split into Morton ranges, one per GPU, "
              "with a one-ring halo exchange of the flow map).", flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2408_02758_amd as F
    from workloads import configs

    dev = "cuda:0"
    torch.cuda.set_device(0)
    only = set(filter(None, args.only.split(",")))
    want = lambda k: (not only) or (k in only)  # noqa: E731
    R = max(1, args.copies)
    result = {}
    variants = {}

    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)       # reads and writes exactly copy_probe_mib MiB each
        torch.cuda.synchronize()
        del src, dst

    # ---- headline: 2D forward at 2048^2 ------------------------------------
    log("generating 2048^2 double-gyre workload (RK4 on the GPU)")
    w2 = cached("scale_2d", lambda: configs.scale_2d(dev), args.cache, dev)
    log("building meshes")
    meshes2 = [F.Mesh(w2.coords, w2.cells, "f32") for _ in range(R)]
    nnz2 = meshes2[0].info()["nnz"]
    flows2 = [w2.flow.to(dev).clone().contiguous() for _ in range(R)]
    outs2 = [torch.empty(w2.n, dtype=torch.float32, device=dev) for _ in range(R)]
    fns = [lambda k=k: meshes2[k].forward(flows2[k], w2.T, out=outs2[k]) for k in range(R)]
    log("timing 2D forward")
    ms = time_steps(fns, args.steps, args.warmup, torch)
    B = alg_bytes_fwd(w2.n, nnz2, 2)
    pts = w2.n / (ms * 1e-3)
    traffic = measured_traffic()
    rl = roofline(B, ms)
    rl["traffic"] = traffic_for(traffic, f"fwd_kernel<2, float, true, 0, {meshes2[0].blocks()[0]}, false>")
    rl["alg_bytes_per_launch"] = B
    rl["format_bytes_per_launch"] = format_bytes_fwd(meshes2[0], 2)
    rl["format_frac"] = round(rl["format_bytes_per_launch"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
    nan = int(torch.isnan(outs2[0]).sum().item())
    keep = {"2d": outs2[0].cpu().numpy()}   # GPU fields checked against the oracle at the end
    result.update({
        "metric": "FTLE points/s (fwd, fwd+bwd, batched) + % HBM roofline at stated err vs FP64",
        "value": round(pts, 1), "unit": "points/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "2D plain FTLE forward, 2048x2048 jittered triangulated grid, double gyre "
                               "(A=0.1, eps=0.25, omega=2pi/10), RK4 dt=0.01, T=15",
                   "points": w2.n, "nnz": nnz2, "T": w2.T, "stencil": "ring1", "input_copies": R,
                   "nan_outputs": nan},
        "roofline": rl,
    })
    log(f"2D forward: {ms * 1e3:.2f} us/step, {pts / 1e9:.2f} G points/s, {rl['achieved']} GB/s alg")
    copy_gbps = copy_probe_gbps(torch, dev)
    result["copy_probe"] = {"GBps": copy_gbps, "kernel": "torch.neg, 1 GiB read + 1 GiB written"}
    rl["frac_of_copy_probe"] = round(rl["achieved"] / copy_gbps, 4)
    del fns

    # ---- variants ----------------------------------------------------------
    if not args.no_variants:
        steps_v = max(10, args.steps // 2)
        if want("f16"):
            # the headline with the flow map stored as binary16 displacements
            # (4 bytes per point instead of 8), float32 arithmetic
            log("f16 flow storage: 2048^2 forward")
            d16 = [meshes2[k].encode_flow_f16(flows2[k]) for k in range(R)]
            fns = [lambda k=k: meshes2[k].forward_f16(d16[k], w2.T, out=outs2[k]) for k in range(R)]
            t = time_steps(fns, args.steps, args.warmup, torch)
            Bh = alg_bytes_fwd_f16(w2.n, nnz2, 2)
            variants["fwd_2d_2048_f16flow"] = {
                "workload": "2D forward on the 2048^2 workload with the flow map stored as binary16 displacements "
                            "phi - x (float32 arithmetic on the decoded map)",
                "points": w2.n, "nnz": nnz2, "ms_per_step": round(t, 5), "points_per_s": round(w2.n / (t * 1e-3), 1),
                "roofline": dict(roofline(Bh, t), alg_bytes_per_launch=Bh,
                                 traffic=traffic_for(traffic, f"fwd16_kernel<{meshes2[0].blocks()[0]}>"))}
            log(f"f16 flow storage: {t * 1e3:.2f} us/step")
            keep["f16"] = outs2[0].cpu().numpy()
            del d16, fns
        if want("fwd3d"):
            log("generating 160^3 ABC workload")
            w3 = cached("abc_3d", lambda: configs.abc_3d(dev), args.cache, dev)
            ms3 = [F.Mesh(w3.coords, w3.cells, "f32") for _ in range(R)]
            nnz3 = ms3[0].info()["nnz"]
            fl3 = [w3.flow.to(dev).clone().contiguous() for _ in range(R)]
            ou3 = [torch.empty(w3.n, dtype=torch.float32, device=dev) for _ in range(R)]
            fns = [lambda k=k: ms3[k].forward(fl3[k], w3.T, out=ou3[k]) for k in range(R)]
            ms3[0].fp64_hits(reset=True)
            t = time_steps(fns, steps_v, args.warmup, torch)
            hits = ms3[0].fp64_hits()
            calls0 = (args.warmup + steps_v + R - 1) // R
            B3 = alg_bytes_fwd(w3.n, nnz3, 3)
            variants["fwd_3d_160"] = {
                "workload": "3D plain FTLE forward, 160^3 Kuhn tetrahedral grid, ABC flow, RK4 dt=0.02, T=10",
                "points": w3.n, "nnz": nnz3, "ms_per_step": round(t, 5), "points_per_s": round(w3.n / (t * 1e-3), 1),
                "roofline": dict(roofline(B3, t), alg_bytes_per_launch=B3,
                                 format_bytes_per_launch=format_bytes_fwd(ms3[0], 3),
                                 traffic=traffic_for(traffic, f"fwd_kernel<3, float, true, 0, {ms3[0].blocks()[0]}, false>")),
                "fp64_eigen_recomputes_per_call": round(hits / max(1, calls0), 1)}
            log(f"3D forward: {t * 1e3:.2f} us/step")
            keep["3d"] = (w3, ou3[0].cpu().numpy())
            del fns, ms3, fl3, ou3
        if want("fwdbwd"):
            log("generating 96^3 ABC workload (differentiated)")
            wd = cached("diff_3d", lambda: configs.diff_3d(dev), args.cache, dev)
            msd = [F.Mesh(wd.coords, wd.cells, "f32") for _ in range(R)]
            nnzd = msd[0].info()["nnz"]
            fld = [wd.flow.to(dev).clone().contiguous() for _ in range(R)]
            gw = torch.as_tensor(wd.extra["weights"], dtype=torch.float32, device=dev)
            outd = [torch.empty(wd.n, dtype=torch.float32, device=dev) for _ in range(R)]
            taped = [torch.empty(wd.n * 7, dtype=torch.float32, device=dev) for _ in range(R)]
            gradd = [torch.empty(wd.n, 3, dtype=torch.float32, device=dev) for _ in range(R)]

            def step(k):
                msd[k].forward_tape(fld[k], wd.T, out=outd[k], tape=taped[k])
                msd[k].backward_tape(taped[k], gw, grad_flow=gradd[k])
            fns = [lambda k=k: step(k) for k in range(R)]
            t = time_steps(fns, steps_v, args.warmup, torch)
            Bd = alg_bytes_fwd(wd.n, nnzd, 3) + alg_bytes_bwd(wd.n, nnzd, 3)
            variants["fwd_bwd_3d_96"] = {
                "workload": "3D FTLE forward + adjoint (dL/dflow, L = sum w_i FTLE_i), 96^3 Kuhn grid, ABC flow, T=10",
                "points": wd.n, "nnz": nnzd, "ms_per_step": round(t, 5), "points_per_s": round(wd.n / (t * 1e-3), 1),
                "roofline": dict(roofline(Bd, t), alg_bytes_per_launch=Bd,
                                 traffic=traffic_for(traffic, f"fwd_kernel<3, float, true, 1, {msd[0].blocks()[0]}, false>",
                                                     f"bwd_kernel<3, float, {msd[0].blocks()[1]}, false, false>"))}
            log(f"fwd+bwd: {t * 1e3:.2f} us/step")
            keep["fwdbwd"] = (wd, outd[0].cpu().numpy(), gw.cpu().numpy(), gradd[0].cpu().numpy())
            del fns, msd, fld, outd, taped, gradd
        if want("batched"):
            log("generating the 48-mesh batched workload")
            wb = cached("batched_2d", lambda: configs.batched_2d(dev), args.cache, dev)
            Rb = 2
            sets = []
            for _ in range(Rb):
                mb = [F.Mesh(w.coords, w.cells, "f32") for w in wb]
                fb = [w.flow.to(dev).clone().contiguous() for w in wb]
                ob = [torch.empty(w.n, dtype=torch.float32, device=dev) for w in wb]
                sets.append((mb, fb, ob))
            Ts = [w.T for w in wb]
            fns = [F.BatchedCall(s[0], s[1], Ts, outs=s[2]) for s in sets]
            t = time_steps(fns, steps_v, args.warmup, torch)
            npts = sum(w.n for w in wb)
            nnzb = sum(m.info()["nnz"] for m in sets[0][0])
            Bb = sum(alg_bytes_fwd(m.n, m.info()["nnz"], 2) for m in sets[0][0])
            variants["batched_2d_48"] = {
                "workload": "48 jittered triangulated double-gyre meshes, sides log-uniform in [64,1024], "
                            "own t0 and T each, one persistent launch from a HIP graph",
                "points": npts, "nnz": nnzb, "ms_per_step": round(t, 5), "points_per_s": round(npts / (t * 1e-3), 1),
                "autotuned": F.batched_config(sets[0][0])}
            cfg = variants["batched_2d_48"]["autotuned"]
            variants["batched_2d_48"]["roofline"] = dict(
                roofline(Bb, t), alg_bytes_per_launch=Bb,
                traffic=traffic_for(traffic, f"batched_kernel<2, float, {cfg['block']}, false>"))
            log(f"batched: {t * 1e3:.2f} us/step")
            keep["batched"] = [(wb[k], sets[0][2][k].cpu().numpy()) for k in (0, 24, 47)]
            del fns, sets
        if want("axis"):
            # the paper's stencil (one nearest neighbour per side of each axis),
            # measured against the paper's fixed-width list (alg_bytes_ell)
            for dim, name, wl in ((2, "axis_2d_2048", lambda: w2),
                                  (3, "axis_3d_160", lambda: cached("abc_3d", lambda: configs.abc_3d(dev),
                                                                    args.cache, dev))):
                log(f"{name}: building meshes")
                wa = wl()
                ma = [F.Mesh(wa.coords, wa.cells, "f32", stencil="axis") for _ in range(R)]
                fa = [wa.flow.to(dev).clone().contiguous() for _ in range(R)]
                oa = [torch.empty(wa.n, dtype=torch.float32, device=dev) for _ in range(R)]
                fns = [lambda k=k: ma[k].forward(fa[k], wa.T, out=oa[k]) for k in range(R)]
                t = time_steps(fns, steps_v, args.warmup, torch)
                Be = alg_bytes_ell(wa.n, dim)
                variants[name] = {
                    "workload": f"{dim}D plain FTLE forward with the paper's axis stencil (2*dim nearest neighbours "
                                f"along the axes, Section 2.2), on the {'2048^2' if dim == 2 else '160^3'} workload",
                    "points": wa.n, "nnz": ma[0].info()["nnz"], "ms_per_step": round(t, 5),
                    "points_per_s": round(wa.n / (t * 1e-3), 1),
                    "roofline": dict(roofline(Be, t), alg_bytes_per_launch=Be, alg_model="paper's fixed-width list",
                                     format_bytes_per_launch=format_bytes_fwd(ma[0], dim))}
                log(f"{name}: {t * 1e3:.2f} us/step")
                keep[name] = (wa, oa[0].cpu().numpy())
                del fns, ma, fa, oa
        if want("neighbours"):
            # the one-ring stencil built on the GPU from the cells (edge pairs,
            # radix sort, deduplication, CSR), each call allocating its sort
            # buffers and returning the entry count to the host
            for name, wk in (("ring1_csr_2d_2048", lambda: w2),
                             ("ring1_csr_3d_160", lambda: cached("abc_3d", lambda: configs.abc_3d(dev), args.cache,
                                                                   dev))):
                wn = wk()
                log(f"{name}: one-ring stencil on the GPU")
                cells_d = torch.as_tensor(wn.cells, dtype=torch.int32, device=dev).contiguous()
                rp, col = F.ring1_csr(wn.dim, wn.n, cells_d)
                t = time_steps([lambda: F.ring1_csr(wn.dim, wn.n, cells_d)], 5, 1, torch)
                Bn = 4 * cells_d.numel() + 8 * (wn.n + 1) + 4 * col.numel()
                variants[name] = {
                    "workload": f"one-ring CSR of the {'2048^2 triangle' if wn.dim == 2 else '160^3 tetrahedron'} "
                                "mesh from its cells on the GPU",
                    "points": wn.n, "cells": int(cells_d.shape[0]), "nnz": int(col.numel()),
                    "ms_per_step": round(t, 4), "points_per_s": round(wn.n / (t * 1e-3), 1),
                    "roofline": dict(roofline(Bn, t), alg_bytes_per_launch=Bn,
                                     alg_model="cells read once, CSR written once")}
                log(f"{name}: {t:.2f} ms per stencil")
                keep[name] = (wn, rp.cpu().numpy(), col.cpu().numpy())
                del cells_d, rp, col, wn
        if want("advect"):
            # the step before the path: the 2048^2 double-gyre flow map by RK4 on
            # the GPU (float64 arithmetic, float32 output), as the headline's
            # input was generated (T = 15, dt = 0.01: 1500 steps per particle)
            log("advect_2d_2048: RK4 flow map on the GPU")
            x0 = torch.as_tensor(w2.coords, dtype=torch.float32, device=dev).contiguous()
            t0 = float(w2.extra.get("t0", 0.0))
            phi = torch.empty_like(x0)
            F.advect_rk4("double_gyre", x0, t0, w2.T, 0.01, out=phi)
            t = time_steps([lambda: F.advect_rk4("double_gyre", x0, t0, w2.T, 0.01, out=phi)], 3, 1, torch)
            nsteps = math.ceil(abs(w2.T) / 0.01 - 1e-9)
            variants["advect_2d_2048"] = {
                "workload": "RK4 flow map of the 2048^2 jittered grid in the double gyre, t0 = 0, T = 15, dt = 0.01 "
                            "(float64 arithmetic, float32 output)",
                "points": w2.n, "steps_per_point": nsteps, "ms_per_step": round(t, 4),
                "points_per_s": round(w2.n / (t * 1e-3), 1),
                "particle_steps_per_s": round(w2.n * nsteps / (t * 1e-3), 1),
                "roofline": alu_roofline(advect_counts(), t)}
            log(f"advect_2d_2048: {t:.2f} ms per flow map")
            keep["advect"] = (w2, x0.cpu().numpy(), t0, phi.cpu().numpy())
            del x0, phi
            # the 160^3 ABC flow map (T = 10, dt = 0.02: 500 steps per particle)
            w3a = cached("abc_3d", lambda: configs.abc_3d(dev), args.cache, dev)
            log("advect_3d_160: RK4 flow map on the GPU")
            x0 = torch.as_tensor(w3a.coords, dtype=torch.float32, device=dev).contiguous()
            phi = torch.empty_like(x0)
            F.advect_rk4("abc", x0, 0.0, w3a.T, 0.02, out=phi)
            t = time_steps([lambda: F.advect_rk4("abc", x0, 0.0, w3a.T, 0.02, out=phi)], 3, 1, torch)
            nsteps = math.ceil(abs(w3a.T) / 0.02 - 1e-9)
            variants["advect_3d_160"] = {
                "workload": "RK4 flow map of the 160^3 Kuhn grid in the ABC flow, t0 = 0, T = 10, dt = 0.02 "
                            "(float64 arithmetic, float32 output)",
                "points": w3a.n, "steps_per_point": nsteps, "ms_per_step": round(t, 4),
                "points_per_s": round(w3a.n / (t * 1e-3), 1),
                "particle_steps_per_s": round(w3a.n * nsteps / (t * 1e-3), 1),
                "roofline": alu_roofline(advect_counts("abc"), t)}
            log(f"advect_3d_160: {t:.2f} ms per flow map")
            keep["advect_abc"] = (w3a, x0.cpu().numpy(), phi.cpu().numpy())
            del x0, phi, w3a
        for v in variants.values():
            if v["roofline"]["bound"] == "hbm":
                v["roofline"]["frac_of_copy_probe"] = round(v["roofline"]["achieved"] / copy_gbps, 4)
        result["variants"] = variants

    if not args.no_cpu_baseline:
        try:
            threads = min(16, len(os.sched_getaffinity(0)))
        except AttributeError:
            threads = min(16, os.cpu_count() or 1)
        log(f"timing the FP64 oracle on {threads} host threads")
        result["cpu_baseline"] = cpu_baseline(w2, threads)
        # the float32 fields of this run against the FP64 oracle on the same inputs
        log("checking the GPU fields against the FP64 oracle")
        err = {"2d_2048": error_vs_oracle(w2, keep["2d"])}
        rng = np.random.default_rng(0)
        if "3d" in keep:
            w3, got3 = keep["3d"]
            err["3d_160_sample"] = error_vs_oracle(w3, got3, sel=np.sort(rng.choice(w3.n, 200000, replace=False)))
        if "fwdbwd" in keep:
            wd, outd0, g0, grad0 = keep["fwdbwd"]
            err["fwd_bwd_96"] = {"ftle": error_vs_oracle(wd, outd0), "grad": grad_error_vs_oracle(wd, g0, grad0)}
        if "batched" in keep:
            err["batched_48"] = {w.name: error_vs_oracle(w, got) for w, got in keep["batched"]}
        if "f16" in keep:
            # against the oracle on the original float32 flow map: the accuracy
            # the binary16 storage gives up (its parity on the decoded map is tested)
            err["f16flow_2d_2048_vs_float32_flow"] = error_vs_oracle(w2, keep["f16"])
        for name in ("ring1_csr_2d_2048", "ring1_csr_3d_160"):
            if name in keep:
                err[name] = stencil_vs_oracle(*keep[name])
        if "advect" in keep:
            wa, x0, t0, phi = keep["advect"]
            sel = np.sort(rng.choice(wa.n, 20000, replace=False))
            ref = oracle_advect(x0[sel].astype(np.float64), t0, wa.T)
            err["advect_2d_2048_sample"] = {"points": int(sel.size),
                                            "max_abs_err": float(np.abs(phi[sel].astype(np.float64) - ref).max())}
        if "advect_abc" in keep:
            wa, x0, phi = keep["advect_abc"]
            sel = np.sort(rng.choice(wa.n, 20000, replace=False))
            ref = oracle_advect(x0[sel].astype(np.float64), 0.0, wa.T, "abc", 0.02)
            err["advect_3d_160_sample"] = {"points": int(sel.size),
                                           "max_abs_err": float(np.abs(phi[sel].astype(np.float64) - ref).max())}
        if "axis_2d_2048" in keep:
            wa, got = keep["axis_2d_2048"]
            err["axis_2d_2048"] = error_vs_oracle(wa, got, stencil="axis")
        if "axis_3d_160" in keep:
            wa, got = keep["axis_3d_160"]
            err["axis_3d_160_sample"] = error_vs_oracle(wa, got, sel=np.sort(rng.choice(wa.n, 200000, replace=False)),
                                                        stencil="axis")
        result["error_vs_fp64"] = err

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
