"""Benchmark of the FTLE hot path on one MI355X.

Headline: forward FTLE on the 2048x2048 jittered triangulated double-gyre
mesh (4,194,304 points, float32), points/s.  Also measured in the same run
and reported under "variants": the 160^3 ABC tetrahedral forward, the 96^3
forward+adjoint, the 48-mesh batched forward, the headline in float64 (the
paper's precision), the headline with its flow map held as binary16
displacements, the axis stencil on the 2048^2 and 160^3 meshes, the one-ring
stencil built on the GPU from those meshes' cells, and the RK4 flow map of
the 2048^2 mesh.

Every timed step reads inputs already resident in HBM.  Each workload is held
in several independent copies (mesh records, coordinates, flow map, output)
and consecutive steps rotate through them, so a step never finds its inputs
in the 256 MB Infinity Cache left there by the previous step.  The default
timing is a burst of --steps launches; the rows the metric names (2D and 3D
forward, forward+adjoint, batched) are also timed sustained (200 launches
after 50 warm-up ones), with the GPU's shader clock sampled from sysfs
during that run.

Algorithmic bytes per launch (each array touched once, 32-bit CSR):
  forward  B = 4 (N + 1) + 4 nnz + 2 D s N + s N
  adjoint  B = 4 (N + 1) + 4 nnz + 3 D s N + s N     (x, flow, grad; g)
with s the storage bytes (4, or 8 in float64).  "format_bytes" is what this
library's own layout (compressed tile records with 10-bit local indices)
holds for the same launch; "traffic" is the HBM bytes the hardware counters
measured for the launch (committed rocprofv3 summary).  The RK4 flow map is
bound by float64 arithmetic: its roofline is its float64 FLOPs per launch
(hardware counters, committed summary) over the launch time, against the
float64 vector peak.

Profiling runs (rocprofv3) must find their workloads in --cache, filled by a
plain run first (--fill-cache): generating a workload launches tens of
thousands of small RK4 kernels, which the profiler must not see.  With
--require-cache a missing workload is an error before any GPU work.
--summarize-trace / --summarize-counters turn rocprofv3's CSV output into
the text summaries under profiles/ (PROFILE_RECIPE lists the commands).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import math
import os
import statistics
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0   # MI355X HBM3E, published
FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X float64 vector, published (256 CUs x 128 FLOP/clk x 2.4 GHz)
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4   # wave64 VALU instructions/s: 4 SIMDs per CU, 4 cycles each

# variant groups of --only, and the cached workloads each needs
GROUPS = ("f16", "fp64", "fwd3d", "fwdbwd", "batched", "axis", "ell", "neighbours", "meshbuild", "advect")
GROUP_WORKLOADS = {"headline": ["scale_2d"], "f16": ["scale_2d"], "fp64": ["scale_2d"], "fwd3d": ["abc_3d"],
                   "fwdbwd": ["diff_3d"], "batched": ["batched_2d"], "axis": ["scale_2d", "abc_3d"],
                   "ell": ["scale_2d", "abc_3d"],
                   "neighbours": ["scale_2d", "abc_3d"], "meshbuild": ["scale_2d", "abc_3d"],
                   "advect": ["scale_2d", "abc_3d"]}

# The commands that made the summaries under profiles/ (run from the
# repository root; the first fills the workload cache without a profiler).
PROFILE_RECIPE = [
    "python -u bench.py --fill-cache --cache /tmp/ftle_wc",
    # kernel durations: the ring-1 rows, then the axis rows (same kernel names)
    "timeout -k 10 600 rocprofv3 --kernel-trace --stats -d gpurun_out/kt_main -o kt --output-format csv -- "
    "python -u bench.py --require-cache --cache /tmp/ftle_wc --steps 30 --no-cpu-baseline --no-sustained "
    "--batched-shape 256,0,0 --only f16,fp64,fwd3d,fwdbwd,batched,ell",
    "timeout -k 10 600 rocprofv3 --kernel-trace --stats -d gpurun_out/kt_axis -o kt --output-format csv -- "
    "python -u bench.py --require-cache --cache /tmp/ftle_wc --steps 30 --no-cpu-baseline --no-sustained "
    "--no-headline --only axis",
    # the build kernels: the one-ring stencil and the whole mesh build on the device
    "timeout -k 10 600 rocprofv3 --kernel-trace --stats -d gpurun_out/kt_build -o kt --output-format csv -- "
    "python -u bench.py --require-cache --cache /tmp/ftle_wc --steps 5 --warmup 1 --no-cpu-baseline --no-sustained "
    "--no-headline --only neighbours,meshbuild",
    # HBM traffic: one counter per run (FETCH_SIZE, then WRITE_SIZE), each run
    # starting with a 256 MiB copy whose counts calibrate the counters
    "timeout -s KILL 300 rocprofv3 --pmc {counter} -d gpurun_out/pmc_{counter}_main -o pmc --output-format csv -- "
    "python -u bench.py --require-cache --cache /tmp/ftle_wc --steps 3 --warmup 1 --copies 1 --no-cpu-baseline "
    "--no-sustained --batched-shape 256,0,0 --copy-probe-mib 256 --only f16,fp64,fwd3d,fwdbwd,batched,ell",
    "timeout -s KILL 300 rocprofv3 --pmc {counter} -d gpurun_out/pmc_{counter}_axis -o pmc --output-format csv -- "
    "python -u bench.py --require-cache --cache /tmp/ftle_wc --steps 3 --warmup 1 --copies 1 --no-cpu-baseline "
    "--no-sustained --no-headline --copy-probe-mib 256 --only axis",
    # the one-ring stencil's kernels (2048^2 and 160^3; the scan and copy kernels serve both)
    "timeout -s KILL 300 rocprofv3 --pmc {counter} -d gpurun_out/pmc_{counter}_build -o pmc --output-format csv -- "
    "python -u bench.py --require-cache --cache /tmp/ftle_wc --steps 2 --warmup 1 --copies 1 --no-cpu-baseline "
    "--no-sustained --no-headline --copy-probe-mib 256 --only neighbours",
]

KERNEL_TRACE = os.path.join(ROOT, "profiles", "ftle_kernel_trace_stats.txt")
COUNTERS = os.path.join(ROOT, "profiles", "ftle_counters_fetch_write.txt")
CSRC = os.path.join(ROOT, "paper_2408_02758_amd", "csrc")
ADVECT_PROFILE = os.path.join(ROOT, "profiles", "ftle_advect_rk4.txt")
# the RK4 kernels: profile key -> (kernel name, source file, particles, steps per particle)
ADVECT_KERNELS = {"dg": ("advect_kernel<0, float>", "ftle_advect.hip", 2048 * 2048, 1500),
                  "abc": ("advect_kernel<1, float>", "ftle_advect.hip", 160 ** 3, 500),
                  "grid_dg": ("advect_grid_kernel<2, true, float, float>", "ftle_advect_grid.hip", 2048 * 2048, 1500)}
ADVECT_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_VALU_FLOPS_FP64", "SQ_INSTS_VALU_FLOPS_FP64_TRANS",
                   "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_TRANS_F64")
# the commands that made profiles/ftle_advect_rk4.txt (from the repository root)
ADVECT_RECIPE = [
    "python -u bench.py --fill-cache --cache /tmp/ftle_wc --only advect",
    "timeout -k 10 300 rocprofv3 --kernel-trace --stats -d gpurun_out/kt_advect -o kt --output-format csv -- "
    "python -u bench.py --require-cache --cache /tmp/ftle_wc --no-cpu-baseline --no-sustained --no-headline "
    "--only advect",
    "timeout -s KILL 300 rocprofv3 --pmc " + " ".join(ADVECT_COUNTERS) + " -d gpurun_out/pmc_advect -o pmc "
    "--output-format csv -- python -u bench.py --require-cache --cache /tmp/ftle_wc --no-cpu-baseline "
    "--no-sustained --no-headline --only advect",
    "python bench.py --summarize-advect gpurun_out/kt_advect gpurun_out/pmc_advect",
]


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


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
class MissingWorkload(RuntimeError):
    pass


class Workloads:
    """Named workloads, generated on first use or loaded from cache_dir (npz).

    require: a workload missing from cache_dir raises MissingWorkload instead
    of being generated (profiling runs).
    """

    def __init__(self, cache_dir, dev, require=False):
        self.cache_dir, self.dev, self.require = cache_dir, dev, require
        self._memo = {}

    def path(self, name):
        return os.path.join(self.cache_dir, name + ".npz") if self.cache_dir else None

    def check(self, names):
        """Fail before any GPU work when require is set and a workload is missing."""
        if not self.require:
            return
        if not self.cache_dir:
            raise MissingWorkload("--require-cache needs --cache DIR")
        missing = [n for n in names if not os.path.exists(self.path(n))]
        if missing:
            raise MissingWorkload(f"workloads {missing} are not in {self.cache_dir}: fill the cache first with "
                                  f"`python bench.py --fill-cache --cache {self.cache_dir}` (without a profiler)")

    def get(self, name):
        if name not in self._memo:
            self._memo[name] = self._load(name)
        return self._memo[name]

    def _make(self, name):
        from workloads import configs
        return {"scale_2d": configs.scale_2d, "abc_3d": configs.abc_3d, "diff_3d": configs.diff_3d,
                "batched_2d": configs.batched_2d}[name](self.dev)

    def _load(self, name):
        import numpy as np
        import torch

        from workloads import configs
        path = self.path(name)
        if path and os.path.exists(path):
            z = np.load(path)
            ws = []
            for k in range(int(z["count"])):
                extra = {"weights": z[f"w{k}"]} if f"w{k}" in z else {}
                if f"t0{k}" in z:
                    extra["t0"] = float(z[f"t0{k}"])
                ws.append(configs.Workload(str(z[f"name{k}"]), int(z[f"dim{k}"]), z[f"x{k}"], z[f"c{k}"],
                                           torch.as_tensor(z[f"f{k}"], device=self.dev), float(z[f"T{k}"]),
                                           str(z[f"dt{k}"]), extra))
            return ws if bool(z["is_list"]) else ws[0]
        if self.require:
            raise MissingWorkload(f"workload {name} is not in {self.cache_dir}")
        w = self._make(name)
        if path:
            ws = w if isinstance(w, list) else [w]
            arrays = {"count": len(ws), "is_list": isinstance(w, list)}
            for k, x in enumerate(ws):
                arrays.update({f"name{k}": x.name, f"dim{k}": x.dim, f"x{k}": x.coords, f"c{k}": x.cells,
                               f"f{k}": x.flow_numpy(), f"T{k}": x.T, f"dt{k}": x.dtype,
                               f"t0{k}": float(x.extra.get("t0", 0.0))})
                if "weights" in x.extra:
                    arrays[f"w{k}"] = x.extra["weights"]
            os.makedirs(self.cache_dir, exist_ok=True)
            np.savez(path, **arrays)
        return w


def needed_workloads(headline, groups):
    names = list(GROUP_WORKLOADS["headline"]) if headline else []
    for g in groups:
        for n in GROUP_WORKLOADS[g]:
            if n not in names:
                names.append(n)
    return names


# ---------------------------------------------------------------------------
# timing
# ---------------------------------------------------------------------------
def time_steps(fns, steps, warmup, torch):
    """Run warmup untimed steps, then exactly `steps` timed ones; ms per step
    from HIP events recorded on the stream the steps are launched on."""
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


class ClockSampler:
    """Samples the GPU's shader clock while active: the current level of the
    device's pp_dpm_sclk sysfs file (the line marked '*'), with the memory and
    fabric clocks of its pp_dpm_mclk / pp_dpm_fclk files, the board power from
    its hwmon power1_input and the hwmon temperatures, every ~5 ms (file reads,
    no process).  Reports min / median / max, or why nothing was recorded."""

    def __init__(self, torch):
        self.sclk = self.power = self.reason = None
        self.clocks, self.temps = {}, {}
        cards = sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk"))
        try:
            p = torch.cuda.get_device_properties(0)
            bdf = f"{p.pci_domain_id:04x}:{p.pci_bus_id:02x}:{p.pci_device_id:02x}.0"
        except Exception:  # noqa: BLE001 - the clock is informational
            bdf = None
        match = [c for c in cards if bdf and os.path.realpath(os.path.dirname(c)).endswith(bdf)]
        if match or len(cards) == 1:
            self.sclk = (match or cards)[0]
            dev_dir = os.path.dirname(self.sclk)
            pw = sorted(glob.glob(os.path.join(dev_dir, "hwmon", "hwmon*", "power1_input")))
            self.power = pw[0] if pw else None
            self.clocks = {k: os.path.join(dev_dir, f"pp_dpm_{k}") for k in ("mclk", "fclk")
                           if os.path.exists(os.path.join(dev_dir, f"pp_dpm_{k}"))}
            self.temps = {}
            for t in sorted(glob.glob(os.path.join(dev_dir, "hwmon", "hwmon*", "temp*_input"))):
                lab = t[:-len("_input")] + "_label"
                try:
                    with open(lab) as f:
                        name = f.read().strip()
                except OSError:
                    name = os.path.basename(t)[:-len("_input")]
                self.temps[name] = t
        else:
            self.reason = f"{len(cards)} pp_dpm_sclk files, none for PCI device {bdf}"
        self.samples, self.watts = [], []
        self.other = {}
        self._stop = threading.Event()
        self._thread = None

    @staticmethod
    def _read_sclk(path):
        with open(path) as f:
            for ln in f:
                if ln.rstrip().endswith("*"):
                    return float(ln.split(":", 1)[1].strip().rstrip("*").strip().lower().rstrip("mhz"))
        return None

    def _sample(self):
        v = self._read_sclk(self.sclk)
        if v is not None:
            self.samples.append(v)
        if self.power:
            with open(self.power) as f:
                self.watts.append(int(f.read().strip()) / 1e6)
        for k, path in self.clocks.items():
            v = self._read_sclk(path)
            if v is not None:
                self.other.setdefault(f"{k}_mhz", []).append(v)
        for k, path in self.temps.items():
            with open(path) as f:
                self.other.setdefault(f"temp_{k}_c", []).append(int(f.read().strip()) / 1000.0)

    def __enter__(self):
        self.samples, self.watts, self.other = [], [], {}
        if self.sclk:
            try:
                self._sample()
            except (OSError, ValueError) as e:
                self.reason, self.sclk = f"{self.sclk}: {e}", None
        if self.sclk:
            self._stop.clear()

            def run():
                while not self._stop.is_set():
                    try:
                        self._sample()
                    except (OSError, ValueError):
                        pass
                    self._stop.wait(0.005)
            self._thread = threading.Thread(target=run, daemon=True)
            self._thread.start()
        return self

    def __exit__(self, *exc):
        if self._thread:
            self._stop.set()
            self._thread.join()
            self._thread = None

    def summary(self):
        if not self.samples:
            return {"recorded": False, "reason": self.reason or "no samples"}
        s = sorted(self.samples)
        out = {"recorded": True, "source": self.sclk, "samples": len(s), "min_mhz": s[0],
               "median_mhz": statistics.median(s), "max_mhz": s[-1]}
        if self.watts:
            out["median_power_w"] = round(statistics.median(self.watts), 1)
        for k, v in sorted(self.other.items()):
            out[f"median_{k}"] = round(statistics.median(v), 1)
        return out


def sustained(fns, torch, alg_bytes, clock, steps=1000, warmup=100):
    """ms per launch over `steps` launches after `warmup` (a few tens of ms of
    back-to-back work, against the fraction of a millisecond a default burst
    takes), with the clock samples."""
    with clock:
        ms = time_steps(fns, steps, warmup, torch)
    gbps = alg_bytes / (ms * 1e-3) / 1e9
    return {"steps": steps, "warmup": warmup, "ms_per_step": round(ms, 5), "achieved": round(gbps, 1),
            "frac": round(gbps / HBM_PEAK_GBPS, 4), "gpu_clock": clock.summary()}


# ---------------------------------------------------------------------------
# committed profile summaries
# ---------------------------------------------------------------------------
def kernel_sources_sha256():
    """SHA-256 over every kernel source (the .hip files and the headers they include)."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.h"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _summary_meta_and_rows(path):
    meta, rows = {}, []
    if not os.path.exists(path):
        return meta, rows
    with open(path) as f:
        for ln in f:
            ln = ln.strip()
            if not ln or ln.startswith("#"):
                continue
            if ln.startswith("run:"):
                rows.append(dict(part.strip().split(": ", 1) for part in ln.split(" | ")))
            elif "=" in ln:
                k, v = ln.split("=", 1)
                meta[k.strip()] = v.strip()
    return meta, rows


def measured_traffic(path=COUNTERS):
    """HBM bytes per dispatch by (run, kernel), from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by the copy-probe factors), or {} when the
    summary was taken from other kernel sources."""
    meta, rows = _summary_meta_and_rows(path)
    if meta.get("kernel_sources_sha256") != kernel_sources_sha256():
        return {}
    out = {}
    for r in rows:
        ff, wf = float(r["fetch_factor"]), float(r["write_factor"])
        out[(r["run"], r["kernel"])] = round((float(r["fetch_kib"]) * ff + float(r["write_kib"]) * wf) * 1024)
    out["batched_shape"] = meta.get("batched_shape")
    return out


def traced_durations(path=KERNEL_TRACE):
    """Average duration (us) by (run, kernel) from the committed kernel-trace summary,
    or {} when it was taken from other kernel sources."""
    meta, rows = _summary_meta_and_rows(path)
    if meta.get("kernel_sources_sha256") != kernel_sources_sha256():
        return {}
    out = {(r["run"], r["kernel"]): float(r["avg_us"]) for r in rows}
    out["batched_shape"] = meta.get("batched_shape")
    return out


def advect_counts(key="dg"):
    """Float64 FLOPs and VALU instructions per launch of a measured flow map
    ("dg": the 2048^2 double gyre; "abc": the 160^3 ABC flow; "grid_dg": the
    2048^2 double gyre sampled on a grid), from the committed rocprofv3
    summary, or {} when that summary was taken from another version of the
    kernel's source."""
    meta = _profile_meta(ADVECT_PROFILE)
    src = ADVECT_KERNELS[key][1]
    with open(os.path.join(CSRC, src), "rb") as f:
        if meta.get(f"sha256 {src}") != hashlib.sha256(f.read()).hexdigest():
            return {}
    if f"{key}_fp64_flops_per_launch" not in meta:
        return {}
    return {"flops": float(meta[f"{key}_fp64_flops_per_launch"]), "valu": float(meta[f"{key}_valu_insts_per_launch"])}


def _profile_meta(path):
    meta = {}
    if os.path.exists(path):
        with open(path) as f:
            for ln in f:
                ln = ln.strip()
                if ln and not ln.startswith("#") and "=" in ln:
                    k, v = ln.split("=", 1)
                    meta[k.strip()] = v.strip()
    return meta


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


def roofline(alg_bytes, ms):
    gbps = alg_bytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(gbps / HBM_PEAK_GBPS, 4), "traffic": None}


def hbm_roofline(alg_bytes, ms, run, kernels, traffic, traced, extra=None):
    """The HBM roofline of one launch (or of a launch pair, the kernels listed),
    with the counter-measured traffic and its fraction of the peak, and the
    committed kernel trace's average duration beside the live one."""
    r = roofline(alg_bytes, ms)
    r["alg_bytes_per_launch"] = alg_bytes
    try:
        r["traffic"] = sum(traffic[(run, k)] for k in kernels)
        r["counter_gbps"] = round(r["traffic"] / (ms * 1e-3) / 1e9, 1)
        r["counter_frac"] = round(r["counter_gbps"] / HBM_PEAK_GBPS, 4)
    except KeyError:
        r["traffic"] = None
    try:
        us = sum(traced[(run, k)] for k in kernels)
        r["trace_avg_us"] = round(us, 2)
        r["trace_frac"] = round(alg_bytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4)
    except KeyError:
        pass
    r["kernels"] = list(kernels)
    if extra:
        r.update(extra)
    return r


# ---------------------------------------------------------------------------
# rocprofv3 CSV -> text summaries
# ---------------------------------------------------------------------------
def _csv_rows(directory, suffix):
    rows = []
    for p in sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True)):
        with open(p, newline="") as f:
            rows.extend(csv.DictReader(f))
    return rows


def _field(row, *names):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    raise KeyError(names)


def short_kernel_name(name):
    """A kernel's name without return type, namespaces and argument list:
    'void ftle::(anonymous namespace)::fwd_kernel<2, float, ...>(...)' ->
    'fwd_kernel<2, float, ...>'."""
    s = name.strip()
    if s.startswith("void "):
        s = s[5:]
    depth, cut = 0, len(s)
    for k, ch in enumerate(s):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0 and not s[max(0, k - 2):k].endswith("::"):
            cut = k
            break
    s = s[:cut]
    depth, start = 0, 0
    for k, ch in enumerate(s):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == ":" and depth == 0 and k + 1 < len(s) and s[k + 1] == ":":
            start = k + 2
    return s[start:].strip()


FTLE_KERNEL_TAGS = ("fwd", "bwd", "batched", "encode16", "ell_", "incidence_pass", "scan_tiles", "scan_partials",
                    "add_partials", "ring_rows", "copy_rows", "long_rows", "advect", "bbox_partial", "gather_pairs", "morton_keys",
                    "radix_hist", "radix_scatter", "iota_u32", "invert_perm", "check_relabel", "tile_extent",
                    "tile_record", "normal_inverse")


def summarize_trace(directory, run):
    """Per kernel of an FTLE source: calls, average, median, min and max duration
    (us), from rocprofv3 --kernel-trace CSV output under directory."""
    per = {}
    for r in _csv_rows(directory, "kernel_trace.csv"):
        name = short_kernel_name(_field(r, "Kernel_Name", "Kernel-Name"))
        t = (int(_field(r, "End_Timestamp")) - int(_field(r, "Start_Timestamp"))) / 1e3
        per.setdefault(name, []).append(t)
    lines = []
    for name, ts in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        if not any(k in name for k in FTLE_KERNEL_TAGS):
            continue
        lines.append(f"run: {run} | kernel: {name} | calls: {len(ts)} | avg_us: {statistics.mean(ts):.2f} | "
                     f"median_us: {statistics.median(ts):.2f} | min_us: {min(ts):.2f} | max_us: {max(ts):.2f}")
    return lines


def summarize_counters(fetch_dir, write_dir, run, probe_mib=256):
    """Per kernel: mean FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two
    rocprofv3 --pmc runs, with the factors that make the first copy-probe
    dispatch (torch.neg over probe_mib MiB, which reads and writes probe_mib MiB)
    read exactly its size."""
    def per_kernel(directory, counter):
        vals, order = {}, []
        for r in _csv_rows(directory, "counter_collection.csv"):
            if _field(r, "Counter_Name") != counter:
                continue
            name = short_kernel_name(_field(r, "Kernel_Name"))
            disp = int(_field(r, "Dispatch_Id"))
            if disp not in vals.setdefault(name, {}):
                vals[name][disp] = 0.0
                order.append((disp, name))
            vals[name][disp] += float(_field(r, "Counter_Value"))
        return vals, sorted(order)

    fetch, forder = per_kernel(fetch_dir, "FETCH_SIZE")
    write, worder = per_kernel(write_dir, "WRITE_SIZE")
    kib = probe_mib * 1024.0

    def factor(vals, order):
        for disp, name in order:
            if "neg" in name:
                return kib / vals[name][disp]
        raise RuntimeError("no copy-probe (neg) dispatch found: run bench.py with --copy-probe-mib")

    ff, wf = factor(fetch, forder), factor(write, worder)
    lines = []
    for name in sorted(set(fetch) & set(write)):
        if not any(k in name for k in FTLE_KERNEL_TAGS):
            continue
        fe = statistics.mean(fetch[name].values())
        wr = statistics.mean(write[name].values())
        lines.append(f"run: {run} | kernel: {name} | dispatches: {len(fetch[name])} | fetch_kib: {fe:.1f} | "
                     f"write_kib: {wr:.1f} | fetch_factor: {ff:.4f} | write_factor: {wf:.4f} | "
                     f"hbm_mb: {(fe * ff + wr * wf) * 1024 / 1e6:.1f}")
    return lines


def summarize_advect(trace_dir, pmc_dir):
    """The RK4 flow-map profile: per kernel of ADVECT_KERNELS its kernel-trace
    durations and the median of each SQ counter over its dispatches, with the
    float64 FLOPs (64 per wave-level count of SQ_INSTS_VALU_FLOPS_FP64) and VALU
    instructions per launch that the ALU rooflines use."""
    durs = {}
    for r in _csv_rows(trace_dir, "kernel_trace.csv"):
        name = short_kernel_name(_field(r, "Kernel_Name", "Kernel-Name"))
        durs.setdefault(name, []).append((int(_field(r, "End_Timestamp")) - int(_field(r, "Start_Timestamp"))) / 1e6)
    counts = {}
    for r in _csv_rows(pmc_dir, "counter_collection.csv"):
        name = short_kernel_name(_field(r, "Kernel_Name"))
        per = counts.setdefault(name, {}).setdefault(_field(r, "Counter_Name"), {})
        disp = int(_field(r, "Dispatch_Id"))
        per[disp] = per.get(disp, 0.0) + float(_field(r, "Counter_Value"))
    lines = ["# rocprofv3 profile of the RK4 flow-map kernels on one MI355X (gfx950): the 2048^2 double gyre "
             "(dg: 4194304 particles, 1500 steps), the 160^3 ABC flow (abc: 4096000 particles, 500 steps) and the "
             "2048^2 double gyre sampled on a 513 x 257 grid at 61 slices (grid_dg: float32 field, 1500 steps); "
             "float64 arithmetic, float32 in and out",
             "# commands, from the repository root:"] + [f"#   {c}" for c in ADVECT_RECIPE]
    for src in sorted({v[1] for v in ADVECT_KERNELS.values()}):
        with open(os.path.join(CSRC, src), "rb") as f:
            lines.append(f"sha256 {src} = {hashlib.sha256(f.read()).hexdigest()}")
    lines.append("# kernel                                    calls    avg_ms    min_ms    max_ms")
    for key, (kname, _, _, _) in ADVECT_KERNELS.items():
        ts = durs.get(kname, [])
        if ts:
            lines.append(f"#   {kname:<40} {len(ts):5d} {statistics.mean(ts):9.3f} {min(ts):9.3f} {max(ts):9.3f}")
    for key, (kname, _, n, steps) in ADVECT_KERNELS.items():
        c = counts.get(kname)
        if not c or any(k not in c for k in ADVECT_COUNTERS):
            continue
        med = {k: statistics.median(c[k].values()) for k in ADVECT_COUNTERS}
        lines.append(f"# {kname}: {len(c['SQ_WAVES'])} dispatches; median counters per dispatch (per wave "
                     "instruction, summed over waves; SQ_INSTS_VALU_FLOPS_FP64 = ADD + MUL + 2 FMA + TRANS, so "
                     "FLOPs = 64 x it):")
        lines += [f"#   {k:<32} {med[k]:.6g}" for k in ADVECT_COUNTERS]
        flops, valu = 64.0 * med["SQ_INSTS_VALU_FLOPS_FP64"], med["SQ_INSTS_VALU"]
        lines += [f"{key}_fp64_flops_per_launch = {flops:.6g}",
                  f"{key}_fp64_flops_per_particle_step = {flops / (n * steps):.2f}",
                  f"{key}_valu_insts_per_launch = {valu:.6g}",
                  f"{key}_valu_per_particle_step = {64.0 * valu / (n * steps):.2f}"]
    return lines


PROFILE_BATCHED_SHAPE = "256,0,0"


def profile_header(kind):
    """Header of a committed profile summary: what it holds, the commands that
    made it (PROFILE_RECIPE, then the summarizer), the hash of the kernel
    sources it was taken from and the batched launch shape pinned in it."""
    if kind == "trace":
        title = "rocprofv3 --kernel-trace: per-kernel durations (us) of the FTLE kernels, one MI355X (gfx950)"
        cmds = PROFILE_RECIPE[:4] + ["python bench.py --profile-header trace",
                                    "python bench.py --summarize-trace gpurun_out/kt_main main",
                                    "python bench.py --summarize-trace gpurun_out/kt_axis axis",
                                    "python bench.py --summarize-trace gpurun_out/kt_build build"]
    else:
        title = ("rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE: HBM KiB per dispatch of the FTLE kernels, one MI355X "
                 "(gfx950); each counter scaled by the factor that makes a 256 MiB copy (torch.neg) read its size")
        cmds = [PROFILE_RECIPE[0]] + [c.replace("{counter}", k) for c in PROFILE_RECIPE[4:]
                                      for k in ("FETCH_SIZE", "WRITE_SIZE")]
        cmds += ["python bench.py --profile-header counters",
                 "python bench.py --summarize-counters gpurun_out/pmc_FETCH_SIZE_main gpurun_out/pmc_WRITE_SIZE_main main",
                 "python bench.py --summarize-counters gpurun_out/pmc_FETCH_SIZE_axis gpurun_out/pmc_WRITE_SIZE_axis axis",
                 "python bench.py --summarize-counters gpurun_out/pmc_FETCH_SIZE_build gpurun_out/pmc_WRITE_SIZE_build build"]
    lines = [f"# {title}", "# commands, from the repository root:"] + [f"#   {c}" for c in cmds]
    lines += ["# run 'main': the ring-1, float64, binary16, forward+adjoint, batched and axis-list rows; run 'axis': "
              "the axis-stencil rows (same kernel names as the ring-1 ones)"
              + ("; run 'build': the one-ring stencil and the mesh build on the device, 2048^2 and 160^3 (the "
                 "mesh build's calls include the warm-up builds and the ones beside the host build)"
                 if kind == "trace" else "; run 'build': the one-ring stencil's kernels, 2048^2 and 160^3 (the "
                 "scan and copy kernels' figures are means over both)"),
              f"kernel_sources_sha256 = {kernel_sources_sha256()}", f"batched_shape = {PROFILE_BATCHED_SHAPE}"]
    return "\n".join(lines)


# ---------------------------------------------------------------------------
# the FP64 oracle on the host: baseline timings and the error of the GPU fields
# ---------------------------------------------------------------------------
def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


class Stencils:
    """The oracle's one-ring stencils, built once per workload."""

    def __init__(self):
        self._memo = {}

    def get(self, w):
        import oracle
        key = (w.name, w.n)
        if key not in self._memo:
            self._memo[key] = oracle.ring1(w.dim, w.n, w.cells)
        return self._memo[key]

    def axis(self, w):
        """The oracle's fixed-width axis list (a Stencil of 2*dim slots per point)."""
        import numpy as np

        import oracle
        key = ("axis", w.name, w.n)
        if key not in self._memo:
            self._memo[key] = oracle.axis(w.dim, w.coords.astype(np.float64), self.get(w))
        return self._memo[key]


def _median_of_3(fn):
    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts), ts


def cpu_table(loads, stencils, threads_all, configs_wanted):
    """The FP64 oracle as it stands (per-point loop only, stencils built
    beforehand), at 1 thread and at threads_all, median of 3 runs, on bounded
    samples of each configuration's workload."""
    import numpy as np

    import oracle
    rows = []
    cases = []
    if "2d" in configs_wanted:
        w = loads.get("scale_2d")
        st = stencils.get(w)
        x, phi = w.coords.astype(np.float64), w.flow_numpy().astype(np.float64)
        cases.append(("fwd_2d_2048", f"all {w.n} points of the 2048^2 workload", w.n,
                      lambda: oracle.ftle(2, x, phi, st, w.T)))
    if "3d" in configs_wanted:
        w3 = loads.get("abc_3d")
        st3 = stencils.get(w3)
        x3, p3 = w3.coords.astype(np.float64), w3.flow_numpy().astype(np.float64)
        sel = np.sort(np.random.default_rng(5).choice(w3.n, 1 << 20, replace=False))
        cases.append(("fwd_3d_160", f"{sel.size} of the {w3.n} points of the 160^3 workload (seeded sample)",
                      sel.size, lambda: oracle.ftle(3, x3, p3, st3, w3.T, sel=sel)))
    if "fwdbwd" in configs_wanted:
        wd = loads.get("diff_3d")
        std = stencils.get(wd)
        xd, pd = wd.coords.astype(np.float64), wd.flow_numpy().astype(np.float64)
        gd = wd.extra["weights"].astype(np.float32).astype(np.float64)
        cases.append(("fwd_bwd_3d_96", f"all {wd.n} points of the 96^3 workload, forward then adjoint", wd.n,
                      lambda: (oracle.ftle(3, xd, pd, std, wd.T), oracle.ftle_grad(3, xd, pd, std, wd.T, gd))))
    if "batched" in configs_wanted:
        wb = loads.get("batched_2d")
        data = [(w, stencils.get(w), w.coords.astype(np.float64), w.flow_numpy().astype(np.float64)) for w in wb]
        npts = sum(w.n for w in wb)
        cases.append(("batched_2d_48", f"all {npts} points of the 48 meshes, one after another", npts,
                      lambda: [oracle.ftle(2, x, p, s, w.T) for w, s, x, p in data]))
    for name, sample, npts, fn in cases:
        for th in sorted({1, threads_all}):
            oracle.set_threads(th)
            med, ts = _median_of_3(fn)
            rows.append({"config": name, "threads": th, "points": npts, "median_s": round(med, 4),
                         "runs_s": [round(t, 4) for t in ts], "points_per_s": round(npts / med, 1),
                         "sample": sample})
            log(f"oracle {name} at {th} threads: {npts / med / 1e6:.2f} M points/s")
    oracle.set_threads(threads_all)
    return rows


def raw_tiles(m):
    """A mesh's tile metadata and record bytes, as the library returns them."""
    import ctypes

    from paper_2408_02758_amd import _lib
    L = _lib.load()
    nt, rb = ctypes.c_int64(), ctypes.c_int64()
    _lib.check(L.ftle_mesh_get_tiles(m.handle, 0, ctypes.byref(nt), ctypes.byref(rb), None, None))
    meta = ctypes.create_string_buffer(max(1, nt.value * 16))
    rec = ctypes.create_string_buffer(max(1, rb.value))
    _lib.check(L.ftle_mesh_get_tiles(m.handle, 0, None, None, meta, rec))
    return meta.raw[:nt.value * 16], rec.raw[:rb.value]


def host_threads():
    """Threads the host mesh builder runs (FTLE_HOST_THREADS, else the hardware threads, at most 32)."""
    env = os.environ.get("FTLE_HOST_THREADS")
    return max(1, int(env)) if env else max(1, min(os.cpu_count() or 1, 32))


def stencil_vs_oracle(stencils, w, row_ptr, col):
    """The GPU-built one-ring stencil against the oracle's, entry for entry."""
    import numpy as np
    ref = stencils.get(w)
    return {"row_ptr_equal": bool(np.array_equal(row_ptr, ref.row_ptr)),
            "col_equal": bool(np.array_equal(col, ref.col)), "nnz": int(ref.col.size)}


def error_vs_oracle(stencils, w, got, sel=None, stencil="ring1"):
    """Error of a GPU FTLE field against the FP64 oracle on the same (float32-
    rounded) inputs: max |error| over finite points, and the relative error
    where the top eigenvalue is separated (gap >= 1e-3) and |ln lambda| >= 0.05,
    the mask the parity tests use."""
    import numpy as np

    import oracle
    st = stencils.axis(w) if stencil == "axis" else stencils.get(w)
    ref, gap, _ = oracle.ftle(w.dim, w.coords.astype(np.float64), w.flow_numpy().astype(np.float64), st, w.T,
                              sel=sel, diagnostics=True)
    g = np.asarray(got, dtype=np.float64)
    if sel is not None:
        g = g[sel]
    fin = np.isfinite(ref)
    mask = fin & (gap >= 1e-3) & (2 * abs(w.T) * np.abs(ref) >= 0.05)
    rel = np.abs(g[mask] - ref[mask]) / np.abs(ref[mask])
    return {"points": int(ref.size), "max_abs_err": float(np.abs(g[fin] - ref[fin]).max(initial=0)),
            "masked_max_rel_err": float(rel.max(initial=0)),
            "masked_p99_rel_err": float(np.percentile(rel, 99)) if rel.size else 0.0,
            "mask_fraction": round(float(mask.mean()), 4),
            "nan_count": int(np.isnan(g).sum()),
            "nan_masks_equal": bool(np.array_equal(np.isnan(g), np.isnan(ref)))}


def grad_error_vs_oracle(stencils, w, g_in, grad):
    """Max |error| of the GPU adjoint over the max |gradient| of the FP64 oracle,
    leaving out points next to a nearly repeated top eigenvalue (gap < 1e-6),
    whose eigenvector is ill-defined (as the parity tests do)."""
    import numpy as np

    import oracle
    st = stencils.get(w)
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


def oracle_advect_grid(vel, spacing, t_step, x0, t0, T, dt):
    """The FP64 oracle's RK4 flow map of the given particles in a sampled field
    whose nodes start at the origin and whose slices start at time 0."""
    import oracle
    return oracle.advect_rk4_grid(vel, [0.0] * len(spacing), list(spacing), 0.0, t_step, x0, t0, T, dt)


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


def parse_shape(text):
    """--batched-shape: 'auto' or 'block,tiles_per_pop,per_cu_cap'."""
    if text == "auto":
        return None
    b, k, c = (int(v) for v in text.split(","))
    return b, k, c


def shape_text(cfg):
    """The --batched-shape text of a flat launch shape, or 'block,k,gridG' of a
    persistent one (its cap is not reported; the grid identifies it)."""
    if cfg["tiles_per_pop"] == 0:
        return f"{cfg['block']},0,0"
    return f"{cfg['block']},{cfg['tiles_per_pop']},grid{cfg['grid']}"


# ---------------------------------------------------------------------------
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--copies", type=int, default=3, help="input copies rotated between steps")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-headline", action="store_true", help="skip the 2D headline (profiling runs of variants)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sustained", action="store_true", help="skip the 200-launch sustained timings")
    ap.add_argument("--only", default="", help="comma list of: " + ",".join(GROUPS))
    ap.add_argument("--cache", default="", help="directory to keep generated workloads in (npz)")
    ap.add_argument("--fill-cache", action="store_true", help="generate the workloads into --cache and exit")
    ap.add_argument("--require-cache", action="store_true",
                    help="fail before any GPU work if a workload is missing from --cache (profiling runs)")
    ap.add_argument("--batched-shape", default="auto",
                    help="'auto' (autotuned) or 'block,tiles_per_pop,per_cu_cap' pinned (profiling runs)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one plain elementwise copy of this many MiB (counter calibration)")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("DIR", "RUN"),
                    help="print the kernel-trace summary lines of rocprofv3 CSV output in DIR and exit")
    ap.add_argument("--summarize-counters", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "RUN"),
                    help="print the FETCH_SIZE / WRITE_SIZE summary lines of two rocprofv3 --pmc runs and exit")
    ap.add_argument("--summarize-advect", nargs=2, metavar=("TRACE_DIR", "PMC_DIR"),
                    help="print the RK4 flow-map profile from a kernel-trace and an SQ-counter run and exit")
    ap.add_argument("--profile-header", choices=("trace", "counters"),
                    help="print the header of a profile summary (commands, source hash) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the FTLE hot path is "
              "built and measured on a single MI355X (meshes would be split into Morton ranges, one per GPU, "
              "with a one-ring halo exchange of the flow map).", flush=True)
        sys.exit(2)
    if args.summarize_trace:
        print("\n".join(summarize_trace(*args.summarize_trace)))
        return
    if args.summarize_counters:
        print("\n".join(summarize_counters(*args.summarize_counters)))
        return
    if args.profile_header:
        print(profile_header(args.profile_header))
        return
    if args.summarize_advect:
        print("\n".join(summarize_advect(*args.summarize_advect)))
        return

    only = [g for g in args.only.split(",") if g]
    bad = [g for g in only if g not in GROUPS]
    if bad:
        ap.error(f"unknown --only groups {bad}")
    groups = [] if args.no_variants else (only or list(GROUPS))
    headline = not args.no_headline
    shape = parse_shape(args.batched_shape)
    if args.fill_cache and not args.cache:
        ap.error("--fill-cache needs --cache DIR")

    dev = "cuda:0"
    loads = Workloads(args.cache, dev, require=args.require_cache)
    try:
        loads.check(needed_workloads(headline, groups))
    except MissingWorkload as e:
        print(f"bench.py: {e}", file=sys.stderr, flush=True)
        sys.exit(3)

    import numpy as np
    import torch

    if args.fill_cache:
        names = needed_workloads(True, groups)
        for name in names:
            log(f"filling the cache: {name}")
            loads.get(name)
        print(json.dumps({"filled": names, "cache": args.cache}), flush=True)
        return

    import paper_2408_02758_amd as F
    from workloads import flows

    torch.cuda.set_device(0)
    want = lambda k: k in groups  # noqa: E731
    R = max(1, args.copies)
    result = {}
    variants = {}
    keep = {}   # GPU fields checked against the oracle at the end
    traffic = measured_traffic()
    traced = traced_durations()
    clock = ClockSampler(torch)
    if shape:
        F.pin_batched_config(*shape)

    if args.copy_probe_mib:
        src = torch.ones(args.copy_probe_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)       # reads and writes exactly copy_probe_mib MiB each
        torch.cuda.synchronize()
        del src, dst

    # ---- headline: 2D forward at 2048^2 ------------------------------------
    w2 = loads.get("scale_2d") if (headline or any(g in groups for g in ("f16", "fp64", "axis", "ell", "neighbours", "meshbuild",
                                                                          "advect"))) else None
    copy_gbps = None
    if headline:
        log("building the 2048^2 meshes")
        meshes2 = [F.Mesh(w2.coords, w2.cells, "f32") for _ in range(R)]
        nnz2 = meshes2[0].info()["nnz"]
        flows2 = [w2.flow.to(dev).clone().contiguous() for _ in range(R)]
        outs2 = [torch.empty(w2.n, dtype=torch.float32, device=dev) for _ in range(R)]
        fns = [lambda k=k: meshes2[k].forward(flows2[k], w2.T, out=outs2[k]) for k in range(R)]
        log("timing 2D forward")
        ms = time_steps(fns, args.steps, args.warmup, torch)
        B = alg_bytes_fwd(w2.n, nnz2, 2)
        pts = w2.n / (ms * 1e-3)
        kname = f"fwd_kernel<2, float, true, 0, {meshes2[0].blocks()[0]}, false>"
        rl = hbm_roofline(B, ms, "main", [kname], traffic, traced)
        rl["format_bytes_per_launch"] = format_bytes_fwd(meshes2[0], 2)
        rl["format_frac"] = round(rl["format_bytes_per_launch"] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
        if not args.no_sustained:
            log("timing 2D forward, sustained")
            rl["sustained"] = sustained(fns, torch, B, clock)
        nan = int(torch.isnan(outs2[0]).sum().item())
        keep["2d"] = outs2[0].cpu().numpy()
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
        del fns, meshes2, flows2, outs2

    # ---- variants ----------------------------------------------------------
    steps_v = max(10, args.steps // 2)
    if want("f16"):
        # the headline with the flow map stored as binary16 displacements
        # (4 bytes per point instead of 8), float32 arithmetic
        log("f16 flow storage: 2048^2 forward")
        m16 = [F.Mesh(w2.coords, w2.cells, "f32") for _ in range(R)]
        nnz = m16[0].info()["nnz"]
        fl = [w2.flow.to(dev).clone().contiguous() for _ in range(R)]
        ou = [torch.empty(w2.n, dtype=torch.float32, device=dev) for _ in range(R)]
        d16 = [m16[k].encode_flow_f16(fl[k]) for k in range(R)]
        fns = [lambda k=k: m16[k].forward_f16(d16[k], w2.T, out=ou[k]) for k in range(R)]
        t = time_steps(fns, args.steps, args.warmup, torch)
        Bh = alg_bytes_fwd_f16(w2.n, nnz, 2)
        variants["fwd_2d_2048_f16flow"] = {
            "workload": "2D forward on the 2048^2 workload with the flow map stored as binary16 displacements "
                        "phi - x (float32 arithmetic on the decoded map)",
            "points": w2.n, "nnz": nnz, "ms_per_step": round(t, 5), "points_per_s": round(w2.n / (t * 1e-3), 1),
            "roofline": hbm_roofline(Bh, t, "main", [f"fwd16_kernel<{m16[0].blocks()[0]}>"], traffic, traced)}
        log(f"f16 flow storage: {t * 1e3:.2f} us/step")
        keep["f16"] = ou[0].cpu().numpy()
        del d16, fns, m16, fl, ou
    if want("fp64"):
        # the headline's inputs widened to float64: the paper's precision
        log("float64: 2048^2 forward")
        x64 = w2.coords.astype(np.float64)
        m64 = [F.Mesh(x64, w2.cells, "f64") for _ in range(R)]
        nnz = m64[0].info()["nnz"]
        fl = [w2.flow.to(dev).double().contiguous() for _ in range(R)]
        ou = [torch.empty(w2.n, dtype=torch.float64, device=dev) for _ in range(R)]
        fns = [lambda k=k: m64[k].forward(fl[k], w2.T, out=ou[k]) for k in range(R)]
        t = time_steps(fns, steps_v, args.warmup, torch)
        B64 = alg_bytes_fwd(w2.n, nnz, 2, s=8)
        variants["fwd_2d_2048_f64"] = {
            "workload": "2D plain FTLE forward in float64 (storage and arithmetic) on the 2048^2 workload "
                        "(its float32 coordinates and flow map widened)",
            "points": w2.n, "nnz": nnz, "ms_per_step": round(t, 5), "points_per_s": round(w2.n / (t * 1e-3), 1),
            "roofline": hbm_roofline(B64, t, "main", [f"fwd_kernel<2, double, true, 0, {m64[0].blocks()[0]}, false>"],
                                     traffic, traced)}
        log(f"float64 2D forward: {t * 1e3:.2f} us/step")
        keep["fp64"] = ou[0].cpu().numpy()
        del fns, m64, fl, ou
    if want("fwd3d"):
        w3 = loads.get("abc_3d")
        log("building the 160^3 meshes")
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
        rl3 = hbm_roofline(B3, t, "main", [f"fwd_kernel<3, float, true, 0, {ms3[0].blocks()[0]}, false>"],
                           traffic, traced, {"format_bytes_per_launch": format_bytes_fwd(ms3[0], 3)})
        if not args.no_sustained:
            log("timing 3D forward, sustained")
            rl3["sustained"] = sustained(fns, torch, B3, clock)
        variants["fwd_3d_160"] = {
            "workload": "3D plain FTLE forward, 160^3 Kuhn tetrahedral grid, ABC flow, RK4 dt=0.02, T=10",
            "points": w3.n, "nnz": nnz3, "ms_per_step": round(t, 5), "points_per_s": round(w3.n / (t * 1e-3), 1),
            "roofline": rl3, "fp64_eigen_recomputes_per_call": round(hits / max(1, calls0), 1)}
        log(f"3D forward: {t * 1e3:.2f} us/step")
        keep["3d"] = (w3, ou3[0].cpu().numpy())
        del fns, ms3, fl3, ou3
    if want("fwdbwd"):
        wd = loads.get("diff_3d")
        log("building the 96^3 meshes (differentiated)")
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
        fb, bb = msd[0].blocks()
        rld = hbm_roofline(Bd, t, "main", [f"fwd_kernel<3, float, true, 1, {fb}, false>",
                                           f"bwd_kernel<3, float, {bb}, false, false>"], traffic, traced)
        if not args.no_sustained:
            log("timing forward+adjoint, sustained")
            rld["sustained"] = sustained(fns, torch, Bd, clock)
        variants["fwd_bwd_3d_96"] = {
            "workload": "3D FTLE forward + adjoint (dL/dflow, L = sum w_i FTLE_i), 96^3 Kuhn grid, ABC flow, T=10: "
                        "tape forward then the adjoint gather",
            "points": wd.n, "nnz": nnzd, "ms_per_step": round(t, 5), "points_per_s": round(wd.n / (t * 1e-3), 1),
            "roofline": rld}
        log(f"fwd+bwd: {t * 1e3:.2f} us/step")
        keep["fwdbwd"] = (wd, outd[0].cpu().numpy(), gw.cpu().numpy(), gradd[0].cpu().numpy())
        del fns, msd, fld, outd, taped, gradd
    if want("batched"):
        wb = loads.get("batched_2d")
        log("building the 48-mesh batched sets")
        Rb = 2
        sets = []
        for _ in range(Rb):
            mb = [F.Mesh(w.coords, w.cells, "f32") for w in wb]
            fb_ = [w.flow.to(dev).clone().contiguous() for w in wb]
            ob = [torch.empty(w.n, dtype=torch.float32, device=dev) for w in wb]
            sets.append((mb, fb_, ob))
        Ts = [w.T for w in wb]
        fns = [F.BatchedCall(s[0], s[1], Ts, outs=s[2]) for s in sets]
        t = time_steps(fns, steps_v, args.warmup, torch)
        npts = sum(w.n for w in wb)
        nnzb = sum(m.info()["nnz"] for m in sets[0][0])
        Bb = sum(alg_bytes_fwd(m.n, m.info()["nnz"], 2) for m in sets[0][0])
        cfg = F.batched_config(sets[0][0])
        cfg_other = F.batched_config(sets[1][0])
        form = ("a flat grid of one workgroup per tile" if cfg["tiles_per_pop"] == 0 else
                f"a persistent grid of {cfg['grid']} workgroups draining an atomic queue, "
                f"{cfg['tiles_per_pop']} tiles per pop")
        # the profiles hold this row's figures only when they were taken in the same launch form
        kb = [f"batched_kernel<2, float, {cfg['block']}, false>"]
        tr = traffic if traffic.get("batched_shape") == shape_text(cfg) else {}
        td = traced if traced.get("batched_shape") == shape_text(cfg) else {}
        rlb = hbm_roofline(Bb, t, "main", kb, tr, td)
        if not args.no_sustained:
            log("timing batched, sustained")
            rlb["sustained"] = sustained(fns, torch, Bb, clock)
        variants["batched_2d_48"] = {
            "workload": "48 jittered triangulated double-gyre meshes, sides log-uniform in [64,1024], "
                        f"own t0 and T each, one launch from a HIP graph: {form}",
            "points": npts, "nnz": nnzb, "ms_per_step": round(t, 5), "points_per_s": round(npts / (t * 1e-3), 1),
            "launch_shape": cfg, "launch_shape_pinned": shape is not None,
            "launch_shape_second_set": cfg_other, "roofline": rlb}
        log(f"batched: {t * 1e3:.2f} us/step ({form})")
        keep["batched"] = [(wb[k], sets[0][2][k].cpu().numpy()) for k in (0, 24, 47)]
        del fns, sets
    if want("axis"):
        # the paper's stencil (one nearest neighbour per side of each axis),
        # measured against the paper's fixed-width list (alg_bytes_ell)
        for dim, name in ((2, "axis_2d_2048"), (3, "axis_3d_160")):
            wa = w2 if dim == 2 else loads.get("abc_3d")
            log(f"{name}: building meshes")
            ma = [F.Mesh(wa.coords, wa.cells, "f32", stencil="axis") for _ in range(R)]
            fa = [wa.flow.to(dev).clone().contiguous() for _ in range(R)]
            oa = [torch.empty(wa.n, dtype=torch.float32, device=dev) for _ in range(R)]
            fns = [lambda k=k: ma[k].forward(fa[k], wa.T, out=oa[k]) for k in range(R)]
            t = time_steps(fns, steps_v, args.warmup, torch)
            Be = alg_bytes_ell(wa.n, dim)
            variants[name] = {
                "workload": f"{dim}D plain FTLE forward with the paper's axis stencil (2*dim nearest neighbours "
                            f"along the axes, Section 2.2), on the {'2048^2' if dim == 2 else '160^3'} workload, "
                            "through the compressed tile records",
                "points": wa.n, "nnz": ma[0].info()["nnz"], "ms_per_step": round(t, 5),
                "points_per_s": round(wa.n / (t * 1e-3), 1),
                "roofline": hbm_roofline(Be, t, "axis",
                                         [f"fwd_kernel<{dim}, float, true, 0, {ma[0].blocks()[0]}, false>"],
                                         traffic, traced,
                                         {"alg_model": "paper's fixed-width list",
                                          "format_bytes_per_launch": format_bytes_fwd(ma[0], dim)})}
            log(f"{name}: {t * 1e3:.2f} us/step")
            keep[name] = (wa, oa[0].cpu().numpy())
            del fns, ma, fa, oa
    if want("ell"):
        # the paper's fixed-width list itself (2*dim int32 per point, -1 where
        # absent, no row pointers, caller order), built on the GPU from the
        # device one-ring stencil, and the forward that streams it: direct
        # gathers (the paper's layout without reuse) and LDS-staged blocks
        for dim, name in ((2, "ell_2d_2048"), (3, "ell_3d_160")):
            we = w2 if dim == 2 else loads.get("abc_3d")
            log(f"{name}: the axis list on the GPU")
            xs, fs, ls, os_ = [], [], [], []
            for _ in range(R):
                cells_d = torch.as_tensor(we.cells, dtype=torch.int32, device=dev).contiguous()
                rp, col = F.ring1_csr(dim, we.n, cells_d)
                x_d = torch.as_tensor(we.coords, device=dev).contiguous()
                ls.append(F.axis_ell(x_d, rp, col))
                xs.append(x_d)
                fs.append(we.flow.to(dev).clone().contiguous())
                os_.append(torch.empty(we.n, dtype=torch.float32, device=dev))
                del cells_d, rp, col
            Be = alg_bytes_ell(we.n, dim)
            for staged in (False, True):
                fns = [lambda k=k: F.forward_ell(xs[k], ls[k], fs[k], we.T, staged=staged, out=os_[k])
                       for k in range(R)]
                t = time_steps(fns, steps_v, args.warmup, torch)
                key = f"{name}_{'staged' if staged else 'direct'}"
                variants[key] = {
                    "workload": f"{dim}D FTLE forward from the paper's fixed-width axis list (2*dim int32 per point, "
                                f"-1 where absent, caller order) on the {'2048^2' if dim == 2 else '160^3'} workload, "
                                + ("each workgroup's 256 points staged in LDS" if staged else "direct gathers"),
                    "points": we.n, "ms_per_step": round(t, 5), "points_per_s": round(we.n / (t * 1e-3), 1),
                    "roofline": hbm_roofline(Be, t, "main", [f"ell_kernel<{dim}, float, {str(staged).lower()}, 256>"],
                                             traffic, traced, {"alg_model": "paper's fixed-width list"})}
                log(f"{key}: {t * 1e3:.2f} us/step")
                keep[key] = (we, os_[0].cpu().numpy(), ls[0].cpu().numpy())
            del fns, xs, fs, ls, os_
    if want("neighbours"):
        # the one-ring stencil built on the GPU from the cells (incidence
        # counts and lists, each point's distinct neighbours sorted in LDS,
        # CSR), with a caller-held workspace, returning the entry count to
        # the host
        for name, wn in (("ring1_csr_2d_2048", w2), ("ring1_csr_3d_160", loads.get("abc_3d"))):
            log(f"{name}: one-ring stencil on the GPU")
            cells_d = torch.as_tensor(wn.cells, dtype=torch.int32, device=dev).contiguous()
            ws = torch.empty(F.ring1_workspace_bytes(wn.dim, wn.n, cells_d.shape[0]), dtype=torch.uint8, device=dev)
            colbuf = torch.empty(cells_d.shape[0] * wn.dim * (wn.dim + 1), dtype=torch.int32, device=dev)
            rp, col = F.ring1_csr(wn.dim, wn.n, cells_d, workspace=ws, col=colbuf)
            t = time_steps([lambda: F.ring1_csr(wn.dim, wn.n, cells_d, workspace=ws, col=colbuf)], 10, 2, torch)
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
            del cells_d, rp, col, ws, colbuf
    if want("meshbuild"):
        # the whole mesh build on the GPU (ftle_create_mesh_device: Morton
        # order, one-ring stencil, tile records, 3D normal matrices) beside
        # the host build of the same mesh with its upload (ftle_create_mesh);
        # wall time of each call, inputs already where each build takes them
        for name, wn in (("meshbuild_2d_2048", w2), ("meshbuild_3d_160", loads.get("abc_3d"))):
            log(f"{name}: mesh build on the GPU and on the host")
            xd = torch.as_tensor(wn.coords, device=dev).contiguous()
            cd = torch.as_tensor(wn.cells, dtype=torch.int32, device=dev).contiguous()
            F.Mesh.on_device(xd, cd).close()
            torch.cuda.synchronize()
            td = []
            for _ in range(5):
                t0 = time.perf_counter()
                md = F.Mesh.on_device(xd, cd)
                td.append(time.perf_counter() - t0)
                md.close()
            th = []
            for _ in range(2):
                t0 = time.perf_counter()
                mh = F.Mesh(wn.coords, wn.cells, wn.dtype)
                th.append(time.perf_counter() - t0)
                if _ == 0:
                    mh.close()
            md = F.Mesh.on_device(xd, cd)
            same = all(np.array_equal(a, b) for a, b in zip(md.csr(), mh.csr())) \
                and md.tile_stats() == mh.tile_stats() and raw_tiles(md) == raw_tiles(mh)
            t_dev, t_host = float(np.median(td)) * 1e3, min(th) * 1e3
            info, stats = md.info(), md.tile_stats()
            Bm = (4 * cd.numel() + xd.numel() * xd.element_size() + 8 * (wn.n + 1) + 4 * info["nnz"]
                  + stats["record_bytes"])
            variants[name] = {
                "workload": f"mesh of the {'2048^2 triangle' if wn.dim == 2 else '160^3 tetrahedron'} grid built "
                            "from device coordinates and cells on the GPU (wall time of the call, median of 5)",
                "points": wn.n, "cells": int(cd.shape[0]), "nnz": info["nnz"], "tiles": stats["n_tiles"],
                "ms_per_step": round(t_dev, 3), "points_per_s": round(wn.n / (t_dev * 1e-3), 1),
                "host_build_ms": round(t_host, 1), "host_build_threads": host_threads(),
                "speedup_vs_host_build": round(t_host / t_dev, 2), "equal_to_host_build": bool(same),
                "roofline": dict(roofline(Bm, t_dev), alg_bytes_per_launch=Bm,
                                 alg_model="cells and coordinates read once; stencil and tile records written once")}
            log(f"{name}: {t_dev:.2f} ms on the GPU, {t_host:.1f} ms on the host, same mesh: {same}")
            md.close()
            mh.close()
            del xd, cd
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
        w3a = loads.get("abc_3d")
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
        del x0, phi
        # the same 2048^2 particles and steps through the double gyre sampled
        # on a grid, as simulation output comes: 513 x 257 nodes over
        # [0, 2] x [0, 1], 61 slices 0.25 apart (float32, 64 MB), bilinear in
        # space and linear in time
        log("advect_grid_2d_2048: RK4 flow map in a sampled field on the GPU")
        gshape, gspacing, gtimes = (513, 257), (2.0 / 512, 1.0 / 256), np.arange(61) * 0.25
        vel = torch.as_tensor(flows.sampled_field(flows.double_gyre_velocity, (0.0, 0.0), gspacing, gshape, gtimes)
                              .astype(np.float32), device=dev)
        x0 = torch.as_tensor(w2.coords, dtype=torch.float32, device=dev).contiguous()
        phi = torch.empty_like(x0)

        def grid_map():
            F.advect_rk4_grid(vel, (0.0, 0.0), gspacing, 0.0, 0.25, x0, t0, w2.T, 0.01, out=phi)
        grid_map()
        t = time_steps([grid_map], 3, 1, torch)
        nsteps = math.ceil(abs(w2.T) / 0.01 - 1e-9)
        variants["advect_grid_2d_2048"] = {
            "workload": "RK4 flow map of the 2048^2 jittered grid in the double gyre sampled on a 513 x 257 grid "
                        "over [0, 2] x [0, 1] at 61 slices 0.25 apart (float32 field, bilinear in space, linear in "
                        "time), t0 = 0, T = 15, dt = 0.01 (float64 arithmetic, float32 output)",
            "points": w2.n, "steps_per_point": nsteps, "ms_per_step": round(t, 4),
            "points_per_s": round(w2.n / (t * 1e-3), 1),
            "particle_steps_per_s": round(w2.n * nsteps / (t * 1e-3), 1),
            "field_bytes": int(vel.numel() * vel.element_size()),
            "roofline": alu_roofline(advect_counts("grid_dg"), t)}
        log(f"advect_grid_2d_2048: {t:.2f} ms per flow map")
        keep["advect_grid"] = (w2, vel.cpu().numpy().astype(np.float64), gspacing, x0.cpu().numpy(), t0,
                               phi.cpu().numpy())
        del x0, phi, vel
    if copy_gbps:
        for v in variants.values():
            if v["roofline"]["bound"] == "hbm":
                v["roofline"]["frac_of_copy_probe"] = round(v["roofline"]["achieved"] / copy_gbps, 4)
    if variants:
        result["variants"] = variants
    if shape:
        F.pin_batched_config(0)

    if not args.no_cpu_baseline and headline:
        try:
            threads = min(16, len(os.sched_getaffinity(0)))
        except AttributeError:
            threads = min(16, os.cpu_count() or 1)
        stencils = Stencils()
        log(f"timing the FP64 oracle at 1 and {threads} host threads")
        table = cpu_table(loads, stencils, threads,
                          {"2d"} | ({"3d"} if want("fwd3d") else set()) | ({"fwdbwd"} if want("fwdbwd") else set())
                          | ({"batched"} if want("batched") else set()))
        head = next(r for r in table if r["config"] == "fwd_2d_2048" and r["threads"] == threads)
        result["cpu_baseline"] = {
            "value": head["points_per_s"], "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": f"{head['sample']}, per-point loop only (stencil built beforehand), float64, OpenMP "
                      f"{threads} threads, median of 3 runs",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "table": table}
        # the GPU fields of this run against the FP64 oracle on the same inputs
        log("checking the GPU fields against the FP64 oracle")
        err = {"2d_2048": error_vs_oracle(stencils, w2, keep["2d"])}
        rng = np.random.default_rng(0)
        if "3d" in keep:
            w3, got3 = keep["3d"]
            err["3d_160_sample"] = error_vs_oracle(stencils, w3, got3,
                                                   sel=np.sort(rng.choice(w3.n, 200000, replace=False)))
        if "fwdbwd" in keep:
            wd, outd0, g0, grad0 = keep["fwdbwd"]
            err["fwd_bwd_96"] = {"ftle": error_vs_oracle(stencils, wd, outd0),
                                 "grad": grad_error_vs_oracle(stencils, wd, g0, grad0)}
        if "batched" in keep:
            err["batched_48"] = {w.name: error_vs_oracle(stencils, w, got) for w, got in keep["batched"]}
        if "fp64" in keep:
            err["fp64_2d_2048_sample"] = error_vs_oracle(stencils, w2, keep["fp64"],
                                                         sel=np.sort(rng.choice(w2.n, 200000, replace=False)))
        if "f16" in keep:
            # against the oracle on the original float32 flow map: the accuracy
            # the binary16 storage gives up (its parity on the decoded map is tested)
            import oracle
            e16 = error_vs_oracle(stencils, w2, keep["f16"])
            # and against the stated bound of that storage (oracle.ftle_perturbation_bound of
            # the binary16 rounding, oracle.flow_error_f16), on a sample
            sel = np.sort(rng.choice(w2.n, 200000, replace=False))
            x32, p32 = w2.coords.astype(np.float32), w2.flow_numpy().astype(np.float32)
            ref = oracle.ftle(2, x32.astype(np.float64), p32.astype(np.float64), stencils.get(w2), w2.T, sel=sel)
            bd = oracle.ftle_perturbation_bound(2, x32, p32, stencils.get(w2), w2.T, oracle.flow_error_f16(x32, p32),
                                                sel=sel)
            fin = np.isfinite(ref) & np.isfinite(bd)
            diff = np.abs(np.asarray(keep["f16"], np.float64)[sel] - ref)
            tol = 2e-5 / (2 * abs(w2.T))
            e16["stated_bound"] = {
                "points": int(sel.size), "finite_fraction": round(float(fin.mean()), 4),
                "within_where_finite": bool(np.all(diff[fin] <= bd[fin] + tol)),
                "median_bound": float(np.median(bd[fin])) if fin.any() else None,
                "max_diff_over_bound": float((diff[fin] / (bd[fin] + tol)).max()) if fin.any() else None}
            err["f16flow_2d_2048_vs_float32_flow"] = e16
        for name in ("ring1_csr_2d_2048", "ring1_csr_3d_160"):
            if name in keep:
                err[name] = stencil_vs_oracle(stencils, *keep[name])
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
        if "advect_grid" in keep:
            wa, vel, gspacing, x0, t0, phi = keep["advect_grid"]
            sel = np.sort(rng.choice(wa.n, 20000, replace=False))
            ref = oracle_advect_grid(vel, gspacing, 0.25, x0[sel].astype(np.float64), t0, wa.T, 0.01)
            err["advect_grid_2d_2048_sample"] = {
                "points": int(sel.size), "max_abs_err": float(np.abs(phi[sel].astype(np.float64) - ref).max())}
        for key in ("ell_2d_2048_direct", "ell_2d_2048_staged", "ell_3d_160_direct", "ell_3d_160_staged"):
            if key in keep:
                we, got, lst = keep[key]
                sel = None if we.dim == 2 else np.sort(rng.choice(we.n, 200000, replace=False))
                e = error_vs_oracle(stencils, we, got, sel=sel, stencil="axis")
                e["list_equals_oracle"] = bool(np.array_equal(lst.ravel(), stencils.axis(we).col))
                err[key] = e
        if "axis_2d_2048" in keep:
            wa, got = keep["axis_2d_2048"]
            err["axis_2d_2048"] = error_vs_oracle(stencils, wa, got, stencil="axis")
        if "axis_3d_160" in keep:
            wa, got = keep["axis_3d_160"]
            err["axis_3d_160_sample"] = error_vs_oracle(stencils, wa, got, stencil="axis",
                                                        sel=np.sort(rng.choice(wa.n, 200000, replace=False)))
        result["error_vs_fp64"] = err

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
