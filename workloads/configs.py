"""The named synthetic FTLE workloads (seeded), built from meshes.py and flows.py.

Five workloads, each with the sizes and structure of a case the FTLE hot path
is measured on:

* ``small_2d``   -- 64x64 jittered triangulated grid on [0,2]x[0,1], double
  gyre (A=0.1, eps=0.25, omega=2 pi/10) from t0=0 over T=15 with RK4 dt=0.01;
  stored in float64 (4096 points).
* ``scale_2d``   -- the same construction at 2048x2048 (4,194,304 points),
  stored in float32.
* ``abc_3d``     -- 160^3 structured points on [0,2 pi]^3, 6 tetrahedra per
  cube, ABC flow (A=sqrt 3, B=sqrt 2, C=1) over T=10 with RK4 dt=0.02, float32.
* ``batched_2d`` -- 48 jittered triangulated meshes with sides log-uniform in
  [64,1024], each with its own window start t0 ~ U[0,10] and length
  T ~ U[5,20], float32.
* ``diff_3d``    -- 96^3 ABC mesh (T=10, float32) with loss weights w ~ N(0,1).

``dtype`` is the storage precision: the float32 workloads round coordinates
and flow map to float32 once, and every consumer (oracle or GPU) reads those
same rounded values.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import flows, meshes


@dataclass
class Workload:
    name: str
    dim: int
    coords: np.ndarray          # (N, dim), storage dtype
    cells: np.ndarray           # (ncells, dim+1) int32
    flow: torch.Tensor          # (N, dim), storage dtype, on the generating device
    T: float
    dtype: str                  # "f64" or "f32"
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.coords.shape[0]

    def flow_numpy(self) -> np.ndarray:
        return self.flow.detach().cpu().numpy()


def _store(coords, flow, dtype):
    if dtype == "f32":
        return coords.astype(np.float32), flow.to(torch.float32)
    return coords.astype(np.float64), flow.to(torch.float64)


def tri2d(nx: int, ny: int, seed: int, t0: float, T: float, dtype: str, device="cpu",
          name: str | None = None) -> Workload:
    coords, cells = meshes.jittered_tri_grid(nx, ny, seed)
    phi = flows.advect_rk4(flows.double_gyre_velocity, coords, t0, T, 0.01, device)
    c, f = _store(coords, phi, dtype)
    return Workload(name or f"tri2d_{nx}x{ny}", 2, c, cells, f, T, dtype,
                    {"seed": seed, "t0": t0})


def small_2d(device="cpu") -> Workload:
    return tri2d(64, 64, seed=1, t0=0.0, T=15.0, dtype="f64", device=device, name="small_2d")


def scale_2d(device="cpu", n: int = 2048) -> Workload:
    return tri2d(n, n, seed=2, t0=0.0, T=15.0, dtype="f32", device=device, name=f"scale_2d_{n}")


def abc3d(n: int, T: float, dtype: str, device="cpu", name: str | None = None) -> Workload:
    coords, cells = meshes.kuhn_tet_grid(n)
    phi = flows.advect_rk4(flows.abc_velocity, coords, 0.0, T, 0.02, device)
    c, f = _store(coords, phi, dtype)
    return Workload(name or f"abc3d_{n}", 3, c, cells, f, T, dtype, {})


def abc_3d(device="cpu", n: int = 160) -> Workload:
    return abc3d(n, 10.0, "f32", device, name=f"abc_3d_{n}")


def diff_3d(device="cpu", n: int = 96, weight_seed: int = 5) -> Workload:
    w = abc3d(n, 10.0, "f32", device, name=f"diff_3d_{n}")
    w.extra["weights"] = np.random.default_rng(weight_seed).standard_normal(w.n)
    return w


def batched_params(count: int = 48, seed: int = 3, lo: int = 64, hi: int = 1024):
    """Draw order: all sides, then all window starts t0, then all lengths T."""
    rng = np.random.default_rng(seed)
    sides = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), count))).astype(int)
    t0 = rng.uniform(0.0, 10.0, count)
    T = rng.uniform(5.0, 20.0, count)
    return sides, t0, T


def batched_2d(device="cpu", count: int = 48, seed: int = 3, lo: int = 64, hi: int = 1024):
    """Independent meshes; mesh k uses jitter seed 1000+k.  All are advected in one call."""
    sides, t0, T = batched_params(count, seed, lo, hi)
    geo = [meshes.jittered_tri_grid(int(s), int(s), 1000 + k) for k, s in enumerate(sides)]
    counts = [g[0].shape[0] for g in geo]
    allc = np.concatenate([g[0] for g in geo])
    t0_pt = np.repeat(t0, counts)
    T_pt = np.repeat(T, counts)
    phi = flows.advect_rk4(flows.double_gyre_velocity, allc, t0_pt, T_pt, 0.01, device)
    out = []
    off = 0
    for k, (c, cells) in enumerate(geo):
        n = c.shape[0]
        cc, ff = _store(c, phi[off:off + n], "f32")
        out.append(Workload(f"batched_{k}_{sides[k]}", 2, cc, cells, ff.contiguous(), float(T[k]),
                            "f32", {"seed": 1000 + k, "t0": float(t0[k])}))
        off += n
    return out
