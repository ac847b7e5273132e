"""Analytic velocity fields and a fourth-order Runge-Kutta advector (float64).

The flow map phi(x) = x(t0 + T) of a particle that starts at x at time t0 is
the input of the FTLE hot path.  The paper's inputs are precomputed flow maps
from UVaFTLE (Section 2.2); these two classic analytic flows stand in for them:

* the double gyre (Shadden, Lekien and Marsden, Physica D 212, 2005):
  psi = A sin(pi f(x,t)) sin(pi y),  f = eps sin(w t) x^2 + (1 - 2 eps sin(w t)) x,
  u = -dpsi/dy,  v = dpsi/dx;
* the ABC (Arnold-Beltrami-Childress) flow:
  u = A sin z + C cos y,  v = B sin x + A cos z,  w = C sin y + B cos x.

Advection runs in float64 with torch on the device the caller names (CPU for
small test meshes, the GPU for the large workloads).  This is input
generation only: no part of the FTLE computation happens here.
"""
from __future__ import annotations

import math

import torch


def double_gyre_velocity(p: torch.Tensor, t: torch.Tensor, A: float = 0.1, eps: float = 0.25,
                         omega: float = 2.0 * math.pi / 10.0) -> torch.Tensor:
    """Velocity of the time-periodic double gyre at points p (N,2) and times t (N,) or scalar."""
    x, y = p[:, 0], p[:, 1]
    s = torch.sin(omega * t)
    a = eps * s
    b = 1.0 - 2.0 * eps * s
    f = a * x * x + b * x
    dfdx = 2.0 * a * x + b
    u = -math.pi * A * torch.sin(math.pi * f) * torch.cos(math.pi * y)
    v = math.pi * A * torch.cos(math.pi * f) * torch.sin(math.pi * y) * dfdx
    return torch.stack([u, v], dim=1)


def abc_velocity(p: torch.Tensor, t: torch.Tensor | None = None, A: float = math.sqrt(3.0),
                 B: float = math.sqrt(2.0), C: float = 1.0) -> torch.Tensor:
    """Velocity of the steady ABC flow at points p (N,3)."""
    x, y, z = p[:, 0], p[:, 1], p[:, 2]
    return torch.stack([A * torch.sin(z) + C * torch.cos(y),
                        B * torch.sin(x) + A * torch.cos(z),
                        C * torch.sin(y) + B * torch.cos(x)], dim=1)


def steps_for(T: float, dt: float) -> int:
    """Number of RK4 steps: ceil(|T|/dt) (the step is then shrunk to T/steps)."""
    return max(1, int(math.ceil(abs(T) / dt - 1e-9)))


@torch.no_grad()
def advect_rk4(velocity, p0, t0, T, dt: float, device=None) -> torch.Tensor:
    """Classical RK4 advection of points p0 from t0 over T.

    p0: array-like (N, D) float64.  t0 and T: scalars or per-point arrays (N,)
    (per-point values let one call advect many independent meshes, each with
    its own window).  Each point takes steps_for(T, dt) steps of size
    T/steps.  Returns a float64 tensor (N, D) on ``device``.
    """
    dev = torch.device(device) if device is not None else torch.device("cpu")
    p = torch.as_tensor(p0, dtype=torch.float64, device=dev).clone()
    n = p.shape[0]
    t0 = torch.as_tensor(t0, dtype=torch.float64, device=dev).expand(n).clone()
    T = torch.as_tensor(T, dtype=torch.float64, device=dev).expand(n).clone()
    nsteps = torch.ceil(T.abs() / dt - 1e-9).clamp_min(1)
    h = T / nsteps
    max_steps = int(nsteps.max().item()) if n else 0
    uniform = bool((nsteps == nsteps[0]).all().item()) if n else True
    for s in range(max_steps):
        t = t0 + s * h
        k1 = velocity(p, t)
        k2 = velocity(p + (0.5 * h)[:, None] * k1, t + 0.5 * h)
        k3 = velocity(p + (0.5 * h)[:, None] * k2, t + 0.5 * h)
        k4 = velocity(p + h[:, None] * k3, t + h)
        incr = (h / 6.0)[:, None] * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        if uniform:
            p += incr
        else:
            p += torch.where((s < nsteps)[:, None], incr, torch.zeros_like(incr))
    return p


@torch.no_grad()
def sampled_field(velocity, origin, spacing, shape, times=(0.0,)) -> "numpy.ndarray":
    """A velocity field sampled on a regular grid, the gridded input of
    ftle_advect_rk4_grid: nodes origin[d] + i spacing[d] for i < shape[d]
    (x fastest) at each of ``times``.  Returns a float64 array of shape
    (len(times), [nz,] ny, nx, D)."""
    D = len(shape)
    axes = [torch.arange(shape[d], dtype=torch.float64) * spacing[d] + origin[d] for d in range(D)]
    grids = torch.meshgrid(*axes[::-1], indexing="ij")          # slowest axis first
    pts = torch.stack([g.reshape(-1) for g in grids[::-1]], dim=1)
    out = []
    for t in times:
        v = velocity(pts, torch.tensor(float(t), dtype=torch.float64))
        out.append(v.reshape(*[shape[d] for d in range(D)][::-1], D))
    return torch.stack(out).numpy()
