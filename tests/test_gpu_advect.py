"""GPU RK4 flow maps (ftle_advect_rk4) against the FP64 oracle, and the
sliding-window pipeline: one advection call over several meshes' windows
feeding one batched FTLE call.

Tolerance: both sides step the same RK4 in float64; they differ only in the
rounding of the velocity's sines and cosines (the GPU forms sin(pi f) as
sinpi(f)), which the flow's stretching amplifies by at most exp(lambda T)
(lambda < 1 on these flows): 1e-9 absolute over T = 15 is ample.  Float32
output adds its own rounding.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2408_02758_amd as F
from workloads import flows, meshes

pytestmark = pytest.mark.gpu
DEV = "cuda"


@pytest.mark.parametrize("flow,dim", [("double_gyre", 2), ("abc", 3)])
def test_advect_vs_oracle(flow, dim):
    if dim == 2:
        x, _ = meshes.jittered_tri_grid(64, 48, seed=4)
        t0, T, dt = 0.5, 15.0, 0.01
    else:
        x, _ = meshes.kuhn_tet_grid(14)
        t0, T, dt = 0.0, 10.0, 0.02
    ref = oracle.advect_rk4(flow, x, t0, T, dt)
    x64 = torch.as_tensor(x, dtype=torch.float64, device=DEV)
    got = F.advect_rk4(flow, x64, t0, T, dt).cpu().numpy()
    err = np.abs(got - ref).max()
    print(f"[advect {flow} f64] max |d| = {err:.3e}", flush=True)
    assert err < 1e-9
    got32 = F.advect_rk4(flow, x64.float().contiguous(), t0, T, dt).cpu().numpy().astype(np.float64)
    ref32 = oracle.advect_rk4(flow, x.astype(np.float32).astype(np.float64), t0, T, dt)
    assert np.all(np.abs(got32 - ref32) <= 1e-9 + 2 ** -23 * np.abs(ref32))
    # backward in time returns the start up to the RK4 truncation error, which
    # the flow's stretching amplifies (1.3e-6 for the ABC flow at dt = 0.02 over
    # T = 10 and back); and T = 0 is the identity
    back = F.advect_rk4(flow, torch.as_tensor(ref, device=DEV), t0 + T, -T, dt).cpu().numpy()
    assert np.abs(back - x).max() < 1e-5
    assert torch.equal(F.advect_rk4(flow, x64, 1.0, 0.0, dt), x64)


def test_windows_pipeline_vs_oracle():
    """Three meshes, each with its own window (t0, T), advected in one call with
    per-particle times, then their FTLE in one batched call; against the
    oracle's flow maps and FTLE."""
    sides, t0s, Ts = (30, 41, 25), (0.0, 2.5, 7.0), (15.0, 10.0, -12.0)
    geo = [meshes.jittered_tri_grid(s, s, seed=100 + k) for k, s in enumerate(sides)]
    counts = [g[0].shape[0] for g in geo]
    allx = np.concatenate([g[0] for g in geo])
    t0p = np.repeat(t0s, counts)
    Tp = np.repeat(Ts, counts)
    xd = torch.as_tensor(allx, dtype=torch.float64, device=DEV)
    phi = F.advect_rk4("double_gyre", xd, torch.as_tensor(t0p, device=DEV), torch.as_tensor(Tp, device=DEV), 0.01)
    ref_phi = oracle.advect_rk4("double_gyre", allx, t0p, Tp, 0.01)
    assert np.abs(phi.cpu().numpy() - ref_phi).max() < 1e-9
    # the same as one call per window, bit for bit
    off = np.concatenate([[0], np.cumsum(counts)])
    for k in range(3):
        one = F.advect_rk4("double_gyre", xd[off[k]:off[k + 1]].contiguous(), t0s[k], Ts[k], 0.01)
        assert torch.equal(one, phi[off[k]:off[k + 1]])
    ms = [F.Mesh(g[0], g[1], "f64") for g in geo]
    flows_k = [phi[off[k]:off[k + 1]].contiguous() for k in range(3)]
    outs = F.batched(ms, flows_k, list(Ts))
    for k, (g, out) in enumerate(zip(geo, outs)):
        st = oracle.ring1(2, g[0].shape[0], g[1])
        ref = oracle.ftle(2, g[0], ref_phi[off[k]:off[k + 1]], st, Ts[k])
        got = out.cpu().numpy()
        fin = np.isfinite(ref)
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        # the flow maps differ by < 1e-9; the stencil differences amplify that by 1/spacing
        assert np.abs(got[fin] - ref[fin]).max() < 1e-6


def test_advect_large_start_time_and_ragged_steps():
    """Double gyre from a start time far from 0 (a large phase omega t) over a
    duration that is not a whole number of steps, forward and backward: the
    kernel's time factor (advanced by rotations, evaluated directly every few
    steps) against the oracle's direct evaluation at every stage."""
    x, _ = meshes.jittered_tri_grid(20, 15, seed=9)
    x64 = torch.as_tensor(x, dtype=torch.float64, device=DEV)
    for t0, T in ((12345.6, 7.305), (-987.25, -3.3333)):
        ref = oracle.advect_rk4("double_gyre", x, t0, T, 0.01)
        got = F.advect_rk4("double_gyre", x64, t0, T, 0.01).cpu().numpy()
        err = np.abs(got - ref).max()
        print(f"[advect double_gyre t0={t0} T={T}] max |d| = {err:.3e}", flush=True)
        assert err < 1e-9


def test_advect_full_2048_sampled():
    """The measured flow map: all 4,194,304 particles of the 2048^2 jittered
    grid (float32 in and out, as the benchmark times it), 3,000 of them
    against the oracle's RK4 on the same float32 starting points."""
    x, _ = meshes.jittered_tri_grid(2048, 2048, seed=7)
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    phi = F.advect_rk4("double_gyre", torch.as_tensor(x32, device=DEV), 0.0, 15.0, 0.01).cpu().numpy()
    sel = np.unique(np.concatenate([np.random.default_rng(2).choice(x32.shape[0], 3000, replace=False),
                                    np.arange(32), np.arange(x32.shape[0] - 32, x32.shape[0])]))
    ref = oracle.advect_rk4("double_gyre", x32[sel].astype(np.float64), 0.0, 15.0, 0.01)
    err = np.abs(phi[sel].astype(np.float64) - ref)
    print(f"[advect 2048^2 sampled] max |d| = {err.max():.3e}", flush=True)
    assert np.all(err <= 1e-9 + 2.0 ** -23 * np.abs(ref))


# ---------------------------------------------------------------------------
# ftle_advect_rk4_grid: a velocity field sampled on a regular grid
# ---------------------------------------------------------------------------
def _gyre_grid(nx, ny, times):
    """The double gyre at the nodes of an nx x ny grid over [0, 2] x [0, 1]."""
    return flows.sampled_field(flows.double_gyre_velocity, [0.0, 0.0], [2.0 / (nx - 1), 1.0 / (ny - 1)], (nx, ny),
                               times)


def _abc_grid(n):
    """The ABC flow at the nodes of an n^3 grid over [0, 2 pi]^3, and the spacing."""
    h = 2 * np.pi / (n - 1)
    return flows.sampled_field(flows.abc_velocity, [0.0] * 3, [h] * 3, (n, n, n)), h


@pytest.mark.parametrize("vel_dtype", [np.float32, np.float64])
def test_advect_grid_vs_oracle(vel_dtype):
    """Both sides step the same RK4 through the same stored field in float64:
    they differ by rounding only (the summation order of the corner weights),
    amplified by the flow's stretching: 1e-9 over T = 15 as for the analytic flows."""
    times = np.arange(0.0, 20.0 + 1e-9, 0.5)
    vel = _gyre_grid(201, 101, times).astype(vel_dtype)
    x, _ = meshes.jittered_tri_grid(64, 48, seed=5)
    g = np.random.default_rng(2)
    t0s = g.uniform(0.0, 5.0, x.shape[0])
    Ts = g.uniform(-4.0, 15.0, x.shape[0])
    Ts[:7] = 0.0
    ref = oracle.advect_rk4_grid(vel.astype(np.float64), [0.0, 0.0], [0.01, 0.01], 0.0, 0.5, x, t0s, Ts, 0.02)
    vd = torch.as_tensor(vel, device=DEV)
    x64 = torch.as_tensor(x, dtype=torch.float64, device=DEV)
    got = F.advect_rk4_grid(vd, [0.0, 0.0], [0.01, 0.01], 0.0, 0.5, x64, torch.as_tensor(t0s, device=DEV),
                            torch.as_tensor(Ts, device=DEV), 0.02).cpu().numpy()
    err = np.abs(got - ref).max()
    print(f"[advect grid gyre vel={np.dtype(vel_dtype).name}] max |d| = {err:.3e}", flush=True)
    assert err < 1e-9
    assert np.array_equal(got[:7], x[:7])
    # float32 particles: the same up to the output's rounding
    got32 = F.advect_rk4_grid(vd, [0.0, 0.0], [0.01, 0.01], 0.0, 0.5, x64.float().contiguous(), 1.5, 9.0,
                              0.02).cpu().numpy().astype(np.float64)
    ref32 = oracle.advect_rk4_grid(vel.astype(np.float64), [0.0, 0.0], [0.01, 0.01], 0.0, 0.5,
                                   x.astype(np.float32).astype(np.float64), 1.5, 9.0, 0.02)
    assert np.all(np.abs(got32 - ref32) <= 1e-9 + 2 ** -23 * np.abs(ref32))


def test_advect_grid_3d_clamping_and_steady():
    """A sampled ABC field (one slice: steady) in 3D, with particles starting
    outside the grid's box (the nearest box point's velocity), against the oracle."""
    vel, h = _abc_grid(33)
    g = np.random.default_rng(4)
    x = np.concatenate([g.uniform(0.0, 2 * np.pi, size=(3000, 3)), g.uniform(-2.0, 9.0, size=(500, 3))])
    ref = oracle.advect_rk4_grid(vel, [0.0] * 3, [h] * 3, 0.0, 1.0, x, 0.0, 5.0, 0.05)
    got = F.advect_rk4_grid(torch.as_tensor(vel, device=DEV), [0.0] * 3, [h] * 3, 0.0, 1.0,
                            torch.as_tensor(x, device=DEV), 0.0, 5.0, 0.05).cpu().numpy()
    err = np.abs(got - ref).max()
    print(f"[advect grid abc] max |d| = {err:.3e}", flush=True)
    assert err < 1e-9
    assert F.advect_rk4_grid(torch.as_tensor(vel, device=DEV), [0.0] * 3, [h] * 3, 0.0, 1.0,
                             torch.empty(0, 3, dtype=torch.float64, device=DEV), 0.0, 5.0, 0.05).numel() == 0


def test_advect_grid_3d_unsteady():
    """A time-dependent 3D field (the ABC flow with amplitudes varying in
    time) on an anisotropic 17 x 19 x 21 grid at 5 slices, with per-particle
    windows, particles inside and outside the box and times outside the
    slices, float64 and float32 fields, against the oracle."""
    def abc_t(p, t):
        return flows.abc_velocity(p) * (1.0 + 0.3 * torch.sin(0.7 * t))
    shape, spacing, origin = (17, 19, 21), (0.4, 0.35, 0.3), (-0.5, 0.2, -1.0)
    vel = flows.sampled_field(abc_t, origin, spacing, shape, np.arange(5) * 0.8 - 0.4)
    g = np.random.default_rng(6)
    lo, hi = np.array(origin), np.array(origin) + (np.array(shape) - 1) * np.array(spacing)
    x = np.concatenate([g.uniform(lo, hi, size=(2500, 3)), g.uniform(lo - 1.0, hi + 1.0, size=(500, 3))])
    t0s = g.uniform(-1.0, 2.0, x.shape[0])
    Ts = g.uniform(-3.0, 4.0, x.shape[0])
    for vdt in (np.float64, np.float32):
        v = vel.astype(vdt)
        ref = oracle.advect_rk4_grid(v.astype(np.float64), list(origin), list(spacing), -0.4, 0.8, x, t0s, Ts, 0.05)
        got = F.advect_rk4_grid(torch.as_tensor(v, device=DEV), list(origin), list(spacing), -0.4, 0.8,
                                torch.as_tensor(x, device=DEV), torch.as_tensor(t0s, device=DEV),
                                torch.as_tensor(Ts, device=DEV), 0.05).cpu().numpy()
        err = np.abs(got - ref).max()
        print(f"[advect grid 3d unsteady vel={np.dtype(vdt).name}] max |d| = {err:.3e}", flush=True)
        assert err < 1e-9


def test_grid_windows_pipeline_vs_oracle():
    """The sliding-window pipeline from gridded data: three meshes' windows in
    a sampled double gyre (101 x 51 nodes, slices 0.5 apart over [0, 20])
    advected in one call with per-particle times, the same as one call per
    window bit for bit, then one batched FTLE call against the oracle's flow
    maps and FTLE."""
    times = np.arange(41) * 0.5
    vel = torch.as_tensor(_gyre_grid(101, 51, times), device=DEV)
    org, spc = [0.0, 0.0], [0.02, 0.02]
    sides, t0s, Ts = (28, 37, 22), (0.0, 3.25, 19.0), (15.0, 9.5, -11.0)
    geo = [meshes.jittered_tri_grid(s, s, seed=200 + k) for k, s in enumerate(sides)]
    counts = [g[0].shape[0] for g in geo]
    allx = np.concatenate([g[0] for g in geo])
    t0p, Tp = np.repeat(t0s, counts), np.repeat(Ts, counts)
    xd = torch.as_tensor(allx, device=DEV)
    phi = F.advect_rk4_grid(vel, org, spc, 0.0, 0.5, xd, torch.as_tensor(t0p, device=DEV),
                            torch.as_tensor(Tp, device=DEV), 0.01)
    ref_phi = oracle.advect_rk4_grid(vel.cpu().numpy(), org, spc, 0.0, 0.5, allx, t0p, Tp, 0.01)
    assert np.abs(phi.cpu().numpy() - ref_phi).max() < 1e-9
    off = np.concatenate([[0], np.cumsum(counts)])
    for k in range(3):
        one = F.advect_rk4_grid(vel, org, spc, 0.0, 0.5, xd[off[k]:off[k + 1]].contiguous(), t0s[k], Ts[k], 0.01)
        assert torch.equal(one, phi[off[k]:off[k + 1]])
    ms = [F.Mesh(g[0], g[1], "f64") for g in geo]
    outs = F.batched(ms, [phi[off[k]:off[k + 1]].contiguous() for k in range(3)], list(Ts))
    for k, (g, out) in enumerate(zip(geo, outs)):
        st = oracle.ring1(2, g[0].shape[0], g[1])
        ref = oracle.ftle(2, g[0], ref_phi[off[k]:off[k + 1]], st, Ts[k])
        got = out.cpu().numpy()
        fin = np.isfinite(ref)
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        assert np.abs(got[fin] - ref[fin]).max() < 1e-6


def test_advect_grid_full_2048_sampled():
    """The headline's 2048^2 particles through a double gyre sampled on a
    513 x 257 grid at 61 slices (float32 field, T = 15, dt = 0.01, float32
    output), against the oracle on 20,000 sampled particles."""
    times = np.arange(0.0, 15.0 + 1e-9, 0.25)
    vel = _gyre_grid(513, 257, times).astype(np.float32)
    x, _ = meshes.jittered_tri_grid(2048, 2048, seed=2)
    x32 = torch.as_tensor(x, dtype=torch.float32, device=DEV)
    got = F.advect_rk4_grid(torch.as_tensor(vel, device=DEV), [0.0, 0.0], [2.0 / 512, 1.0 / 256], 0.0, 0.25, x32,
                            0.0, 15.0, 0.01).cpu().numpy().astype(np.float64)
    sel = np.sort(np.random.default_rng(8).choice(x.shape[0], 20000, replace=False))
    ref = oracle.advect_rk4_grid(vel.astype(np.float64), [0.0, 0.0], [2.0 / 512, 1.0 / 256], 0.0, 0.25,
                                 x[sel].astype(np.float32).astype(np.float64), 0.0, 15.0, 0.01)
    err = np.abs(got[sel] - ref) - 2 ** -23 * np.abs(ref)
    print(f"[advect grid 2048^2] max |d| beyond output rounding = {err.max():.3e}", flush=True)
    assert np.all(err <= 1e-9)


def test_wrappers_reject_bad_outputs():
    """The Python wrappers check the output tensor (shape, dtype, device, not
    the input) and the grid's origin and spacing lengths before any launch."""
    x = torch.zeros(10, 2, dtype=torch.float64, device=DEV)
    vel = torch.zeros(2, 3, 4, 2, dtype=torch.float32, device=DEV)
    bad = [torch.empty(9, 2, dtype=torch.float64, device=DEV), torch.empty(10, 2, dtype=torch.float32, device=DEV),
           torch.empty(10, 2, dtype=torch.float64), x]
    for out in bad:
        with pytest.raises(ValueError):
            F.advect_rk4("double_gyre", x, 0.0, 1.0, 0.1, out=out)
        with pytest.raises(ValueError):
            F.advect_rk4_grid(vel, [0.0, 0.0], [1.0, 1.0], 0.0, 1.0, x, 0.0, 1.0, 0.1, out=out)
    with pytest.raises(ValueError):
        F.advect_rk4_grid(vel, [0.0, 0.0, 0.0], [1.0, 1.0], 0.0, 1.0, x, 0.0, 1.0, 0.1)
    ok = F.advect_rk4_grid(vel, [0.0, 0.0], [1.0, 1.0], 0.0, 1.0, x, 0.0, 1.0, 0.1)
    assert torch.equal(ok, x)   # a zero field leaves every particle in place
