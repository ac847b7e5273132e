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
from workloads import meshes

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
