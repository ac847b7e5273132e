"""The oracle's RK4 flow maps (oracle_advect_rk4) against what fixes them (CPU only).

* a second implementation of the same steps (the workload generator's
  torch RK4 in workloads/flows.py) agrees to rounding;
* an independent integrator (scipy's DOP853 at tolerance 1e-12) agrees within
  the RK4 truncation error;
* time reversal: advecting back from t0 + T over -T returns the start;
* the steady double gyre (eps = 0) keeps its stream function constant along
  trajectories;
* the ABC flow is divergence free: det of the flow map's Jacobian is 1;
* T = 0 is the identity; per-particle windows equal separate calls.
"""
import math

import numpy as np
import pytest

import oracle
from workloads import flows, meshes

GYRE = dict(A=0.1, eps=0.25, omega=2.0 * math.pi / 10.0)


def _pts2(n=15, seed=1):
    x, _ = meshes.jittered_tri_grid(n, n, seed=seed)
    return x


def _pts3(n=5):
    x, _ = meshes.kuhn_tet_grid(n)
    return x


def test_matches_second_implementation():
    x2 = _pts2()
    a = oracle.advect_rk4("double_gyre", x2, 0.5, 15.0, 0.01)
    b = flows.advect_rk4(flows.double_gyre_velocity, x2, 0.5, 15.0, 0.01).numpy()
    assert np.abs(a - b).max() < 1e-12
    x3 = _pts3()
    a = oracle.advect_rk4("abc", x3, 0.0, 10.0, 0.02)
    b = flows.advect_rk4(flows.abc_velocity, x3, 0.0, 10.0, 0.02).numpy()
    assert np.abs(a - b).max() < 1e-11


def _gyre_rhs(t, p):
    s = math.sin(GYRE["omega"] * t)
    a, b = GYRE["eps"] * s, 1.0 - 2.0 * GYRE["eps"] * s
    f = a * p[0] ** 2 + b * p[0]
    return [-math.pi * GYRE["A"] * math.sin(math.pi * f) * math.cos(math.pi * p[1]),
            math.pi * GYRE["A"] * math.cos(math.pi * f) * math.sin(math.pi * p[1]) * (2 * a * p[0] + b)]


def _abc_rhs(t, p):
    A, B, C = math.sqrt(3.0), math.sqrt(2.0), 1.0
    return [A * math.sin(p[2]) + C * math.cos(p[1]), B * math.sin(p[0]) + A * math.cos(p[2]),
            C * math.sin(p[1]) + B * math.cos(p[0])]


def test_independent_integrator():
    from scipy.integrate import solve_ivp
    for flow, rhs, x, t0, T, dt, tol in (("double_gyre", _gyre_rhs, _pts2(6), 1.0, 5.0, 0.01, 1e-9),
                                         ("abc", _abc_rhs, _pts3(3), 0.0, 2.0, 0.01, 1e-8)):
        got = oracle.advect_rk4(flow, x, t0, T, dt)
        for i in range(x.shape[0]):
            ref = solve_ivp(rhs, (t0, t0 + T), x[i], method="DOP853", rtol=1e-12, atol=1e-12).y[:, -1]
            assert np.abs(got[i] - ref).max() < tol, (flow, i)


@pytest.mark.parametrize("flow,x", [("double_gyre", _pts2(10)), ("abc", _pts3(4))])
def test_time_reversal(flow, x):
    t0, T, dt = 0.3, 4.0, 0.005
    fwd = oracle.advect_rk4(flow, x, t0, T, dt)
    back = oracle.advect_rk4(flow, fwd, t0 + T, -T, dt)
    assert np.abs(back - x).max() < 1e-8


def test_steady_gyre_keeps_stream_function():
    x = _pts2(12)
    phi = oracle.advect_rk4("double_gyre", x, 0.0, 8.0, 0.005, params=(0.1, 0.0, 1.0))
    psi = lambda p: 0.1 * np.sin(np.pi * p[:, 0]) * np.sin(np.pi * p[:, 1])  # noqa: E731
    assert np.abs(psi(phi) - psi(x)).max() < 1e-10
    assert np.abs(phi - x).max() > 1e-2   # the particles did move


def test_abc_preserves_volume():
    x = np.array([[0.3, 1.1, 2.0], [4.0, 0.5, 5.5]])
    h = 1e-5
    for p in x:
        J = np.empty((3, 3))
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            J[:, k] = (oracle.advect_rk4("abc", p + e, 0.0, 3.0, 0.01)[0] -
                       oracle.advect_rk4("abc", p - e, 0.0, 3.0, 0.01)[0]) / (2 * h)
        assert abs(np.linalg.det(J) - 1.0) < 1e-5


def test_identity_and_windows():
    x = _pts2(8)
    assert np.array_equal(oracle.advect_rk4("double_gyre", x, 2.0, 0.0, 0.01), x)
    n = x.shape[0]
    t0 = np.where(np.arange(n) % 2 == 0, 0.0, 3.0)
    T = np.where(np.arange(n) % 3 == 0, 5.0, -2.5)
    got = oracle.advect_rk4("double_gyre", x, t0, T, 0.01)
    for i in range(0, n, 7):
        assert np.array_equal(got[i], oracle.advect_rk4("double_gyre", x[i:i + 1], t0[i], T[i], 0.01)[0])


# ---------------------------------------------------------------------------
# advect_rk4_grid: a velocity field sampled on a regular grid
# ---------------------------------------------------------------------------
def _sample_field(fn, dim, n_nodes, lo, hi, times):
    """fn(points (m, dim), t) sampled at the nodes, array (n_times, [nz,] ny, nx, dim)."""
    axes = [np.linspace(lo, hi, n_nodes) for _ in range(dim)]
    if dim == 2:
        yy, xx = np.meshgrid(axes[1], axes[0], indexing="ij")
        pts = np.stack([xx, yy], axis=-1).reshape(-1, 2)
    else:
        zz, yy, xx = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
        pts = np.stack([xx, yy, zz], axis=-1).reshape(-1, 3)
    shape = (n_nodes,) * dim
    return np.stack([fn(pts, t).reshape(*shape, dim) for t in times])


@pytest.mark.parametrize("dim", [2, 3])
def test_grid_affine_field_matches_closed_form(dim):
    """u = A x + b is reproduced exactly by multilinear interpolation, and the
    flow map of a linear ODE is expm(A T) x0 + A^-1 (expm(A T) - I) b: RK4 agrees
    within its truncation error."""
    from scipy.linalg import expm
    g = np.random.default_rng(dim)
    A = g.normal(size=(dim, dim)) * 0.15
    b = g.normal(size=dim) * 0.2
    vel = _sample_field(lambda p, t: p @ A.T + b, dim, 13, -6.0, 6.0, [0.0])
    x0 = g.uniform(-1, 1, size=(50, dim))
    T = 1.5
    got = oracle.advect_rk4_grid(vel, [-6.0] * dim, [1.0] * dim, 0.0, 1.0, x0, 0.3, T, 0.01)
    E = expm(A * T)
    want = x0 @ E.T + np.linalg.solve(A, (E - np.eye(dim)) @ b)
    assert np.abs(want).max() < 5.0   # the particles stay inside the grid's box
    assert np.abs(got - want).max() < 1e-8


def test_grid_time_linear_field_matches_independent_integrator():
    """u = A x + b + t c: linear interpolation in time between slices is exact;
    scipy's DOP853 on the exact field agrees within the RK4 error."""
    from scipy.integrate import solve_ivp
    g = np.random.default_rng(7)
    A = g.normal(size=(2, 2)) * 0.3
    b, c = g.normal(size=2) * 0.2, g.normal(size=2) * 0.1
    times = np.arange(0.0, 3.01, 0.5)
    vel = _sample_field(lambda p, t: p @ A.T + b + t * c, 2, 5, -5.0, 5.0, times)
    x0 = g.uniform(-1, 1, size=(20, 2))
    got = oracle.advect_rk4_grid(vel, [-5.0, -5.0], [2.5, 2.5], 0.0, 0.5, x0, 0.2, 2.5, 0.01)
    for i in range(20):
        ref = solve_ivp(lambda t, y: A @ y + b + t * c, (0.2, 2.7), x0[i], method="DOP853", rtol=1e-12, atol=1e-12)
        assert np.abs(got[i] - ref.y[:, -1]).max() < 1e-8


def test_grid_double_gyre_converges_at_second_order():
    """The double gyre sampled on grids of spacing h and h/2: the flow maps
    approach the analytic field's (oracle.advect_rk4) by the factor 4 that
    multilinear interpolation's O(h^2) error gives."""
    ga = oracle.FLOWS["double_gyre"][2]
    x0 = _pts2(12, seed=3)
    T, t0 = 2.0, 0.5
    ref = oracle.advect_rk4("double_gyre", x0, t0, T, 0.01)
    errs = []
    for nx in (41, 81):
        ny = (nx - 1) // 2 + 1
        h = 2.0 / (nx - 1)
        times = np.arange(0.0, 3.0 + 1e-9, 0.05)

        def fn(p, t):
            v = np.empty_like(p)
            for k in range(p.shape[0]):
                v[k] = _gyre_velocity(p[k], t, ga)
            return v
        xs, ys = np.linspace(0, 2, nx), np.linspace(0, 1, ny)
        yy, xx = np.meshgrid(ys, xs, indexing="ij")
        pts = np.stack([xx, yy], -1).reshape(-1, 2)
        vel = np.stack([fn(pts, t).reshape(ny, nx, 2) for t in times])
        got = oracle.advect_rk4_grid(vel, [0.0, 0.0], [h, h], 0.0, 0.05, x0, t0, T, 0.01)
        errs.append(np.abs(got - ref).max())
    assert errs[1] < errs[0] / 3.0, errs


def _gyre_velocity(p, t, prm):
    A, eps, om = prm
    s = math.sin(om * t)
    a, b = eps * s, 1 - 2 * eps * s
    f = a * p[0] ** 2 + b * p[0]
    return np.array([-math.pi * A * math.sin(math.pi * f) * math.cos(math.pi * p[1]),
                     math.pi * A * math.cos(math.pi * f) * math.sin(math.pi * p[1]) * (2 * a * p[0] + b)])


def test_grid_clamping_in_space_and_time():
    """Outside the grid's box the velocity is the nearest box point's, before
    the first slice or after the last that slice's; one slice is a steady
    field; RK4 integrates the piecewise polynomial velocities here exactly."""
    # u = (x, 0) sampled on [0, 1]^2: a particle at x = 2 sees u = 1, one at x = -1 sees 0
    vel = _sample_field(lambda p, t: np.stack([p[:, 0], 0 * p[:, 1]], 1), 2, 3, 0.0, 1.0, [0.0])
    got = oracle.advect_rk4_grid(vel, [0.0, 0.0], [0.5, 0.5], 0.0, 1.0, np.array([[2.0, 0.5], [-1.0, 3.0]]),
                                 0.0, 1.5, 0.1)
    assert np.allclose(got, [[3.5, 0.5], [-1.0, 3.0]], rtol=0, atol=1e-14)
    # uniform u = (1 + t, 0) on slices t = 0, 1: x(1) - x(0) = 1.5; after the last slice u = 2
    vel = np.stack([np.tile([1.0, 0.0], (2, 2, 1)), np.tile([2.0, 0.0], (2, 2, 1))])
    got = oracle.advect_rk4_grid(vel, [0.0, 0.0], [1.0, 1.0], 0.0, 1.0, np.zeros((2, 2)), np.array([0.0, 5.0]),
                                 1.0, 0.25)
    assert np.allclose(got, [[1.5, 0.0], [2.0, 0.0]], rtol=0, atol=1e-13)
    # one slice = two equal slices
    g = np.random.default_rng(1)
    v1 = g.normal(size=(1, 4, 5, 2))
    x0 = g.uniform(0, 3, size=(30, 2))
    a = oracle.advect_rk4_grid(v1, [0.0, 0.0], [1.0, 1.0], 0.0, 1.0, x0, 0.0, 2.0, 0.05)
    b = oracle.advect_rk4_grid(np.concatenate([v1, v1]), [0.0, 0.0], [1.0, 1.0], 0.0, 1.0, x0, 0.0, 2.0, 0.05)
    assert np.abs(a - b).max() < 1e-13
