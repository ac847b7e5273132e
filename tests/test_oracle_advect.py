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
