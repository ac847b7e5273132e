"""Pins of the FTLE oracle against what the mathematics fixes.

The paper prints no FTLE value, gradient formula or worked example, so the
oracle is pinned by closed forms, invariants, library routines it must reduce
to, and brute force:

  check_ring1_bruteforce   stencil = every vertex sharing a cell (Section 2.2 list)
  check_eig3_vs_numpy      3x3 Jacobi eigenpairs == numpy.linalg.eigh
  check_lstsq_fan          per-point J == numpy.linalg.lstsq on random stencils;
                           rank-deficient stencils give NaN
  check_affine             phi = A x + b  ->  FTLE = ln sigma_max(A) / |T|  (numpy svd)
  check_rigid_and_scaling  rotations/translations -> 0; phi = s x -> ln|s|/|T|;
                           FTLE*|T| independent of T, sign of T irrelevant
  check_axis_gradient      the paper's 4/6-slot list on a regular grid reduces
                           the least-squares gradient to numpy.gradient
                           (central inside, one-sided at the edge)
  check_invariances        FTLE(Q phi + b) = FTLE(phi); joint rotation of x, phi
  check_relabel            relabelling points/cells permutes the output
  check_adjoint_fd         dL/dphi == central differences (h = 1e-6) of the oracle
  check_adjoint_identities translation, scaling and rotation identities of dL/dphi

Each check takes an oracle library handle (``lib=None`` is the normal build)
and raises AssertionError when the pin does not hold, so that the same checks
can be run against builds of the oracle with a deliberately planted mistake.
"""
from __future__ import annotations

import numpy as np

import oracle
from workloads import flows, meshes


def _rot2(th):
    c, s = np.cos(th), np.sin(th)
    return np.array([[c, -s], [s, c]])


def _rand_rot(dim, rng):
    q, r = np.linalg.qr(rng.standard_normal((dim, dim)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def _rand_well_conditioned(dim, rng, lo=0.5, hi=5.0):
    u = _rand_rot(dim, rng)
    v = _rand_rot(dim, rng)
    s = np.sort(rng.uniform(lo, hi, dim))[::-1]
    return u @ np.diag(s) @ v.T


def _mesh2d(nx=12, ny=9, seed=4):
    return meshes.jittered_tri_grid(nx, ny, seed)


def _mesh3d(n=5, seed=7, jitter=0.2):
    x, cells = meshes.kuhn_tet_grid(n)
    h = 2 * np.pi / (n - 1)
    rng = np.random.default_rng(seed)
    return x + rng.uniform(-jitter, jitter, x.shape) * h, cells


def _smooth_map(x):
    """A nonlinear smooth map R^D -> R^D used as a test flow map."""
    if x.shape[1] == 2:
        return np.stack([np.sin(1.3 * x[:, 0]) + 0.4 * x[:, 1] ** 2,
                         np.cos(0.7 * x[:, 1]) + 0.3 * x[:, 0] * x[:, 1]], 1)
    return np.stack([np.sin(0.9 * x[:, 0]) + 0.2 * x[:, 1] * x[:, 2],
                     np.cos(0.6 * x[:, 1]) + 0.3 * x[:, 0] ** 2,
                     0.5 * x[:, 2] + 0.1 * np.sin(x[:, 0] * x[:, 1])], 1)


# --------------------------------------------------------------------------


def check_ring1_bruteforce(lib=None):
    cases = [(2,) + _mesh2d(9, 7, 3), (3,) + _mesh3d(4)]
    x2, c2, _ = meshes.relabel(*_mesh2d(9, 7, 3), seed=9)
    cases.append((2, x2, c2))
    # degenerate cells with a repeated vertex must not make a point its own neighbour
    cases.append((2, np.zeros((4, 2)), np.array([[0, 1, 1], [1, 2, 3], [3, 3, 3]], dtype=np.int32)))
    for dim, x, cells in cases:
        n = x.shape[0]
        st = oracle.ring1(dim, n, cells, lib=lib)
        nb = [set() for _ in range(n)]
        for cell in cells:
            for a in cell:
                for b in cell:
                    if a != b:
                        nb[a].add(int(b))
        for i in range(n):
            got = list(st.col[st.row_ptr[i]:st.row_ptr[i + 1]])
            assert got == sorted(nb[i]), (dim, i, got, sorted(nb[i]))


def check_eig3_vs_numpy(lib=None):
    rng = np.random.default_rng(11)
    mats = []
    for _ in range(300):
        a = rng.standard_normal((3, 3)) * 10 ** rng.uniform(-3, 3)
        mats.append(a + a.T)
    q = _rand_rot(3, rng)
    mats += [np.zeros((3, 3)), np.diag([2.0, 2.0, 5.0]), np.diag([4.0, 1.0, 1.0]),
             q @ np.diag([3.0, 3.0, -1.0]) @ q.T, q @ np.diag([7.0, 7.0 * (1 + 1e-9), 0.5]) @ q.T,
             np.outer([1.0, 2.0, -0.5], [1.0, 2.0, -0.5])]
    for m in mats:
        vals, vecs = oracle.jacobi_eig3(m, lib=lib)
        ref = np.linalg.eigvalsh(m)
        scale = max(1.0, np.linalg.norm(m))
        assert np.allclose(vals, ref, rtol=0, atol=1e-13 * scale), (m, vals, ref)
        assert np.allclose(m @ vecs, vecs * vals, rtol=0, atol=1e-12 * scale)
        assert np.allclose(vecs.T @ vecs, np.eye(3), atol=1e-12)


def _ref_ftle_from_J(J, T):
    C = np.einsum("...ra,...rb->...ab", J, J)
    lam = np.linalg.eigvalsh(C)[..., -1]
    return 0.5 * np.log(lam) / abs(T)


def check_lstsq_fan(lib=None):
    rng = np.random.default_rng(12)
    T = 2.5
    for dim in (2, 3):
        for k in range(dim, 13):
            x = np.vstack([rng.uniform(-1, 1, (1, dim)), rng.uniform(-1, 1, (k, dim))])
            phi = rng.standard_normal((k + 1, dim))
            if dim == 2:
                cells = np.array([[0, j, j + 1] for j in range(1, k)] or [[0, 1, 1]], dtype=np.int32)
            else:
                cells = np.array([[0, j, j + 1, j + 2] for j in range(1, k - 1)] or [[0, 1, 2, 2]],
                                 dtype=np.int32)
            if k < dim + (1 if dim == 2 else 2):
                # not enough distinct cells: connect point 0 to all k directly
                cells = np.array([[0] + [1 + (j + t) % k for t in range(dim)] for j in range(k)],
                                 dtype=np.int32)
            st = oracle.ring1(dim, k + 1, cells, lib=lib)
            assert list(st.col[:st.row_ptr[1]]) == list(range(1, k + 1))
            f = oracle.ftle(dim, x, phi, st, T, sel=[0], lib=lib)[0]
            X = x[1:] - x[0]
            F = phi[1:] - phi[0]
            Jt = np.linalg.lstsq(X, F, rcond=None)[0]
            ref = _ref_ftle_from_J(Jt.T, T)
            assert abs(f - ref) <= 1e-12 * max(1.0, abs(ref)), (dim, k, f, ref)
    # rank-deficient stencils and isolated points give NaN
    x = np.array([[0.0, 0.0], [1.0, 1.0], [2.0, 2.0], [-1.0, -1.0], [5.0, 0.0]])
    cells = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    st = oracle.ring1(2, 5, cells, lib=lib)
    f = oracle.ftle(2, x, rng.standard_normal((5, 2)), st, 1.0, lib=lib)
    assert np.isnan(f[0]) and np.isnan(f[4])
    x3 = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0], [3, 3, 3]], dtype=np.float64)
    cells3 = np.array([[0, 1, 2, 3]], dtype=np.int32)
    st3 = oracle.ring1(3, 5, cells3, lib=lib)
    f3 = oracle.ftle(3, x3, rng.standard_normal((5, 3)), st3, 1.0, lib=lib)
    assert np.all(np.isnan(f3))


def check_affine(lib=None):
    rng = np.random.default_rng(13)
    for dim, (x, cells) in ((2, _mesh2d()), (3, _mesh3d())):
        st = oracle.ring1(dim, x.shape[0], cells, lib=lib)
        for _ in range(3):
            A = _rand_well_conditioned(dim, rng)
            b = rng.standard_normal(dim)
            phi = x @ A.T + b
            for T in (3.7, -0.8):
                f = oracle.ftle(dim, x, phi, st, T, lib=lib)
                ref = np.log(np.linalg.svd(A, compute_uv=False)[0]) / abs(T)
                assert np.all(np.isfinite(f))
                assert np.max(np.abs(f - ref)) <= 1e-12 * max(1.0, abs(ref)), (dim, T, f[:4], ref)


def check_rigid_and_scaling(lib=None):
    rng = np.random.default_rng(14)
    for dim, (x, cells) in ((2, _mesh2d()), (3, _mesh3d())):
        st = oracle.ring1(dim, x.shape[0], cells, lib=lib)
        Q = _rand_rot(dim, rng)
        for phi in (x @ Q.T + rng.standard_normal(dim), x + 3.0):
            f = oracle.ftle(dim, x, phi, st, 4.0, lib=lib)
            assert np.max(np.abs(f)) <= 1e-13, np.max(np.abs(f))
        for s in (2.5, -0.7):
            f = oracle.ftle(dim, x, s * x, st, 1.5, lib=lib)
            assert np.allclose(f, np.log(abs(s)) / 1.5, rtol=1e-13, atol=0)
        phi = _smooth_map(x)
        f1 = oracle.ftle(dim, x, phi, st, 1.0, lib=lib)
        f2 = oracle.ftle(dim, x, phi, st, 7.5, lib=lib)
        f3 = oracle.ftle(dim, x, phi, st, -7.5, lib=lib)
        assert np.allclose(f1, 7.5 * f2, rtol=1e-14, atol=1e-15)
        assert np.array_equal(f2, f3)


def check_axis_gradient(lib=None):
    # 2D: regular grid, the triangulation of jittered_tri_grid with zero jitter
    nx, ny = 11, 7
    x, cells = meshes.jittered_tri_grid(nx, ny, seed=0, jitter=0.0)
    hx, hy = 2.0 / nx, 1.0 / ny
    ring = oracle.ring1(2, x.shape[0], cells, lib=lib)
    ax = oracle.axis(2, x, ring, lib=lib)
    slots = ax.col.reshape(-1, 4)
    for j in range(ny):
        for i in range(nx):
            p = j * nx + i
            want = [p - 1 if i > 0 else -1, p + 1 if i < nx - 1 else -1,
                    p - nx if j > 0 else -1, p + nx if j < ny - 1 else -1]
            assert list(slots[p]) == want, (i, j, list(slots[p]), want)
    phi = _smooth_map(x)
    T = 3.0
    f = oracle.ftle(2, x, phi, ax, T, lib=lib)
    J = np.empty((x.shape[0], 2, 2))
    for r in range(2):
        F = phi[:, r].reshape(ny, nx)
        J[:, r, 0] = np.gradient(F, hx, axis=1, edge_order=1).ravel()
        J[:, r, 1] = np.gradient(F, hy, axis=0, edge_order=1).ravel()
    ref = _ref_ftle_from_J(J, T)
    assert np.max(np.abs(f - ref)) <= 1e-11 * max(1.0, np.max(np.abs(ref))), np.max(np.abs(f - ref))
    # 3D: structured Kuhn grid
    n = 6
    x3, cells3 = meshes.kuhn_tet_grid(n)
    h = 2 * np.pi / (n - 1)
    ring3 = oracle.ring1(3, x3.shape[0], cells3, lib=lib)
    ax3 = oracle.axis(3, x3, ring3, lib=lib)
    phi3 = _smooth_map(x3)
    f3 = oracle.ftle(3, x3, phi3, ax3, T, lib=lib)
    J3 = np.empty((x3.shape[0], 3, 3))
    for r in range(3):
        F = phi3[:, r].reshape(n, n, n)      # [k, j, i]
        for c, axis in ((0, 2), (1, 1), (2, 0)):
            J3[:, r, c] = np.gradient(F, h, axis=axis, edge_order=1).ravel()
    ref3 = _ref_ftle_from_J(J3, T)
    assert np.max(np.abs(f3 - ref3)) <= 1e-11 * max(1.0, np.max(np.abs(ref3)))


def check_invariances(w2, w3, lib=None):
    rng = np.random.default_rng(15)
    for w in (w2, w3):
        x = w.coords.astype(np.float64)
        phi = w.flow_numpy().astype(np.float64)
        st = oracle.ring1(w.dim, w.n, w.cells, lib=lib)
        f0 = oracle.ftle(w.dim, x, phi, st, w.T, lib=lib)
        scale = max(1.0, np.max(np.abs(f0)))
        Q = _rand_rot(w.dim, rng)
        f1 = oracle.ftle(w.dim, x, phi @ Q.T + rng.standard_normal(w.dim), st, w.T, lib=lib)
        assert np.max(np.abs(f1 - f0)) <= 1e-11 * scale
        R = _rand_rot(w.dim, rng)
        f2 = oracle.ftle(w.dim, x @ R.T, phi @ R.T, st, w.T, lib=lib)
        assert np.max(np.abs(f2 - f0)) <= 1e-11 * scale


def check_relabel(w2, lib=None):
    x = w2.coords.astype(np.float64)
    phi = w2.flow_numpy()
    st = oracle.ring1(2, w2.n, w2.cells, lib=lib)
    f0 = oracle.ftle(2, x, phi, st, w2.T, lib=lib)
    x2, c2, p = meshes.relabel(x, w2.cells, seed=21)
    phi2 = np.empty_like(phi)
    phi2[p] = phi
    st2 = oracle.ring1(2, w2.n, c2, lib=lib)
    f2 = oracle.ftle(2, x2, phi2, st2, w2.T, lib=lib)
    assert np.max(np.abs(f2[p] - f0)) <= 1e-12 * max(1.0, np.max(np.abs(f0)))


def _adjoint_cases(w3=None):
    x2, c2 = meshes.jittered_tri_grid(12, 10, seed=5)
    phi2 = flows.advect_rk4(flows.double_gyre_velocity, x2, 0.0, 5.0, 0.01).numpy()
    cases = [(2, x2, c2, phi2, 5.0, np.random.default_rng(16).standard_normal(x2.shape[0]))]
    if w3 is not None:
        cases.append((3, w3.coords.astype(np.float64), w3.cells, w3.flow_numpy(), w3.T,
                      np.random.default_rng(6).standard_normal(w3.n)))
    else:
        x3, c3 = _mesh3d(5)
        phi3 = flows.advect_rk4(flows.abc_velocity, x3, 0.0, 2.0, 0.02).numpy()
        cases.append((3, x3, c3, phi3, 2.0, np.random.default_rng(17).standard_normal(x3.shape[0])))
    return cases


def check_adjoint_fd(w3=None, lib=None, h=1e-6, max_points=None):
    """Central differences of L = sum g_i FTLE_i, evaluated locally: moving phi_j
    changes FTLE only at j and at the points whose stencil holds j (for the
    symmetric RING1 stencil, j's own neighbours)."""
    for dim, x, cells, phi, T, g in _adjoint_cases(w3):
        n = x.shape[0]
        st = oracle.ring1(dim, n, cells, lib=lib)
        grad = oracle.ftle_grad(dim, x, phi, st, T, g, lib=lib)
        _, gap, _ = oracle.ftle(dim, x, phi, st, T, diagnostics=True, lib=lib)
        gmax = np.max(np.abs(grad))
        pts = range(n) if max_points is None else np.random.default_rng(0).choice(n, max_points, replace=False)
        checked = 0
        for j in pts:
            aff = np.concatenate([[j], st.col[st.row_ptr[j]:st.row_ptr[j + 1]]]).astype(np.int64)
            if np.any(gap[aff] < 1e-4):
                continue
            for c in range(dim):
                old = phi[j, c]
                phi[j, c] = old + h
                lp = np.dot(g[aff], oracle.ftle(dim, x, phi, st, T, sel=aff, lib=lib))
                phi[j, c] = old - h
                lm = np.dot(g[aff], oracle.ftle(dim, x, phi, st, T, sel=aff, lib=lib))
                phi[j, c] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - grad[j, c]) <= 1e-6 * gmax + 1e-5 * abs(grad[j, c]), \
                    (dim, j, c, fd, grad[j, c])
                checked += 1
        assert checked >= 0.9 * dim * len(pts)


def check_adjoint_identities(w3=None, lib=None):
    for dim, x, cells, phi, T, g in _adjoint_cases(w3):
        st = oracle.ring1(dim, x.shape[0], cells, lib=lib)
        grad = oracle.ftle_grad(dim, x, phi, st, T, g, lib=lib)
        f = oracle.ftle(dim, x, phi, st, T, lib=lib)
        fin = np.isfinite(f)
        scale = np.sum(np.abs(grad)) + 1.0
        assert np.max(np.abs(grad.sum(axis=0))) <= 1e-12 * scale
        lhs = np.sum(grad * phi)
        rhs = np.sum(g[fin]) / abs(T)
        assert abs(lhs - rhs) <= 1e-10 * (np.sum(np.abs(grad * phi)) + abs(rhs))
        S = grad.T @ phi
        assert np.max(np.abs(S - S.T)) <= 1e-10 * (np.sum(np.abs(grad) * np.abs(phi).sum(1, keepdims=True)) + 1)


ALL_BASIC = [check_ring1_bruteforce, check_eig3_vs_numpy, check_lstsq_fan, check_affine,
             check_rigid_and_scaling, check_axis_gradient]
