"""FTLE oracle -- TEST INFRASTRUCTURE ONLY.

Python face of ``ftle_oracle.c``: a plain double-precision CPU implementation
of the per-point FTLE computation (least-squares flow-map gradient over the
mesh neighbours, Cauchy-Green tensor, largest eigenvalue, ln sqrt(lambda)/|T|)
and of its adjoint.  It exists to check the GPU library; only the tests, the
smoke check and the benchmark's CPU-baseline leg may import it.  It shares no
code with the GPU library and does not import it.

It also holds the two steps around the path that the library offers on the
GPU: RK4 flow maps (of analytic flows, and in a velocity field sampled on a
regular grid, multilinear in space and linear in time), and the binary16
storage of a flow map
(numpy), with the error bound that storage carries: the storage's rounding
per point (flow_error_f16) and the FTLE change any flow-map error within given
per-point limits can cause (ftle_perturbation_bound, from the least squares'
linearity in phi and Weyl's inequality).  What pins each function is in the
test modules
``tests/test_oracle_pins.py``, ``tests/test_oracle_advect.py`` and
``tests/test_oracle_f16.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ftle_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def compile_source(src: str, out: str) -> str:
    """gcc -O2, OpenMP, no FMA contraction; writes the shared library atomically."""
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                           "-fPIC", "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    """Compile the oracle library next to its source."""
    if force or not os.path.exists(_LIB):
        compile_source(_SRC, _LIB)
    return _LIB


def source_path() -> str:
    return _SRC


class _Lib:
    """ctypes bindings of one compiled oracle library."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        i64, vp = ctypes.c_int64, ctypes.c_void_p
        lib.oracle_ring1_bound.restype = i64
        lib.oracle_ring1_bound.argtypes = [ctypes.c_int, i64]
        lib.oracle_ring1.restype = i64
        lib.oracle_ring1.argtypes = [ctypes.c_int, i64, i64, vp, vp, vp]
        lib.oracle_axis.restype = None
        lib.oracle_axis.argtypes = [ctypes.c_int, i64, vp, vp, vp, vp]
        lib.oracle_ftle.restype = None
        lib.oracle_ftle.argtypes = [ctypes.c_int, i64, vp, vp, vp, vp, ctypes.c_double,
                                    i64, vp, vp, vp, vp]
        lib.oracle_ftle_grad.restype = None
        lib.oracle_ftle_grad.argtypes = [ctypes.c_int, i64, vp, vp, vp, vp, ctypes.c_double,
                                         vp, vp]
        lib.oracle_advect_rk4.restype = None
        lib.oracle_advect_rk4.argtypes = [ctypes.c_int, vp, i64, vp, vp, vp, ctypes.c_double, vp]
        lib.oracle_advect_rk4_grid.restype = None
        lib.oracle_advect_rk4_grid.argtypes = [ctypes.c_int, vp, vp, vp, i64, ctypes.c_double, ctypes.c_double, vp,
                                               i64, vp, vp, vp, ctypes.c_double, vp]
        lib.oracle_jacobi_eig3.restype = None
        lib.oracle_jacobi_eig3.argtypes = [vp, vp, vp]
        lib.oracle_set_threads.restype = None
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_max_threads.argtypes = []
        self.c = lib
        self.path = path


def load_library(path: str):
    """Load another build of the oracle (used by the tests that plant mistakes)."""
    return _Lib(path)


def _load(lib=None):
    global _lib
    if lib is not None:
        return lib.c
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _Lib(_LIB)
    return _lib.c


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


class Stencil:
    """CSR stencil in the caller's point order: row_ptr (n+1, int64), col (nnz, int32).

    Entries equal to -1 stand for an absent neighbour and are skipped.
    """

    def __init__(self, row_ptr, col):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col = np.ascontiguousarray(col, dtype=np.int32)

    @property
    def n(self):
        return self.row_ptr.shape[0] - 1

    @property
    def nnz(self):
        return int(self.row_ptr[-1])


def ring1(dim: int, n: int, cells, lib=None) -> Stencil:
    """Every vertex sharing a cell with i (excluding i), deduplicated, ascending."""
    lib = _load(lib)
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    ncells = cells.shape[0]
    assert cells.shape[1] == dim + 1
    cap = int(lib.oracle_ring1_bound(dim, ncells))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(max(cap, 1), dtype=np.int32)
    nnz = lib.oracle_ring1(dim, n, ncells, _p(cells), _p(row_ptr), _p(col))
    if nnz < 0:
        raise ValueError("cell references a point outside [0, n)")
    return Stencil(row_ptr, col[:nnz].copy())


def axis(dim: int, coords, st: Stencil, lib=None) -> Stencil:
    """The paper's fixed-width list: 2*dim slots per point, -1 where absent."""
    lib = _load(lib)
    x = _f64(coords)
    n = x.shape[0]
    slots = np.full(n * 2 * dim, -1, dtype=np.int32)
    lib.oracle_axis(dim, n, _p(x), _p(st.row_ptr), _p(st.col), _p(slots))
    return Stencil(np.arange(n + 1, dtype=np.int64) * 2 * dim, slots)


def ftle(dim: int, coords, flow, st: Stencil, T: float, sel=None, diagnostics: bool = False, lib=None):
    """FTLE per point (float64).  sel: optional point indices to evaluate.

    With diagnostics=True also returns (gap, detratio): the relative gap
    (lam1 - lam2)/lam1 of C's top eigenvalue and det M / (tr M / D)^D.
    """
    lib = _load(lib)
    x, f = _f64(coords), _f64(flow)
    n = x.shape[0]
    assert x.shape == (n, dim) and f.shape == (n, dim) and st.n == n
    if sel is None:
        cnt, selp = n, None
    else:
        sel = np.ascontiguousarray(sel, dtype=np.int64)
        cnt, selp = sel.shape[0], _p(sel)
    out = np.empty(cnt, dtype=np.float64)
    gap = np.empty(cnt, dtype=np.float64) if diagnostics else None
    det = np.empty(cnt, dtype=np.float64) if diagnostics else None
    lib.oracle_ftle(dim, n, _p(x), _p(f), _p(st.row_ptr), _p(st.col), float(T),
                    cnt, selp, _p(out), _p(gap) if diagnostics else None,
                    _p(det) if diagnostics else None)
    if diagnostics:
        return out, gap, det
    return out


def ftle_grad(dim: int, coords, flow, st: Stencil, T: float, g, lib=None):
    """dL/dflow (n x dim, float64) for L = sum_i g_i FTLE_i."""
    lib = _load(lib)
    x, f, gg = _f64(coords), _f64(flow), _f64(g)
    n = x.shape[0]
    grad = np.empty((n, dim), dtype=np.float64)
    lib.oracle_ftle_grad(dim, n, _p(x), _p(f), _p(st.row_ptr), _p(st.col), float(T),
                         _p(gg), _p(grad))
    return grad


def jacobi_eig3(m, lib=None):
    """Eigenvalues (ascending) and unit eigenvectors (columns) of a symmetric 3x3."""
    lib = _load(lib)
    m = _f64(m).reshape(3, 3)
    vals = np.empty(3)
    vecs = np.empty((3, 3))
    lib.oracle_jacobi_eig3(_p(m), _p(vals), _p(vecs))
    return vals, vecs


FLOWS = {"double_gyre": (0, 2, (0.1, 0.25, 2.0 * np.pi / 10.0)),
         "abc": (1, 3, (np.sqrt(3.0), np.sqrt(2.0), 1.0))}


def advect_rk4(flow: str, x0, t0, T, dt: float, params=None, lib=None):
    """Flow map x(t0 + T) of the analytic flow ("double_gyre": params A, eps,
    omega; "abc": params A, B, C) by classical RK4 in float64: per point
    max(1, ceil(|T|/dt - 1e-9)) steps of T/steps.  t0 and T: scalars or per-point
    arrays."""
    lib = _load(lib)
    kind, dim, default = FLOWS[flow]
    prm = _f64(default if params is None else params)
    x = _f64(x0).reshape(-1, dim)
    n = x.shape[0]
    t0a = _f64(np.broadcast_to(np.asarray(t0, dtype=np.float64), (n,)))
    Ta = _f64(np.broadcast_to(np.asarray(T, dtype=np.float64), (n,)))
    out = np.empty_like(x)
    lib.oracle_advect_rk4(kind, _p(prm), n, _p(x), _p(t0a), _p(Ta), float(dt), _p(out))
    return out


def advect_rk4_grid(vel, origin, spacing, t_first, t_step, x0, t0, T, dt: float, lib=None):
    """advect_rk4 in a velocity field sampled on a regular grid: vel of shape
    (n_times, [nz,] ny, nx, dim) holds the velocity at node origin + index *
    spacing (x fastest) and time t_first + k * t_step; multilinear in space,
    linear in time, the nearest point of the grid's box (and the nearest
    slice) outside it."""
    lib = _load(lib)
    v = _f64(vel)
    dim = v.shape[-1]
    nt = v.shape[0]
    shape = np.ascontiguousarray(v.shape[1:-1][::-1], dtype=np.int64)   # nx, ny[, nz]
    assert shape.size == dim and np.all(shape >= 2)
    x = _f64(x0).reshape(-1, dim)
    n = x.shape[0]
    t0a = _f64(np.broadcast_to(np.asarray(t0, dtype=np.float64), (n,)))
    Ta = _f64(np.broadcast_to(np.asarray(T, dtype=np.float64), (n,)))
    out = np.empty_like(x)
    lib.oracle_advect_rk4_grid(dim, _p(shape), _p(_f64(origin)), _p(_f64(spacing)), nt, float(t_first),
                               float(t_step), _p(v), n, _p(x), _p(t0a), _p(Ta), float(dt), _p(out))
    return out


def encode_flow_f16(coords, flow):
    """Half-precision flow-map storage (the paper's precision-for-speed trade,
    Section 1.1): the displacement phi - x taken in float32, then rounded to
    binary16, each step to nearest even (IEEE 754; numpy's float32 arithmetic
    and float32 -> float16 conversion)."""
    x32 = np.asarray(coords, dtype=np.float32)
    p32 = np.asarray(flow, dtype=np.float32)
    with np.errstate(over="ignore"):
        return (p32 - x32).astype(np.float16)


def decode_flow_f16(coords, delta):
    """The flow map the stored displacements stand for: x + d in float32 (one
    rounding), d widened exactly from binary16."""
    return np.asarray(coords, dtype=np.float32) + np.asarray(delta, dtype=np.float16).astype(np.float32)


def flow_error_f16(coords, flow):
    """Per point, a bound on max_k |phi'_k - phi_k| for the binary16 storage
    above (the precision-for-bandwidth trade of Section 1.1),
    phi' = decode_flow_f16(coords, encode_flow_f16(coords, flow)), with
    coords and flow the float32 values stored: the float32 difference
    (<= 2^-24 |phi - x|), its rounding to binary16 (<= 2^-11 of its magnitude
    in the normal range, <= 2^-25 in the subnormal range) and the float32 sum
    x + d (<= 2^-24 |x + d|).  inf where the displacement overflows binary16."""
    x = np.asarray(coords, dtype=np.float32).astype(np.float64)
    p = np.asarray(flow, dtype=np.float32).astype(np.float64)
    a = np.abs(p - x)
    e1 = 2.0 ** -24 * a
    e2 = np.maximum(2.0 ** -11 * (a + e1), 2.0 ** -25)
    e3 = 2.0 ** -24 * (np.abs(p) + e1 + e2)
    e = e1 + e2 + e3
    e[a + e1 > 65504.0] = np.inf
    return e.max(axis=1)


def ftle_perturbation_bound(dim: int, coords, flow, st: Stencil, T: float, delta, sel=None):
    """For each point i, a bound on |FTLE_i(phi') - FTLE_i(phi)| over every
    flow map phi' with max_k |phi'_jk - phi_jk| <= delta_j at each point j
    (numpy, float64).  In the least squares of ftle(), J = B M^-1 and phi'
    changes B by sum_j (e_j - e_i)(x_j - x_i)^T, hence J by sum_j (e_j - e_i)
    w_j^T with w_j = M^-1 (x_j - x_i); its Frobenius norm is at most
    eps_i = sum_j sqrt(D) (delta_j + delta_i) |w_j|.  The largest singular value
    of J moves by at most eps_i (Weyl's inequality), so FTLE = ln(sigma_max)/|T|
    moves by at most -ln(1 - eps_i / sigma_max) / |T| while eps_i < sigma_max,
    and without bound beyond.  NaN where ftle() gives NaN for the stencil
    (det M <= 1e-12 (tr M / D)^D).  sel: optional point indices (the result
    then holds only those points)."""
    x = _f64(coords).reshape(-1, dim)
    p = _f64(flow).reshape(-1, dim)
    delta = np.asarray(delta, dtype=np.float64)
    pts = np.arange(x.shape[0]) if sel is None else np.asarray(sel, dtype=np.int64)
    n = pts.shape[0]
    lens = st.row_ptr[pts + 1] - st.row_ptr[pts]
    rows = np.repeat(np.arange(n), lens)                      # local row of each entry
    starts = np.repeat(st.row_ptr[pts] - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
    cols = st.col[np.arange(rows.shape[0]) + starts].astype(np.int64)
    keep = cols >= 0
    rows, cols = rows[keep], cols[keep]
    owner = pts[rows]                                         # global index of each entry's point
    dx = x[cols] - x[owner]
    dp = p[cols] - p[owner]
    M = np.empty((n, dim, dim))
    B = np.empty((n, dim, dim))
    for a in range(dim):
        for b in range(dim):
            M[:, a, b] = np.bincount(rows, weights=dx[:, a] * dx[:, b], minlength=n)
            B[:, a, b] = np.bincount(rows, weights=dp[:, a] * dx[:, b], minlength=n)
    tr = np.trace(M, axis1=1, axis2=2) / dim
    ok = np.linalg.det(M) > 1e-12 * tr ** dim
    Msafe = np.where(ok[:, None, None], M, np.eye(dim))
    Minv = np.linalg.inv(Msafe)
    sigma = np.linalg.svd(B @ Minv, compute_uv=False)[:, 0]
    w = np.einsum("nab,nb->na", Minv[rows], dx)
    eps = np.sqrt(dim) * np.bincount(rows, weights=(delta[cols] + delta[owner]) * np.linalg.norm(w, axis=1),
                                     minlength=n)
    with np.errstate(divide="ignore", invalid="ignore"):
        out = np.where(eps < sigma, -np.log1p(-eps / sigma) / abs(T), np.inf)
    out[eps == 0] = 0.0
    out[~ok] = np.nan
    return out
