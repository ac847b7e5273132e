"""Seeded synthetic meshes for the FTLE workloads.

The paper evaluates on the inputs of UVaFTLE (Section 2.2, last paragraphs:
point coordinates plus the mesh faces of the original application), which are
not available.  These generators stand in for them with meshes of the same
kind: 2D triangulations and 3D tetrahedralisations of scattered points.

Nothing here computes any part of the FTLE method; the module only produces
coordinates (float64) and cell connectivity (int32).  It is shared by the
oracle-side tests and by the GPU-side tests and bench, and holds no stencil,
gradient, eigenvalue or logarithm arithmetic.
"""
from __future__ import annotations

import numpy as np


def jittered_tri_grid(nx: int, ny: int, seed: int, lx: float = 2.0, ly: float = 1.0,
                      jitter: float = 0.3):
    """Jittered nx-by-ny point grid on [0,lx]x[0,ly], triangulated.

    Points are cell-centred, x = (i + 1/2) hx + U(-jitter, jitter) hx with
    hx = lx/nx (same in y with hy = ly/ny).  User order is row-major with x
    fastest: index = j*nx + i.  The jitter is drawn as one array of shape
    (ny, nx, 2) from ``numpy.random.default_rng(seed)``.

    Each grid cell (i, j) .. (i+1, j+1) is split into two triangles along its
    shorter diagonal (measured on the jittered points); a tie goes to the
    p00-p11 diagonal.
    Returns (coords float64 (N,2), cells int32 (2*(nx-1)*(ny-1), 3)).
    """
    hx, hy = lx / nx, ly / ny
    rng = np.random.default_rng(seed)
    jit = rng.uniform(-jitter, jitter, size=(ny, nx, 2))
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    x = (ii + 0.5) * hx + jit[..., 0] * hx
    y = (jj + 0.5) * hy + jit[..., 1] * hy
    coords = np.stack([x.ravel(), y.ravel()], axis=1)

    ci, cj = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="xy")
    ci, cj = ci.ravel(), cj.ravel()
    p00 = cj * nx + ci
    p10 = p00 + 1
    p01 = p00 + nx
    p11 = p01 + 1
    d_main = np.sum((coords[p11] - coords[p00]) ** 2, axis=1)
    d_anti = np.sum((coords[p01] - coords[p10]) ** 2, axis=1)
    main = d_main <= d_anti
    t1 = np.where(main[:, None], np.stack([p00, p10, p11], 1), np.stack([p00, p10, p01], 1))
    t2 = np.where(main[:, None], np.stack([p00, p11, p01], 1), np.stack([p10, p11, p01], 1))
    cells = np.empty((2 * len(p00), 3), dtype=np.int32)
    cells[0::2] = t1
    cells[1::2] = t2
    return coords, cells


def regular_quad_points(nx: int, ny: int, lx: float = 2.0, ly: float = 1.0):
    """Unjittered cell-centred grid (same placement as jittered_tri_grid with zero jitter)."""
    hx, hy = lx / nx, ly / ny
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    return np.stack([((ii + 0.5) * hx).ravel(), ((jj + 0.5) * hy).ravel()], axis=1)


# The six axis permutations of the Kuhn (Freudenthal) split of a cube along its
# (0,0,0)->(1,1,1) diagonal: one tetrahedron per ordering of the unit steps.
_KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def kuhn_tet_grid(n: int, length: float = 2.0 * np.pi, nz: int | None = None,
                  ny: int | None = None):
    """Structured n^3 points on [0,length]^3 (inclusive ends, no periodic wrap).

    x_i = i * length / (n - 1).  User order: index = (k*ny + j)*nx + i.
    Each cube is split into 6 tetrahedra, one per permutation of the unit
    steps from corner (0,0,0) to corner (1,1,1); the split is conforming and
    gives interior vertices 14 mesh neighbours.
    Returns (coords float64 (N,3), cells int32 (6*(nx-1)*(ny-1)*(nz-1), 4)).
    """
    nx = n
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    h = length / (n - 1)
    kk, jj, ii = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    coords = np.stack([ii.ravel() * h, jj.ravel() * h, kk.ravel() * h], axis=1).astype(np.float64)

    ck, cj, ci = np.meshgrid(np.arange(nz - 1), np.arange(ny - 1), np.arange(nx - 1), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    strides = (1, nx, nx * ny)
    base = (ck * ny + cj) * nx + ci
    cells = np.empty((6 * len(base), 4), dtype=np.int32)
    for t, perm in enumerate(_KUHN_PERMS):
        v = base.copy()
        cells[t::6, 0] = v
        for s, axis in enumerate(perm):
            v = v + strides[axis]
            cells[t::6, s + 1] = v
    return coords, cells


def relabel(coords, cells, seed: int):
    """Random relabelling of points and shuffling of cells (and of vertex order in cells).

    Returns (coords', cells', p) with coords'[p[i]] = coords[i]: old point i is new point p[i].
    """
    rng = np.random.default_rng(seed)
    n = coords.shape[0]
    p = rng.permutation(n)
    new_coords = np.empty_like(coords)
    new_coords[p] = coords
    new_cells = p[cells].astype(np.int32)
    new_cells = new_cells[rng.permutation(new_cells.shape[0])]
    new_cells = np.take_along_axis(new_cells, rng.permuted(
        np.tile(np.arange(cells.shape[1]), (cells.shape[0], 1)), axis=1), axis=1)
    return new_coords, np.ascontiguousarray(new_cells, dtype=np.int32), p
