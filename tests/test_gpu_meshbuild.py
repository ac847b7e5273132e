"""The mesh built on the GPU (ftle_create_mesh_device) against the host build
and the oracle.

Integer work with one correct answer, so every comparison is exact: the
stencil mapped back to caller indices equals the oracle's one-ring stencil
(the neighbour determination of Section 2.2); the permutation, stencil, tile
metadata and record bytes equal those of ftle_create_mesh on the same
arguments; and since every later call reads only those, the FTLE of both
meshes agrees bit for bit (the 3D tape forward also reads the inverse normal
matrices, formed on each side in float64 without contraction)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2408_02758_amd as F
from paper_2408_02758_amd import _lib
from workloads import meshes

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _raw_tiles(m, adjoint=0):
    L = _lib.load()
    nt, rb = ctypes.c_int64(), ctypes.c_int64()
    _lib.check(L.ftle_mesh_get_tiles(m.handle, adjoint, ctypes.byref(nt), ctypes.byref(rb), None, None))
    meta = np.empty(nt.value * 16, np.uint8)
    rec = np.empty(max(rb.value, 16), np.uint8)
    _lib.check(L.ftle_mesh_get_tiles(m.handle, adjoint, None, None, meta.ctypes.data, rec.ctypes.data))
    return meta, rec[:rb.value]


def _device_mesh(x, cells, dtype, stencil="ring1", **kw):
    npdt = np.float64 if dtype == "f64" else np.float32
    xd = torch.as_tensor(np.ascontiguousarray(x, dtype=npdt), device=DEV)
    cd = torch.as_tensor(np.ascontiguousarray(cells, dtype=np.int32).reshape(-1, x.shape[1] + 1), device=DEV)
    return F.Mesh.on_device(xd, cd, stencil=stencil, **kw)


def _oracle_rows(dim, n, cells):
    st = oracle.ring1(dim, n, cells)
    return st.row_ptr, st.col


def _user_order_csr(m):
    """The mesh's stencil in caller indices, rows ascending (compare with the oracle's)."""
    rp, col, perm = m.csr()
    n = m.n
    lens = np.diff(rp.astype(np.int64))
    rows_user = np.repeat(perm.astype(np.int64), lens)
    cols_user = perm[col].astype(np.int64)
    order = np.lexsort((cols_user, rows_user))
    out_rp = np.zeros(n + 1, np.int64)
    np.add.at(out_rp, rows_user + 1, 1)
    return np.cumsum(out_rp), cols_user[order].astype(np.int32)


def same_bits(a, b):
    """Equal bit patterns (NaN where a point has no usable FTLE on both sides)."""
    it = torch.int64 if a.dtype == torch.float64 else torch.int32
    return a.shape == b.shape and torch.equal(a.contiguous().view(it), b.contiguous().view(it))


def _flow(x, seed):
    g = np.random.default_rng(seed)
    a = g.normal(size=(x.shape[1], x.shape[1])) * 0.3
    return x + np.sin(x @ a) * 0.05


def assert_same_mesh(x, cells, dtype="f32", tile_log2=0, reorder=True, check_oracle=True, T=2.0, stencil="ring1"):
    dim = x.shape[1]
    n = x.shape[0]
    print(f"[device mesh dim={dim} n={n} cells={len(cells)} {dtype} tile={tile_log2} reorder={reorder} "
          f"stencil={stencil}]", flush=True)
    host = F.Mesh(x, cells, dtype, tile_log2=tile_log2, reorder=reorder, stencil=stencil)
    dev = _device_mesh(x, cells, dtype, tile_log2=tile_log2, reorder=reorder, stencil=stencil)
    assert dev.info() == host.info()
    for name, a, b in zip(("row_ptr", "col", "perm"), dev.csr(), host.csr()):
        assert a.shape == b.shape and np.array_equal(a, b), \
            f"{name} differs at {np.flatnonzero(a != b)[:8] if a.shape == b.shape else a.shape}"
    assert dev.tile_stats() == host.tile_stats()
    for adjoint in (0, 1):
        dm, dr = _raw_tiles(dev, adjoint)
        hm, hr = _raw_tiles(host, adjoint)
        assert np.array_equal(dm, hm), f"tile metadata differs (adjoint={adjoint})"
        assert np.array_equal(dr, hr), f"tile record bytes differ (adjoint={adjoint})"
    if check_oracle:
        rp, col = _user_order_csr(dev)
        if stencil == "ring1":
            orp, ocol = _oracle_rows(dim, n, cells)
        else:
            xx = np.asarray(x, np.float32 if dtype == "f32" else np.float64).astype(np.float64)
            st = oracle.axis(dim, xx, oracle.ring1(dim, n, cells))
            sl = st.col.reshape(n, 2 * dim)
            keep = sl >= 0
            orp = np.concatenate([[0], np.cumsum(keep.sum(1))]).astype(np.int64)
            ocol = np.concatenate([np.sort(r[r >= 0]) for r in sl]).astype(np.int32) if n else np.zeros(0, np.int32)
        assert np.array_equal(rp, orp) and np.array_equal(col, ocol)
    # every later call reads the same data: bit-identical results
    tdt = torch.float64 if dtype == "f64" else torch.float32
    phi = torch.as_tensor(_flow(x, 11), dtype=tdt, device=DEV)
    assert same_bits(dev.forward(phi, T), host.forward(phi, T))
    g = torch.as_tensor(np.random.default_rng(7).normal(size=n), dtype=tdt, device=DEV)
    assert same_bits(dev.backward(phi, T, g), host.backward(phi, T, g))
    if dim == 3:
        a, _ = dev.forward_tape(phi, T)
        b, _ = host.forward_tape(phi, T)
        assert same_bits(a, b)
    return host, dev


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_tri_grid_row_order(dtype):
    # points numbered along grid rows: the caller-order axis is detected
    x, cells = meshes.jittered_tri_grid(97, 61, seed=3)
    assert_same_mesh(x, cells, dtype)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_tet_grid(dtype):
    x, cells = meshes.kuhn_tet_grid(13, nz=11)
    assert_same_mesh(x, cells, dtype)


@pytest.mark.parametrize("dim", [2, 3])
def test_shuffled_points(dim):
    x, cells = meshes.jittered_tri_grid(80, 50, seed=2) if dim == 2 else meshes.kuhn_tet_grid(12)
    xr, cr, _ = meshes.relabel(x, cells, seed=9)
    assert_same_mesh(xr, cr, "f32")


@pytest.mark.parametrize("tile_log2", [5, 8, 11])
def test_tile_sizes(tile_log2):
    # 2^11-point chunks exceed the 1024 staged slots: the extents halve them
    x, cells = meshes.kuhn_tet_grid(14)
    assert_same_mesh(x, cells, "f32", tile_log2=tile_log2)
    x, cells = meshes.jittered_tri_grid(70, 66, seed=4)
    assert_same_mesh(x, cells, "f32", tile_log2=tile_log2)


def test_no_reorder():
    x, cells = meshes.jittered_tri_grid(60, 45, seed=6)
    assert_same_mesh(x, cells, "f32", reorder=False)
    x, cells = meshes.kuhn_tet_grid(9)
    assert_same_mesh(x, cells, "f64", reorder=False)


@pytest.mark.parametrize("dim", [2, 3])
def test_delaunay_point_cloud(dim):
    """Irregular meshes: explicit rows, short runs, uneven degrees."""
    from scipy.spatial import Delaunay
    g = np.random.default_rng(40 + dim)
    n = 6000 if dim == 2 else 3000
    x = g.random((n, dim))
    cells = Delaunay(x).simplices.astype(np.int32)
    assert_same_mesh(x, cells, "f32")
    assert_same_mesh(x, cells, "f64", tile_log2=7)


def test_edge_cases():
    # one point, no cells
    x = np.array([[0.5, 0.25]])
    assert_same_mesh(x, np.zeros((0, 3), np.int32), check_oracle=False)
    # points in no cell, around a few cells; no cells at all
    x, cells = meshes.jittered_tri_grid(20, 20, seed=1)
    assert_same_mesh(x, cells[:7])
    assert_same_mesh(x, np.zeros((0, 3), np.int32), check_oracle=False)
    # under 64 points (no caller-order sample), and two points
    x, cells = meshes.jittered_tri_grid(6, 5, seed=2)
    assert_same_mesh(x, cells)
    assert_same_mesh(np.array([[0.0, 0.0, 0.0], [1.0, 0.5, 0.25]]), np.zeros((0, 4), np.int32), check_oracle=False)
    # all points on a line in one axis (zero spans elsewhere)
    x = np.stack([np.linspace(0, 1, 300), np.zeros(300)], axis=1)
    cells = np.array([[i, i + 1, i + 2] for i in range(298)], dtype=np.int32)
    assert_same_mesh(x, cells)


def test_duplicate_points_and_far_offset():
    """Equal Morton codes (every point twice, the copies in no cell, shuffled)
    keep the stable order on both builds; a mesh far from the origin (offset
    10^6, float64) quantises to the same codes on both."""
    x, cells = meshes.jittered_tri_grid(24, 17, seed=5)
    n = x.shape[0]
    perm = np.random.default_rng(7).permutation(2 * n)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(2 * n)
    xx = np.concatenate([x, x])[perm]
    assert_same_mesh(xx, inv[cells].astype(np.int32))
    x3, c3 = meshes.kuhn_tet_grid(7)
    assert_same_mesh(x3 + 1.0e6, c3, dtype="f64")
    assert_same_mesh(x3 + 1.0e6, c3, dtype="f64", stencil="axis")


def test_high_degree_fan():
    """A fan of triangles around one centre: a 900-neighbour row (tiles halve
    down to few points), then one past a tile's capacity (both builds refuse)."""
    for k, ok in ((900, True), (1100, False)):
        t = np.linspace(0, 2 * np.pi, k, endpoint=False)
        x = np.concatenate([[[0.0, 0.0]], np.stack([np.cos(t), np.sin(t)], 1)])
        cells = np.array([[0, 1 + i, 1 + (i + 1) % k] for i in range(k)], dtype=np.int32)
        if ok:
            assert_same_mesh(x, cells)
        else:
            with pytest.raises(F.FTLEError) as e:
                F.Mesh(x, cells, "f32")
            assert e.value.status == 4
            with pytest.raises(F.FTLEError) as e2:
                _device_mesh(x, cells, "f32")
            assert e2.value.status == 4 and "point 0 has 1100 neighbours" in str(e2.value)


def test_errors():
    x, cells = meshes.jittered_tri_grid(10, 8, seed=1)
    for bad, word in (([0, 1, 200], "out of range"), ([3, -2, 4], "out of range"), ([5, 6, 5], "repeated vertex")):
        c = cells.copy()
        c[11] = bad
        c[17] = bad
        with pytest.raises(F.FTLEError) as e:
            _device_mesh(x, c, "f32")
        assert e.value.status == 2 and word in str(e.value) and "cell 11" in str(e.value)
    xb = x.copy()
    xb[33, 1] = np.nan
    xb[40, 0] = np.inf
    with pytest.raises(F.FTLEError) as e:
        _device_mesh(xb, cells, "f64")
    assert e.value.status == 1 and "coordinate 33" in str(e.value)
    # a device-built mesh cannot be host-only
    L = _lib.load()
    xd = torch.as_tensor(x, dtype=torch.float32, device=DEV)
    cd = torch.as_tensor(cells, dtype=torch.int32, device=DEV)
    h = ctypes.c_void_p()
    st = L.ftle_create_mesh_device(2, x.shape[0], ctypes.c_void_p(xd.data_ptr()), _lib.F32, cells.shape[0],
                                   ctypes.c_void_p(cd.data_ptr()), _lib.HOST_ONLY, None, ctypes.byref(h))
    assert st == 4 and not h.value


def test_side_stream_and_adjoint():
    """Built on a side stream; the adjoint (which reuses the forward tiles of the
    symmetric one-ring stencil) agrees bit for bit too."""
    x, cells = meshes.kuhn_tet_grid(10)
    s = torch.cuda.Stream()
    xd = torch.as_tensor(x.astype(np.float32), device=DEV)
    cd = torch.as_tensor(cells.astype(np.int32), device=DEV)
    torch.cuda.synchronize()
    dev = F.Mesh.on_device(xd, cd, stream=s)
    host = F.Mesh(x, cells, "f32")
    phi = torch.as_tensor(_flow(x, 3), dtype=torch.float32, device=DEV)
    g = torch.as_tensor(np.random.default_rng(5).normal(size=x.shape[0]), dtype=torch.float32, device=DEV)
    assert same_bits(dev.backward(phi, 1.5, g), host.backward(phi, 1.5, g))


def test_full_size_2d_equals_host():
    """At the benchmark's 2048^2-point triangle grid: permutation, stencil
    and record bytes equal the host build's."""
    x, cells = meshes.jittered_tri_grid(2048, 2048, seed=2)
    print(f"[device mesh full 2D n={x.shape[0]}]", flush=True)
    host = F.Mesh(x, cells, "f32")
    dev = _device_mesh(x, cells, "f32")
    for a, b in zip(dev.csr(), host.csr()):
        assert np.array_equal(a, b)
    dm, dr = _raw_tiles(dev)
    hm, hr = _raw_tiles(host)
    assert np.array_equal(dm, hm) and np.array_equal(dr, hr)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_axis_stencil(dim, dtype):
    """The paper's axis stencil built on the device: slot order, repeats kept,
    its transpose for the adjoint tiles, all equal to the host build."""
    x, cells = meshes.jittered_tri_grid(71, 53, seed=8) if dim == 2 else meshes.kuhn_tet_grid(12, nz=10)
    assert_same_mesh(x, cells, dtype, stencil="axis")
    xr, cr, _ = meshes.relabel(x, cells, seed=4)
    assert_same_mesh(xr, cr, dtype, stencil="axis", tile_log2=7)


def test_axis_stencil_irregular():
    from scipy.spatial import Delaunay
    g = np.random.default_rng(12)
    for dim, n in ((2, 4000), (3, 2500)):
        x = g.random((n, dim))
        cells = Delaunay(x).simplices.astype(np.int32)
        assert_same_mesh(x, cells, "f32", stencil="axis")


def assert_same_csr_mesh(x, row_ptr, col, dtype="f32", tile_log2=0, reorder=True, T=2.0):
    """ftle_create_mesh_device_from_csr against ftle_create_mesh_from_csr on the
    same list: permutation, stencil, both tile sets byte for byte, forward and
    adjoint bit for bit."""
    n, dim = x.shape
    print(f"[device csr mesh dim={dim} n={n} nnz={len(col)} {dtype} tile={tile_log2}]", flush=True)
    host = F.Mesh.from_csr(x, row_ptr, col, dtype, tile_log2=tile_log2, reorder=reorder)
    npdt = np.float64 if dtype == "f64" else np.float32
    dev = F.Mesh.from_csr_on_device(torch.as_tensor(np.ascontiguousarray(x, dtype=npdt), device=DEV),
                                    torch.as_tensor(np.asarray(row_ptr, np.int64), device=DEV),
                                    torch.as_tensor(np.asarray(col, np.int32), device=DEV),
                                    tile_log2=tile_log2, reorder=reorder)
    assert dev.info() == host.info()
    for name, a, b in zip(("row_ptr", "col", "perm"), dev.csr(), host.csr()):
        assert a.shape == b.shape and np.array_equal(a, b), name
    for adjoint in (0, 1):
        dm, dr = _raw_tiles(dev, adjoint)
        hm, hr = _raw_tiles(host, adjoint)
        assert np.array_equal(dm, hm) and np.array_equal(dr, hr), f"tiles differ (adjoint={adjoint})"
    tdt = torch.float64 if dtype == "f64" else torch.float32
    phi = torch.as_tensor(_flow(x, 5), dtype=tdt, device=DEV)
    g = torch.as_tensor(np.random.default_rng(9).normal(size=n), dtype=tdt, device=DEV)
    assert same_bits(dev.forward(phi, T), host.forward(phi, T))
    assert same_bits(dev.backward(phi, T, g), host.backward(phi, T, g))
    return host, dev


@pytest.mark.parametrize("dim", [2, 3])
def test_from_csr_knn_with_repeats_self_and_absent(dim):
    """A non-symmetric k-nearest-neighbour list in shuffled caller order, with
    -1 entries, self entries and repeated entries planted."""
    from scipy.spatial import cKDTree
    x, _ = meshes.jittered_tri_grid(60, 41, seed=3) if dim == 2 else meshes.kuhn_tet_grid(11)
    k = 6 if dim == 2 else 10
    _, nb = cKDTree(x).query(x, k + 1)
    nb = np.ascontiguousarray(nb[:, 1:], dtype=np.int32)
    g = np.random.default_rng(dim)
    nb = g.permuted(nb, axis=1)
    rows = g.choice(x.shape[0], 200, replace=False)
    nb[rows[:80], 0] = -1
    nb[rows[80:140], 1] = rows[80:140]          # self
    nb[rows[140:], 2] = nb[rows[140:], 3]        # a repeat
    row_ptr = np.arange(x.shape[0] + 1, dtype=np.int64) * k
    assert_same_csr_mesh(x, row_ptr, nb.ravel(), "f32")
    assert_same_csr_mesh(x, row_ptr, nb.ravel(), "f64", tile_log2=6)


def test_from_csr_paper_list_and_ring1_output():
    """The paper's fixed-width list straight from ftle_axis_ell, and the one-ring
    CSR straight from ftle_ring1_csr, each into a device-built mesh."""
    x, cells = meshes.jittered_tri_grid(90, 70, seed=5)
    n = x.shape[0]
    xd = torch.as_tensor(x.astype(np.float32), device=DEV)
    rp, col = F.ring1_csr(2, n, torch.as_tensor(cells, dtype=torch.int32, device=DEV))
    ell = F.axis_ell(xd, rp, col)
    ell_rp = torch.arange(n + 1, dtype=torch.int64, device=DEV) * 4
    assert_same_csr_mesh(x, ell_rp.cpu().numpy(), ell.cpu().numpy().ravel(), "f32")
    dev = F.Mesh.from_csr_on_device(xd, ell_rp, ell.reshape(-1).contiguous())
    host = F.Mesh(x, cells, "f32", stencil="axis")
    phi = torch.as_tensor(_flow(x, 2), dtype=torch.float32, device=DEV)
    # the same neighbours as the axis mesh (its rows in slot order, these ascending): equal to rounding
    a, b = dev.forward(phi, 3.0).cpu().numpy(), host.forward(phi, 3.0).cpu().numpy()
    assert np.array_equal(np.isnan(a), np.isnan(b)) and np.nanmax(np.abs(a - b)) <= 1e-5
    assert_same_csr_mesh(x, rp.cpu().numpy(), col.cpu().numpy(), "f32")


def test_from_csr_errors():
    x, _ = meshes.jittered_tri_grid(10, 8, seed=1)
    n = x.shape[0]
    xd = torch.as_tensor(x.astype(np.float32), device=DEV)
    rp = np.arange(n + 1, dtype=np.int64) * 3
    col = np.tile(np.array([1, 2, 3], np.int32), n)

    def mk(r, c):
        return F.Mesh.from_csr_on_device(xd, torch.as_tensor(r, device=DEV), torch.as_tensor(c, device=DEV))

    bad = rp.copy()
    bad[0] = 1
    with pytest.raises(F.FTLEError) as e:
        mk(bad, col)
    assert e.value.status == 2 and "row_ptr[0]" in str(e.value)
    bad = rp.copy()
    bad[20], bad[30] = bad[22], bad[33]          # rows 20 and 30 decrease; the lowest is reported
    with pytest.raises(F.FTLEError) as e:
        mk(bad, col)
    assert e.value.status == 2 and "decreases at row 20" in str(e.value)
    c = col.copy()
    c[[50, 71]] = [n, -2]
    with pytest.raises(F.FTLEError) as e:
        mk(rp, c)
    assert e.value.status == 2 and "col[50]" in str(e.value)


def test_edge_cases_axis_and_lists():
    # the axis stencil of a mesh without cells, of one point, and of a tiny 3D mesh
    x, cells = meshes.jittered_tri_grid(9, 7, seed=3)
    assert_same_mesh(x, np.zeros((0, 3), np.int32), stencil="axis", check_oracle=False)
    assert_same_mesh(np.array([[0.25, 0.5]]), np.zeros((0, 3), np.int32), stencil="axis", check_oracle=False)
    x3, c3 = meshes.kuhn_tet_grid(3)
    assert_same_mesh(x3, c3, stencil="axis")
    # lists with no entries, and lists of -1 and self entries only
    n = x.shape[0]
    assert_same_csr_mesh(x, np.zeros(n + 1, np.int64), np.zeros(0, np.int32))
    rp = np.arange(n + 1, dtype=np.int64) * 2
    col = np.stack([np.full(n, -1), np.arange(n)], 1).astype(np.int32).ravel()
    assert_same_csr_mesh(x, rp, col)


def test_build_scratch_is_kept_and_released():
    """A device build keeps its scratch for the next one; the builds before and
    after a release give byte-identical meshes."""
    x, cells = meshes.kuhn_tet_grid(9)
    F.release_cached_memory()
    a = _device_mesh(x, cells, "f32")
    held = F.cached_memory_bytes()
    assert held > 0
    b = _device_mesh(x, cells, "f32")
    assert F.cached_memory_bytes() == held          # reused, not grown
    F.release_cached_memory()
    assert F.cached_memory_bytes() == 0
    c = _device_mesh(x, cells, "f32")
    for m in (b, c):
        for adjoint in (0, 1):
            ma, ra = _raw_tiles(a, adjoint)
            mm, rm = _raw_tiles(m, adjoint)
            assert np.array_equal(ma, mm) and np.array_equal(ra, rm)
