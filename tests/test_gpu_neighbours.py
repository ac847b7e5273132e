"""The one-ring stencil built on the GPU (ftle_ring1_csr) against the oracle's
host construction, bit for bit: integer work, one correct answer (each row's
neighbours ascending, once each)."""
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


def device_ring1(dim, n, cells):
    c = torch.as_tensor(np.ascontiguousarray(cells, dtype=np.int32), device=DEV)
    row_ptr, col = F.ring1_csr(dim, n, c)
    return row_ptr.cpu().numpy(), col.cpu().numpy()


def assert_same(dim, n, cells):
    rp, col = device_ring1(dim, n, cells)
    ref = oracle.ring1(dim, n, cells)
    assert rp.dtype == np.int64 and col.dtype == np.int32
    assert np.array_equal(rp, ref.row_ptr)
    assert np.array_equal(col, ref.col)
    return rp, col


@pytest.mark.parametrize("dim", [2, 3])
def test_ring1_csr_vs_oracle(dim):
    if dim == 2:
        x, cells = meshes.jittered_tri_grid(64, 48, seed=3)
    else:
        x, cells = meshes.kuhn_tet_grid(10)
    print(f"[ring1_csr dim={dim} n={x.shape[0]} cells={cells.shape[0]}]", flush=True)
    assert_same(dim, x.shape[0], cells)


def test_ring1_csr_edge_cases():
    # points in no cell (at the start, between and after the used ones), a cell
    # with a repeated point, a single cell, and no cells at all
    cells = np.array([[2, 3, 5], [3, 5, 9], [5, 5, 7]], dtype=np.int32)
    rp, _ = assert_same(2, 12, cells)
    assert rp[1] == 0 and rp[12] == rp[11]
    assert_same(3, 5, np.array([[4, 0, 2, 1]], dtype=np.int32))
    rp, col = device_ring1(2, 7, np.zeros((0, 3), dtype=np.int32))
    assert np.array_equal(rp, np.zeros(8, dtype=np.int64)) and col.size == 0
    # a cell index outside [0, n) is reported, not used
    for bad in ([0, 1, 6], [0, -1, 2]):
        with pytest.raises(F.FTLEError) as e:
            device_ring1(2, 6, np.array([[0, 1, 2], bad], dtype=np.int32))
        assert e.value.status == 2   # FTLE_ERR_BAD_MESH


def test_ring1_csr_capacity_reported():
    """Through the C ABI: too small a col_capacity fails with the count needed."""
    x, cells = meshes.jittered_tri_grid(6, 5, seed=1)
    n = x.shape[0]
    ref = oracle.ring1(2, n, cells)
    c = torch.as_tensor(cells, dtype=torch.int32, device=DEV)
    rp = torch.empty(n + 1, dtype=torch.int64, device=DEV)
    col = torch.empty(ref.col.size, dtype=torch.int32, device=DEV)
    nnz = ctypes.c_int64(-1)
    lib = _lib.load()
    st = lib.ftle_ring1_csr(2, n, cells.shape[0], ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(rp.data_ptr()),
                            ctypes.c_void_p(col.data_ptr()), ref.col.size - 1, ctypes.byref(nnz), None)
    assert st == 4 and nnz.value == ref.col.size   # FTLE_ERR_UNSUPPORTED
    st = lib.ftle_ring1_csr(2, n, cells.shape[0], ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(rp.data_ptr()),
                            ctypes.c_void_p(col.data_ptr()), ref.col.size, ctypes.byref(nnz), None)
    assert st == 0 and nnz.value == ref.col.size
    assert np.array_equal(rp.cpu().numpy(), ref.row_ptr) and np.array_equal(col.cpu().numpy(), ref.col)


@pytest.mark.parametrize("dim", [2, 3])
def test_ring1_csr_full_size(dim):
    """The measured workloads' meshes: 2048^2 triangles, 160^3 Kuhn tetrahedra."""
    if dim == 2:
        x, cells = meshes.jittered_tri_grid(2048, 2048, seed=7)
    else:
        x, cells = meshes.kuhn_tet_grid(160)
    print(f"[ring1_csr full dim={dim} n={x.shape[0]} cells={cells.shape[0]}]", flush=True)
    assert_same(dim, x.shape[0], cells)


def test_mesh_from_device_stencil_matches_cells():
    """A mesh built from the device stencil gives the same FTLE, bit for bit,
    as the mesh the host builds from the cells."""
    x, cells = meshes.jittered_tri_grid(40, 30, seed=5)
    rp, col = device_ring1(2, x.shape[0], cells)
    m_cells = F.Mesh(x, cells, "f32")
    m_csr = F.Mesh.from_csr(x, rp, col, "f32")
    phi = torch.as_tensor(x * 1.7 + 0.1 * np.sin(3 * x), dtype=torch.float32, device=DEV)
    a = m_cells.forward(phi, 2.0).cpu().numpy()
    b = m_csr.forward(phi, 2.0).cpu().numpy()
    assert np.array_equal(a, b, equal_nan=True)


def test_ring1_csr_long_rows_and_workspace():
    """Points with more distinct neighbours than a lane keeps in LDS go to the
    long-row path: a fan of 70 triangles around one point (70 neighbours), and
    a point shared by 300 triangles of a star (600 candidates); with a
    caller-held workspace, and with cells that are not 16-byte aligned."""
    k = 70
    fan = np.array([[0, 1 + i, 1 + (i + 1) % k] for i in range(k)], dtype=np.int32)
    rp, col = assert_same(2, k + 1, fan)
    assert rp[1] - rp[0] == k
    m = 300
    star = np.array([[0, 1 + 2 * i, 2 + 2 * i] for i in range(m)], dtype=np.int32)
    x, grid = meshes.jittered_tri_grid(30, 20, seed=2)
    cells = np.concatenate([star, grid + 2 * m + 1]).astype(np.int32)
    n = 2 * m + 1 + x.shape[0]
    assert_same(2, n, cells)
    c = torch.as_tensor(cells, device=DEV)
    ws = torch.empty(F.ring1_workspace_bytes(2, n, cells.shape[0]), dtype=torch.uint8, device=DEV)
    ref = oracle.ring1(2, n, cells)
    for _ in range(2):   # the workspace is reused as it is left
        rp2, col2 = F.ring1_csr(2, n, c, workspace=ws)
        assert np.array_equal(rp2.cpu().numpy(), ref.row_ptr) and np.array_equal(col2.cpu().numpy(), ref.col)
    with pytest.raises(F.FTLEError):
        F.ring1_csr(2, n, c, workspace=ws[:100])
    # 3D cells at a 4-byte offset
    xt, tets = meshes.kuhn_tet_grid(7)
    flat = torch.empty(tets.size + 1, dtype=torch.int32, device=DEV)
    flat[1:] = torch.as_tensor(tets.ravel(), device=DEV)
    shifted = flat[1:].view(-1, 4)
    assert shifted.data_ptr() % 16 != 0
    rp3, col3 = F.ring1_csr(3, xt.shape[0], shifted)
    ref3 = oracle.ring1(3, xt.shape[0], tets)
    assert np.array_equal(rp3.cpu().numpy(), ref3.row_ptr) and np.array_equal(col3.cpu().numpy(), ref3.col)


def test_ring1_csr_too_long_a_row_is_unsupported():
    """A point in 2100 triangles (4200 candidate entries, over the 4096 a
    long-row workgroup sorts) is reported, not truncated."""
    m = 2100
    star = np.array([[0, 1 + 2 * i, 2 + 2 * i] for i in range(m)], dtype=np.int32)
    with pytest.raises(F.FTLEError) as e:
        device_ring1(2, 2 * m + 1, star)
    assert e.value.status == 4 and "4096" in e.value.message
