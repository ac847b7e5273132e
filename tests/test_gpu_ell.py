"""The paper's fixed-width axis list (Section 2.2) as its own kernels, on the GPU:

* ftle_axis_ell builds the list from the device one-ring stencil: entry for
  entry equal to the oracle's list (oracle.axis), small meshes and the full
  2048^2 and 160^3 meshes;
* ftle_forward_ell (direct gathers, and staged through LDS blocks) against
  the oracle's FTLE on the oracle's list, element by element, float32 and
  float64, 2D and 3D, with ragged last blocks, absent slots and indices
  outside [0, n); the full-size workloads sampled.

Tolerances as in test_gpu_parity.py.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2408_02758_amd as F
from workloads import configs

from test_gpu_parity import DEV, check_f32, check_f64, _sample

pytestmark = pytest.mark.gpu


def _oracle_list(w):
    st = oracle.ring1(w.dim, w.n, w.cells)
    ax = oracle.axis(w.dim, w.coords.astype(np.float64), st)
    return st, ax


def _device_list(w, dtype=None):
    cells = torch.as_tensor(w.cells, dtype=torch.int32, device=DEV).contiguous()
    rp, col = F.ring1_csr(w.dim, w.n, cells)
    x = torch.as_tensor(w.coords, device=DEV).contiguous()
    return x, F.axis_ell(x, rp, col)


@pytest.mark.parametrize("dim,dtype", [(2, "f32"), (3, "f32"), (2, "f64"), (3, "f64")])
def test_axis_list_and_forward_vs_oracle(dim, dtype):
    w = (configs.tri2d(93, 71, seed=4, t0=1.0, T=8.0, dtype=dtype, device=DEV) if dim == 2
         else configs.abc3d(19, 6.0, dtype, DEV))
    st, ax = _oracle_list(w)
    x, ell = _device_list(w)
    assert np.array_equal(ell.cpu().numpy().ravel(), ax.col), "device list differs from the oracle's"
    ref, gap, _ = oracle.ftle(dim, w.coords.astype(np.float64), w.flow_numpy().astype(np.float64), ax, w.T,
                              diagnostics=True)
    fl = w.flow.to(DEV).contiguous()
    assert w.n % 256 != 0   # a ragged last block
    for staged in (False, True):
        got = F.forward_ell(x, ell, fl, w.T, staged=staged).cpu().numpy().astype(np.float64)
        tag = f"ell {dim}D {dtype} {'staged' if staged else 'direct'}"
        if dtype == "f64":
            check_f64(tag, got, ref, gap, w.T, dim)
        else:
            check_f32(tag, got, ref, gap, w.T)


def test_forward_ell_absent_and_out_of_range_slots():
    """Slots that are -1 or outside [0, n) are skipped; a point left with fewer
    than dim usable slots is NaN, as the oracle gives for its list with those
    slots set to -1."""
    w = configs.tri2d(40, 33, seed=7, t0=0.0, T=5.0, dtype="f32", device=DEV)
    _, ax = _oracle_list(w)
    lst = ax.col.reshape(w.n, 4).copy()
    rng = np.random.default_rng(3)
    hit = rng.choice(w.n, 300, replace=False)
    lst[hit, rng.integers(0, 4, 300)] = -1
    bad = rng.choice(w.n, 50, replace=False)
    lst[bad, 0] = w.n + 5            # outside [0, n): absent
    lst[bad[:10], 1] = -7
    iso = rng.choice(w.n, 5, replace=False)
    lst[iso] = -1                    # no neighbour at all
    clean = np.where((lst < 0) | (lst >= w.n), -1, lst).astype(np.int32)
    ref, _, detratio = oracle.ftle(2, w.coords.astype(np.float64), w.flow_numpy().astype(np.float64),
                                   oracle.Stencil(np.arange(w.n + 1, dtype=np.int64) * 4, clean.ravel()), w.T,
                                   diagnostics=True)
    assert np.isnan(ref[iso]).all()
    # the float32 rank test (det ratio 1e-5) and the oracle's (1e-12) differ in between
    clear = ~((detratio > 1e-12) & (detratio < 1e-4))
    x = torch.as_tensor(w.coords, device=DEV).contiguous()
    ell = torch.as_tensor(lst, dtype=torch.int32, device=DEV).contiguous()
    fl = w.flow.to(DEV).contiguous()
    for staged in (False, True):
        got = F.forward_ell(x, ell, fl, w.T, staged=staged).cpu().numpy().astype(np.float64)
        assert np.array_equal(np.isnan(got)[clear], np.isnan(ref)[clear])
        fin = np.isfinite(ref) & clear
        assert np.abs(2 * w.T * (got[fin] - ref[fin])).max() <= 2e-5


def test_forward_ell_tiny_and_empty():
    x = torch.tensor([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]], device=DEV)
    ell = torch.tensor([[-1, 1, -1, 2], [0, -1, -1, 2], [-1, 1, 0, -1]], dtype=torch.int32, device=DEV)
    phi = 3.0 * x
    for staged in (False, True):
        out = F.forward_ell(x, ell, phi, 2.0, staged=staged).cpu().numpy()
        assert np.allclose(out, np.log(3.0) / 2.0, rtol=1e-6)
    e = torch.empty(0, 2, device=DEV)
    assert F.forward_ell(e, torch.empty(0, 4, dtype=torch.int32, device=DEV), e, 1.0).numel() == 0
    # an output of the wrong size, dtype or device is refused before the launch
    for out in (torch.empty(2, device=DEV), torch.empty(3, dtype=torch.float64, device=DEV), torch.empty(3)):
        with pytest.raises(ValueError):
            F.forward_ell(x, ell, phi, 2.0, out=out)


@pytest.mark.parametrize("which", ["scale_2d", "abc_3d"])
def test_axis_list_full_size(which):
    """The bench's workloads: the device list equals the oracle's entry for
    entry; the direct and staged forwards (the bench's launches) match the
    oracle on sampled points and each other to rounding."""
    w = configs.scale_2d(DEV) if which == "scale_2d" else configs.abc_3d(DEV)
    st, ax = _oracle_list(w)
    x, ell = _device_list(w)
    assert np.array_equal(ell.cpu().numpy().ravel(), ax.col)
    fl = w.flow.to(DEV).contiguous()
    sel = _sample(w.n, 20000, 31)
    ref, gap, _ = oracle.ftle(w.dim, w.coords.astype(np.float64), w.flow_numpy().astype(np.float64), ax, w.T,
                              sel=sel, diagnostics=True)
    for staged in (False, True):
        got = F.forward_ell(x, ell, fl, w.T, staged=staged).cpu().numpy().astype(np.float64)
        check_f32(f"ell {which} {'staged' if staged else 'direct'} sampled", got[sel], ref, gap, w.T)
