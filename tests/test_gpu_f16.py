"""Half-precision flow-map storage on the GPU (ftle_encode_flow_f16,
ftle_forward_f16) against the oracle: the encoding bit for bit, and the FTLE
of the decoded flow map x + d at the float32 tolerances of the full-precision
path (the kernel computes in float32 from the same decoded values)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2408_02758_amd as F
from paper_2408_02758_amd import _lib
from test_gpu_parity import _sample, check_f32
from workloads import configs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _case(w, sel=None, tile_log2=0):
    m = F.Mesh(w.coords, w.cells, "f32", tile_log2=tile_log2)
    flow = w.flow.to(DEV).float().contiguous()
    d = m.encode_flow_f16(flow)
    got = m.forward_f16(d, w.T).cpu().numpy().astype(np.float64)
    x32 = np.asarray(w.coords, dtype=np.float32)
    d_ref = oracle.encode_flow_f16(x32, w.flow_numpy().astype(np.float32))
    assert np.array_equal(d.cpu().numpy().view(np.uint16), d_ref.view(np.uint16)), "encodings differ"
    phi_dec = oracle.decode_flow_f16(x32, d_ref)
    st = oracle.ring1(2, w.n, w.cells)
    ref, gap, _ = oracle.ftle(2, x32.astype(np.float64), phi_dec.astype(np.float64), st, w.T, sel=sel,
                              diagnostics=True)
    # the same decoded map through the float32 forward: identical values in LDS
    plain = m.forward(torch.as_tensor(phi_dec, device=DEV), w.T).cpu().numpy().astype(np.float64)
    assert np.array_equal(got, plain, equal_nan=True)
    return got, ref, gap


@pytest.mark.parametrize("tile_log2", [0, 5])
def test_f16_flow_vs_oracle(tile_log2):
    w = configs.tri2d(200, 131, seed=2, t0=0.0, T=15.0, dtype="f32", device=DEV)
    got, ref, gap = _case(w, tile_log2=tile_log2)
    check_f32(f"f16 flow tri2d 200x131 tile={tile_log2}", got, ref, gap, w.T)


def test_f16_flow_2048_sampled():
    w = configs.scale_2d(DEV)
    sel = _sample(w.n, 20000, 12)
    got, ref, gap = _case(w, sel=sel)
    check_f32("f16 flow 2048^2 sampled", got[sel], ref, gap, w.T)


def test_f16_flow_2048_within_stated_bound():
    """Against the FTLE of the float32 flow map itself: at sampled points of the
    2048^2 map the binary16 storage's FTLE stays within the stated bound (the
    oracle's ftle_perturbation_bound for the storage error flow_error_f16)
    plus the float32 path's own tolerance, wherever that bound is finite."""
    w = configs.scale_2d(DEV)
    m = F.Mesh(w.coords, w.cells, "f32")
    flow = w.flow.to(DEV).float().contiguous()
    got = m.forward_f16(m.encode_flow_f16(flow), w.T).cpu().numpy().astype(np.float64)
    x32 = np.asarray(w.coords, dtype=np.float32)
    p32 = w.flow_numpy().astype(np.float32)
    st = oracle.ring1(2, w.n, w.cells)
    sel = _sample(w.n, 20000, 13)
    ref = oracle.ftle(2, x32.astype(np.float64), p32.astype(np.float64), st, w.T, sel=sel)
    bd = oracle.ftle_perturbation_bound(2, x32, p32, st, w.T, oracle.flow_error_f16(x32, p32), sel=sel)
    fin = np.isfinite(ref) & np.isfinite(bd)
    tol = 2e-5 / (2 * abs(w.T))
    diff = np.abs(got[sel] - ref)
    print(f"[f16 2048^2] bound finite at {fin.mean():.4f} of the sample, median {np.median(bd[fin]):.3e}, "
          f"max |diff| {diff[fin].max():.3e}, max diff/bound {(diff[fin] / (bd[fin] + tol)).max():.3f}", flush=True)
    assert np.all(diff[fin] <= bd[fin] + tol)
    assert fin.mean() > 0.5


def test_f16_flow_rejects_3d_and_f64():
    w3 = configs.abc_3d(DEV, n=6)
    m3 = F.Mesh(w3.coords, w3.cells, "f32")
    with pytest.raises(F.FTLEError) as e:
        m3.encode_flow_f16(w3.flow.to(DEV).float().contiguous())
    assert e.value.status == 4
    w = configs.small_2d(DEV)
    m = F.Mesh(w.coords, w.cells, "f64")
    d = torch.zeros(w.n, 2, dtype=torch.float16, device=DEV)
    out = torch.empty(w.n, dtype=torch.float32, device=DEV)
    st = _lib.load().ftle_forward_f16(m._h, ctypes.c_void_p(d.data_ptr()), w.T, ctypes.c_void_p(out.data_ptr()),
                                      None)
    assert st == 4   # FTLE_ERR_UNSUPPORTED
