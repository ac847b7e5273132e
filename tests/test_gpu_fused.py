"""ftle_forward_backward: FTLE and its adjoint in one persistent launch (the
forward tiles publish their tape per tile, the adjoint tiles wait for the
tiles they depend on), against the two-launch path (ftle_forward_tape then
ftle_backward_tape, itself checked against the oracle in test_gpu_parity.py)
bit for bit, and against the oracle directly on a small case.  Every case
also checks that no dependency wait ran out of its bound."""
import numpy as np
import pytest
import torch

import oracle
import paper_2408_02758_amd as F
from workloads import configs

from test_gpu_parity import DEV, _grad_case, check_f32

pytestmark = pytest.mark.gpu


def _same(a, b):
    return torch.equal(torch.nan_to_num(a, nan=7.0), torch.nan_to_num(b, nan=7.0))


def _two_launch(m, fl, T, g):
    out, tape = m.forward_tape(fl, T)
    return out, m.backward_tape(tape, g)


def _check_mesh(m, fl, T, seed, one_launch=True, reps=3):
    gs = [torch.as_tensor(np.random.default_rng(seed + r).standard_normal(m.n), dtype=fl.dtype, device=DEV)
          for r in range(reps)]
    Ts = [T * (1.0 + 0.25 * r) * (-1) ** r for r in range(reps)]
    # back to back: each launch reuses the queue counters and flags of the previous one
    got = [m.forward_backward(fl, Ts[r], gs[r]) for r in range(reps)]
    torch.cuda.synchronize()
    for r in range(reps):
        ref = _two_launch(m, fl, Ts[r], gs[r])
        assert _same(got[r][0], ref[0]), f"FTLE differs (rep {r})"
        assert _same(got[r][1], ref[1]), f"gradient differs (rep {r})"
    # on a second stream, then on the current one
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        a = m.forward_backward(fl, Ts[0], gs[1])
    b = m.forward_backward(fl, Ts[1], gs[0])
    torch.cuda.synchronize()
    assert _same(a[1], _two_launch(m, fl, Ts[0], gs[1])[1])
    assert _same(b[1], _two_launch(m, fl, Ts[1], gs[0])[1])
    info = m.fused_info()
    print(f"fused n={m.n}: {info}", flush=True)
    assert info["one_launch"] == one_launch and info["late_waits"] == 0
    if one_launch:
        assert info["grid"] > 0


@pytest.mark.parametrize("dim,dtype", [(2, "f32"), (2, "f64"), (3, "f32"), (3, "f64")])
@pytest.mark.parametrize("tile_log2", [0, 6])
def test_fused_matches_two_launches(dim, dtype, tile_log2):
    x, cells, phi, T = _grad_case(dim, dtype)
    m = F.Mesh(x, cells, dtype, tile_log2=tile_log2)
    _check_mesh(m, phi, T, 10 * dim + tile_log2)


def test_fused_relabelled_and_block_sizes():
    from workloads import meshes
    x0, c0, phi0, T = _grad_case(3, "f32", 14)
    x, cells, p = meshes.relabel(x0, c0, seed=5)
    phi = torch.empty_like(phi0)
    phi[torch.as_tensor(p, device=DEV)] = phi0
    for blocks in ((128, 128), (256, 256), (512, 512)):
        m = F.Mesh(x.astype(np.float32), cells, "f32")
        m.set_blocks(*blocks)
        _check_mesh(m, phi, T, 3, reps=2)


def test_fused_falls_back_for_non_symmetric_stencils():
    """The axis stencil from cells is not symmetric (j being i's nearest
    neighbour along +x does not make i j's along -x): two launches, the same
    results."""
    x, cells, phi, T = _grad_case(2, "f32")
    m = F.Mesh(x, cells, "f32", stencil="axis")
    _check_mesh(m, phi, T, 4, one_launch=False, reps=2)


def test_fused_vs_oracle_small():
    x, cells, phi, T = _grad_case(3, "f32", 12)
    m = F.Mesh(x, cells, "f32")
    g = np.random.default_rng(2).standard_normal(m.n)
    out, grad = m.forward_backward(phi, T, torch.as_tensor(g, dtype=torch.float32, device=DEV))
    st = oracle.ring1(3, m.n, cells)
    xd, pd = x.astype(np.float64), phi.cpu().numpy().astype(np.float64)
    ref, gap, _ = oracle.ftle(3, xd, pd, st, T, diagnostics=True)
    check_f32("fused 12^3 FTLE", out.cpu().numpy().astype(np.float64), ref, gap, T)
    gref = oracle.ftle_grad(3, xd, pd, st, T, g.astype(np.float32).astype(np.float64))
    bad = np.zeros(m.n, bool)
    for i in np.nonzero(np.isfinite(gap) & ~(gap >= 1e-6))[0]:
        bad[i] = True
        bad[st.col[st.row_ptr[i]:st.row_ptr[i + 1]]] = True
    err = np.abs(grad.cpu().numpy() - gref)[~bad].max() / np.abs(gref).max()
    print(f"fused 12^3 adjoint max err/scale = {err:.3e}", flush=True)
    assert err <= 2e-4


def test_fused_diff_96():
    """The measured workload: 96^3 ABC, float32, weights w ~ N(0, 1)."""
    w = configs.diff_3d(DEV)
    m = F.Mesh(w.coords, w.cells, "f32")
    fl = w.flow.to(DEV).contiguous()
    _check_mesh(m, fl, w.T, 5, reps=2)
