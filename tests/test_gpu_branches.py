"""GPU code paths that the default launches take rarely or not at all, each
checked against the FP64 oracle or against the path it must reproduce:

* the float64 recompute of the 3D float32 eigenvalue (taken where the two
  largest eigenvalues of C nearly coincide): forced on every point through the
  run-time threshold, and reached with the default threshold on a flow map
  built to be nearly degenerate;
* every launch form of the batched kernel (the flat grid and the persistent
  grid draining the atomic queue with 1, 2, 4 and 8 tiles per pop), pinned
  instead of autotuned, replayed back to back and across two streams;
* the float64 forward at the measured sizes (2048^2 and 96^3), sampled.

Tolerances as in test_gpu_parity.py.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2408_02758_amd as F
from workloads import configs, meshes

from test_gpu_parity import DEV, check_f32, check_f64, ref_ftle, _sample

pytestmark = pytest.mark.gpu


@pytest.fixture
def default_threshold():
    yield
    F.set_eig_threshold(-1.0)


def _grad_ref(w, g, st):
    xd, pd = w.coords.astype(np.float64), w.flow_numpy().astype(np.float64)
    ref = oracle.ftle_grad(w.dim, xd, pd, st, w.T, g.astype(np.float64))
    _, gap, _ = oracle.ftle(w.dim, xd, pd, st, w.T, diagnostics=True)
    bad = np.zeros(w.n, bool)
    for i in np.nonzero(np.isfinite(gap) & ~(gap >= 1e-6))[0]:
        bad[i] = True
        bad[st.col[st.row_ptr[i]:st.row_ptr[i + 1]]] = True
    return ref, bad


def test_fp64_eigen_branch_forced_everywhere(default_threshold):
    """Every point of a 3D float32 mesh through the float64 recompute (a
    threshold above 2 admits every r in [-1, 1]): forward, tape forward,
    adjoint and batched against the oracle, with the hit count equal to the
    points that have a usable stencil."""
    w = configs.abc3d(21, 10.0, "f32", DEV)
    m = F.Mesh(w.coords, w.cells, "f32")
    fl = w.flow.to(DEV).contiguous()
    ref, gap, st = ref_ftle(w)
    usable = int((~np.isnan(ref)).sum())

    F.set_eig_threshold(0.0)
    assert F.eig_threshold() == 0.0
    m.fp64_hits(reset=True)
    off = m.forward(fl, w.T).cpu().numpy().astype(np.float64)
    assert m.fp64_hits(reset=True) == 0

    F.set_eig_threshold(3.0)
    got = m.forward(fl, w.T).cpu().numpy().astype(np.float64)
    hits = m.fp64_hits(reset=True)
    print(f"forced: {hits} recomputes of {w.n} points ({usable} usable)", flush=True)
    assert hits == usable
    check_f32("fp64 branch forced, forward", got, ref, gap, w.T)
    # the branch did run: its float64 result differs from the float32 formula's
    assert not np.array_equal(np.nan_to_num(got, nan=7.0), np.nan_to_num(off, nan=7.0))

    g = np.random.default_rng(4).standard_normal(w.n)
    gt = torch.as_tensor(g, dtype=torch.float32, device=DEV)
    out, tape = m.forward_tape(fl, w.T)
    grad = m.backward_tape(tape, gt).cpu().numpy()
    assert m.fp64_hits(reset=True) == usable
    check_f32("fp64 branch forced, tape forward", out.cpu().numpy().astype(np.float64), ref, gap, w.T)
    gref, bad = _grad_ref(w, g.astype(np.float32), st)
    err = np.abs(grad - gref)[~bad].max() / np.abs(gref).max()
    print(f"fp64 branch forced, adjoint: max err/scale = {err:.3e}, excluded {bad.sum()}", flush=True)
    assert err <= 2e-4

    outs = F.batched([m], [fl], [w.T])
    torch.cuda.synchronize()
    assert torch.equal(torch.nan_to_num(outs[0], nan=7.0), torch.nan_to_num(m.forward(fl, w.T), nan=7.0))


@pytest.mark.parametrize("eps", [1e-3, 1e-4])
def test_fp64_eigen_branch_near_degenerate(default_threshold, eps):
    """phi = A x with A = Q diag(s, s (1 + eps), s / 3) Q^T: the two largest
    eigenvalues of C = A^T A differ by about 2 eps, so r + 1 is about 1.7e-5
    (eps = 1e-3) or 1.7e-7 (eps = 1e-4), far inside the default threshold 2e-3.
    Every point takes the float64 recompute; its FTLE matches the oracle and
    ln(s (1 + eps)) / |T|."""
    F.set_eig_threshold(-1.0)
    assert F.eig_threshold() == pytest.approx(2e-3)
    x, cells = meshes.kuhn_tet_grid(13)
    Q, _ = np.linalg.qr(np.random.default_rng(9).standard_normal((3, 3)))
    s = 1.7
    A = Q @ np.diag([s, s * (1 + eps), s / 3]) @ Q.T
    C = A.T @ A
    q = np.trace(C) / 3
    Bm = C - q * np.eye(3)
    p = math.sqrt((Bm * Bm).sum() / 6)
    r = np.linalg.det(Bm / p) / 2
    assert r + 1 < 1e-4
    x32 = x.astype(np.float32)
    phi = (x32.astype(np.float64) @ A.T).astype(np.float32)
    w = configs.Workload("near_degenerate", 3, x32, cells, torch.as_tensor(phi, device=DEV), 4.0, "f32")
    m = F.Mesh(x32, cells, "f32")
    m.fp64_hits(reset=True)
    got = m.forward(w.flow.contiguous(), w.T).cpu().numpy().astype(np.float64)
    hits = m.fp64_hits(reset=True)
    ref, gap, _ = ref_ftle(w)
    print(f"near-degenerate eps={eps}: {hits} recomputes of {w.n}", flush=True)
    assert hits > 0.9 * w.n
    check_f32(f"near-degenerate eps={eps}", got, ref, gap, w.T)
    exact = math.log(s * (1 + eps)) / w.T
    assert np.abs(got - exact).max() <= 2e-5 / (2 * w.T) + 1e-6
    # without the recompute the float32 formula is further off (reported only)
    F.set_eig_threshold(0.0)
    got0 = m.forward(w.flow.contiguous(), w.T).cpu().numpy().astype(np.float64)
    print(f"  max |f - exact|: float64 branch {np.abs(got - exact).max():.3e}, "
          f"float32 formula {np.abs(got0 - exact).max():.3e}", flush=True)


@pytest.fixture(scope="module")
def batched48():
    ws = configs.batched_2d(DEV)
    ms = [F.Mesh(w.coords, w.cells, "f32") for w in ws]
    fl = [w.flow.to(DEV).contiguous() for w in ws]
    fl2 = [torch.flip(f, dims=[0]).contiguous() for f in fl]
    Ts = [w.T for w in ws]
    Ts2 = [-0.5 * T for T in Ts]
    single = [m.forward(f, T) for m, f, T in zip(ms, fl, Ts)]
    single2 = [m.forward(f, T) for m, f, T in zip(ms, fl2, Ts2)]
    torch.cuda.synchronize()
    yield ws, ms, fl, fl2, Ts, Ts2, single, single2
    F.pin_batched_config(0)


def _same(a, b):
    return torch.equal(torch.nan_to_num(a, nan=7.0), torch.nan_to_num(b, nan=7.0))


@pytest.mark.parametrize("block,k,cap", [(256, 0, 0), (256, 1, 4), (256, 2, 4), (512, 4, 2), (128, 8, 8),
                                         (256, 1, 1)])
def test_batched_every_form_matches_forward(batched48, block, k, cap):
    """The 48-mesh set in a pinned launch form: two calls back to back (the
    second's queue counters are the ones the first's last workgroup reset),
    then two more on different streams, each output equal to ftle_forward's
    bit for bit."""
    ws, ms, fl, fl2, Ts, Ts2, single, single2 = batched48
    F.pin_batched_config(block, k, cap)
    a = F.batched(ms, fl, Ts)
    b = F.batched(ms, fl2, Ts2)
    torch.cuda.synchronize()
    cfg = F.batched_config(ms)
    print(f"pinned block {block} tiles/pop {k} cap {cap}: {cfg}", flush=True)
    assert cfg["block"] == block and cfg["tiles_per_pop"] == k
    if k == 0:
        assert cfg["grid"] == sum(m.tile_stats()["n_tiles"] for m in ms)
    else:
        assert 1 <= cfg["grid"] <= 256 * cap
    for s1, o1, s2, o2 in zip(single, a, single2, b):
        assert _same(o1, s1) and _same(o2, s2)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        c = F.batched(ms, fl2, Ts2)
    d = F.batched(ms, fl, Ts)
    torch.cuda.synchronize()
    for s1, o1, s2, o2 in zip(single, d, single2, c):
        assert _same(o1, s1) and _same(o2, s2)


def test_batched_pin_rejects_and_unpins():
    with pytest.raises(F.FTLEError):
        F.pin_batched_config(96, 1, 4)
    with pytest.raises(F.FTLEError):
        F.pin_batched_config(256, 1, 0)
    F.pin_batched_config(0)


def _widen(w):
    return configs.Workload(w.name + "_f64", w.dim, w.coords.astype(np.float64), w.cells,
                            w.flow.to(torch.float64).contiguous(), w.T, "f64", dict(w.extra))


@pytest.mark.parametrize("which", ["scale_2d_2048", "abc_3d_96"])
def test_fp64_forward_at_scale_sampled(which):
    """The float64 forward (the paper's precision) on the 2048^2 and 96^3
    workloads, sampled against the oracle at the float64 tolerances."""
    w = _widen(configs.scale_2d(DEV) if which == "scale_2d_2048" else configs.abc3d(96, 10.0, "f32", DEV))
    m = F.Mesh(w.coords, w.cells, "f64")
    got = m.forward(w.flow, w.T).cpu().numpy()
    sel = _sample(w.n, 20000, 21)
    ref, gap, _ = ref_ftle(w, sel=sel)
    check_f64(f"{which} float64 sampled", got[sel], ref, gap, w.T, w.dim)
    assert np.isfinite(got).all()
