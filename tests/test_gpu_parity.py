"""Parity of the HIP path (through the C ABI) with the FP64 oracle, on the GPU.

Tolerances (from the float32 arithmetic: short sums of products over at most
~16 neighbours, an adjugate solve with cond(M) <= 10 on these meshes, and
the hardware log2's ~1 ulp; the observed errors sit two orders below):
  float64 meshes: |f_gpu - f_ref| <= 1e-12 + 1e-10 |f_ref|    (3D: 1e-9 where the
                  top eigenvalue pair is closer than 1e-3 relative, where the
                  trigonometric formula loses half the digits)
  float32 meshes, on the same float32-rounded inputs:
    all finite points        |ln lam_gpu - ln lam_ref| = 2|T| |f_gpu - f_ref| <= 2e-5
    well separated points    |f_gpu - f_ref| <= 1e-5 |f_ref|
                             (gap (lam1-lam2)/lam1 >= 1e-3 and |ln lam_ref| >= 0.05)
  NaN exactly where the oracle gives NaN.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2408_02758_amd as F
from workloads import configs, flows, meshes

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _report(tag, got, ref, T, gap=None):
    fin = np.isfinite(ref)
    d = np.abs(got[fin] - ref[fin])
    msg = f"[{tag}] n={ref.size} finite={fin.sum()} max|d|={d.max() if d.size else 0:.3e}"
    if gap is not None:
        lnl = 2 * abs(T) * np.abs(ref)
        mask = fin & (gap >= 1e-3) & (lnl >= 0.05)
        if mask.any():
            rel = np.abs(got[mask] - ref[mask]) / np.abs(ref[mask])
            msg += f" masked={mask.mean():.4f} max_rel={rel.max():.3e} p99_rel={np.quantile(rel, 0.99):.3e}"
        msg += f" max|dlnlam|={2 * abs(T) * (d.max() if d.size else 0):.3e}"
    print(msg, flush=True)


def check_f32(tag, got, ref, gap, T):
    _report(tag, got, ref, T, gap)
    assert np.array_equal(np.isnan(got), np.isnan(ref)), f"{tag}: NaN masks differ"
    fin = np.isfinite(ref)
    assert np.all(np.isfinite(got[fin]))
    dl = 2 * abs(T) * np.abs(got[fin] - ref[fin])
    assert dl.max(initial=0) <= 2e-5, f"{tag}: max |d ln lam| {dl.max()}"
    lnl = 2 * abs(T) * np.abs(ref)
    mask = fin & (gap >= 1e-3) & (lnl >= 0.05)
    rel = np.abs(got[mask] - ref[mask]) / np.abs(ref[mask])
    assert rel.max(initial=0) <= 1e-5, f"{tag}: max rel {rel.max()}"


def check_f64(tag, got, ref, gap=None, T=1.0, dim=2):
    _report(tag, got, ref, T, gap)
    assert np.array_equal(np.isnan(got), np.isnan(ref)), f"{tag}: NaN masks differ"
    fin = np.isfinite(ref)
    tol = 1e-12 + 1e-10 * np.abs(ref[fin])
    if dim == 3 and gap is not None:
        tol = np.where(gap[fin] < 1e-3, 1e-9 + 1e-9 * np.abs(ref[fin]), tol)
    assert np.all(np.abs(got[fin] - ref[fin]) <= tol), f"{tag}: max {np.abs(got[fin] - ref[fin]).max()}"


def gpu_ftle(w, **mesh_kw):
    m = F.Mesh(w.coords, w.cells, w.dtype, **mesh_kw)
    out = m.forward(w.flow.to(DEV).contiguous(), w.T)
    torch.cuda.synchronize()
    return m, out.cpu().numpy().astype(np.float64)


def ref_ftle(w, stencil="ring1", sel=None):
    st = oracle.ring1(w.dim, w.n, w.cells)
    if stencil == "axis":
        st = oracle.axis(w.dim, w.coords.astype(np.float64), st)
    f, gap, _ = oracle.ftle(w.dim, w.coords.astype(np.float64), w.flow_numpy().astype(np.float64), st, w.T,
                            sel=sel, diagnostics=True)
    return f, gap, st


# ---------------------------------------------------------------------------
# forward
# ---------------------------------------------------------------------------

def test_small_2d_f64():
    w = configs.small_2d(DEV)
    _, got = gpu_ftle(w)
    ref, gap, _ = ref_ftle(w)
    check_f64("small_2d f64", got, ref, gap, w.T)


@pytest.mark.parametrize("tile_log2", [0, 5, 8, 11])
def test_tri2d_f32_tiles(tile_log2):
    w = configs.tri2d(200, 131, seed=2, t0=0.0, T=15.0, dtype="f32", device=DEV)
    _, got = gpu_ftle(w, tile_log2=tile_log2)
    ref, gap, _ = ref_ftle(w)
    check_f32(f"tri2d 200x131 f32 tile={tile_log2}", got, ref, gap, w.T)


def test_abc3d_f32():
    w = configs.abc3d(33, 10.0, "f32", DEV)
    m, got = gpu_ftle(w)
    ref, gap, _ = ref_ftle(w)
    check_f32("abc3d 33^3 f32", got, ref, gap, w.T)
    print("fp64 eigen recomputes:", m.fp64_hits())


def test_abc3d_f64():
    w = configs.abc3d(17, 10.0, "f64", DEV)
    _, got = gpu_ftle(w)
    ref, gap, _ = ref_ftle(w)
    check_f64("abc3d 17^3 f64", got, ref, gap, w.T, dim=3)


@pytest.mark.parametrize("dim", [2, 3])
def test_axis_stencil(dim):
    w = (configs.tri2d(90, 70, seed=4, t0=1.0, T=8.0, dtype="f32", device=DEV) if dim == 2
         else configs.abc3d(20, 6.0, "f32", DEV))
    _, got = gpu_ftle(w, stencil="axis")
    ref, gap, _ = ref_ftle(w, "axis")
    check_f32(f"axis {dim}D f32", got, ref, gap, w.T)


def test_relabel_and_no_reorder():
    w = configs.tri2d(120, 77, seed=8, t0=0.5, T=10.0, dtype="f32", device=DEV)
    ref, gap, _ = ref_ftle(w)
    _, got = gpu_ftle(w, reorder=False)
    check_f32("no_reorder", got, ref, gap, w.T)
    x2, c2, p = meshes.relabel(w.coords, w.cells, seed=3)
    f2 = torch.empty_like(w.flow)
    f2[torch.as_tensor(p, device=w.flow.device)] = w.flow
    w2 = configs.Workload("relabel", 2, x2, c2, f2, w.T, "f32")
    _, got2 = gpu_ftle(w2)
    check_f32("relabel", got2[p], ref, gap, w.T)


def test_negative_T_and_scaling_closed_form():
    rng = np.random.default_rng(3)
    x, cells = meshes.jittered_tri_grid(64, 48, seed=5)
    A = np.array([[2.0, 1.0], [0.3, 0.7]])
    phi = x @ A.T + rng.standard_normal(2)
    m = F.Mesh(x, cells, "f64")
    out = m.forward(torch.as_tensor(phi, device=DEV), -4.0).cpu().numpy()
    ref = math.log(np.linalg.svd(A, compute_uv=False)[0]) / 4.0
    assert np.allclose(out, ref, rtol=1e-12, atol=1e-13)


def test_degenerate_points_and_nan_flow():
    # isolated point, a collinear fan, a lone triangle, then NaN in the flow map
    x = np.array([[0, 0], [1, 0], [0, 1], [5, 5], [6, 6], [7, 7], [8, 8], [20, 0], [21, 0], [20, 1]], np.float64)
    cells = np.array([[0, 1, 2], [3, 4, 5], [3, 5, 6], [7, 8, 9]], np.int32)
    phi = x * 1.5 + 0.25
    for dt in ("f64", "f32"):
        m = F.Mesh(x, cells, dt)
        t = torch.as_tensor(phi, dtype=m.torch_dtype, device=DEV)
        got = m.forward(t, 2.0).cpu().numpy()
        st = oracle.ring1(2, x.shape[0], cells)
        ref = oracle.ftle(2, x.astype(m.torch_dtype == torch.float32 and np.float32 or np.float64), phi, st, 2.0)
        assert np.array_equal(np.isnan(got), np.isnan(ref)), (dt, got, ref)
        fin = np.isfinite(ref)
        assert np.allclose(got[fin], ref[fin], rtol=1e-5, atol=1e-6)
        t2 = t.clone()
        t2[1, 0] = float("nan")
        got2 = m.forward(t2, 2.0).cpu().numpy()
        assert np.isnan(got2[[0, 1, 2]]).all() and np.isfinite(got2[[7, 8, 9]]).all()


def test_single_point_and_tiny():
    m = F.Mesh(np.zeros((1, 3)), np.zeros((0, 4), np.int32), "f32")
    out = m.forward(torch.zeros(1, 3, device=DEV), 1.0)
    assert torch.isnan(out).all()
    x = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], np.float64)
    m = F.Mesh(x, np.array([[0, 1, 2, 3]], np.int32), "f64")
    out = m.forward(torch.as_tensor(2 * x, device=DEV), 0.5).cpu().numpy()
    assert np.allclose(out, math.log(2) / 0.5, rtol=1e-12)


# ---------------------------------------------------------------------------
# full-size workloads, sampled against the oracle (same launch as the bench)
# ---------------------------------------------------------------------------

def _sample(n, k, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([rng.choice(n, k, replace=False), np.arange(64), np.arange(n - 64, n)]))


def test_scale_2d_2048_sampled():
    w = configs.scale_2d(DEV)
    m, got = gpu_ftle(w)
    sel = _sample(w.n, 20000, 11)
    ref, gap, _ = ref_ftle(w, sel=sel)
    check_f32("scale_2d 2048^2 sampled", got[sel], ref, gap, w.T)
    assert np.isfinite(got).all()


def test_abc_3d_160_sampled():
    w = configs.abc_3d(DEV)
    m, got = gpu_ftle(w)
    sel = _sample(w.n, 20000, 12)
    ref, gap, _ = ref_ftle(w, sel=sel)
    check_f32("abc_3d 160^3 sampled", got[sel], ref, gap, w.T)
    assert np.isfinite(got).all()
    print("fp64 eigen recomputes (160^3):", m.fp64_hits())


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------

def _grad_case(dim, dtype, n=None):
    if dim == 2:
        x, cells = meshes.jittered_tri_grid(40, 30, seed=5)
        phi = flows.advect_rk4(flows.double_gyre_velocity, x, 0.0, 5.0, 0.01, DEV)
        T = 5.0
    else:
        n = n or 16
        x, cells = meshes.kuhn_tet_grid(n)
        phi = flows.advect_rk4(flows.abc_velocity, x, 0.0, 10.0, 0.02, DEV)
        T = 10.0
    npd = np.float32 if dtype == "f32" else np.float64
    td = torch.float32 if dtype == "f32" else torch.float64
    return x.astype(npd), cells, phi.to(td).contiguous(), T


@pytest.mark.parametrize("dim,dtype", [(2, "f64"), (3, "f64"), (2, "f32"), (3, "f32")])
@pytest.mark.parametrize("stencil", ["ring1", "axis"])
def test_adjoint_vs_oracle(dim, dtype, stencil):
    x, cells, phi, T = _grad_case(dim, dtype)
    m = F.Mesh(x, cells, dtype, stencil=stencil)
    g = torch.as_tensor(np.random.default_rng(6).standard_normal(x.shape[0]), dtype=phi.dtype, device=DEV)
    out, tape = m.forward_tape(phi, T)
    g1 = m.backward_tape(tape, g).cpu().numpy()
    g2 = m.backward(phi, T, g).cpu().numpy()
    st = oracle.ring1(dim, x.shape[0], cells)
    if stencil == "axis":
        st = oracle.axis(dim, x.astype(np.float64), st)
    xd, pd = x.astype(np.float64), phi.cpu().numpy().astype(np.float64)
    ref = oracle.ftle_grad(dim, xd, pd, st, T, g.cpu().numpy().astype(np.float64))
    fref, gap, _ = oracle.ftle(dim, xd, pd, st, T, diagnostics=True)
    # points next to a nearly repeated top eigenvalue have an ill-defined eigenvector
    bad = np.zeros(x.shape[0], bool)
    for i in np.nonzero(~(gap >= 1e-6))[0]:
        bad[i] = True
        bad[st.col[st.row_ptr[i]:st.row_ptr[i + 1]]] = True
    scale = np.abs(ref).max()
    for tag, got in (("tape", g1), ("recompute", g2)):
        err = np.abs(got - ref)[~bad].max() / scale
        print(f"[adjoint {dim}D {dtype} {stencil} {tag}] max err/scale = {err:.3e}, excluded {bad.sum()}", flush=True)
        assert err <= (1e-10 if dtype == "f64" else 2e-4), (tag, err)
    assert np.array_equal(g1, g2)
    check = check_f64 if dtype == "f64" else check_f32
    if dtype == "f64":
        check("adjoint fwd", out.cpu().numpy(), fref, gap, T, dim)
    else:
        check("adjoint fwd", out.cpu().numpy().astype(np.float64), fref, gap, T)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("relabel", [True, False])
def test_3d_records_worst_case_and_empty_rows(dtype, relabel):
    """Compressed records at their worst and at edges: a 3D grid plus a
    cluster of points in no cell (empty rows) and one point whose only cell is
    flat (a rank-deficient stencil of points that are themselves fine).
    Relabelled at random: every row explicit, one index run per slot, the
    empty rows scattered.  In grid order: the empty rows are consecutive
    slots, stored as shifts of one another.  Forward and adjoint against the
    oracle: the flat point's NaN FTLE adds nothing to its neighbours'
    gradients."""
    x0, c0, phi0, T = _grad_case(3, dtype, 14)
    n0 = x0.shape[0]
    extra = 5
    xe = (np.asarray(x0, np.float64).max(0) + 3.0 + 0.01 * np.arange(extra)[:, None]).astype(x0.dtype)
    # flat cell: three top-face corners of the grid and a new point in their plane
    top = np.nonzero(x0[:, 2] == x0[:, 2].max())[0]
    b, c, d = top[0], top[1], top[14]   # (0,0), (1,0), (0,1) of the top face
    xf = (x0[b] + 0.5 * (x0[b] - x0[c]) + 0.5 * (x0[b] - x0[d]))[None, :].astype(x0.dtype)
    x1 = np.concatenate([x0, xe, xf])
    nf = x1.shape[0] - 1
    c1 = np.concatenate([c0, np.array([[b, c, d, nf]], np.int32)])
    phi1 = torch.cat([phi0, torch.as_tensor(np.concatenate([2.0 * xe, 2.0 * xf]), dtype=phi0.dtype,
                                            device=phi0.device)]).contiguous()
    if relabel:
        x, cells, p = meshes.relabel(x1, c1, seed=11)
    else:
        x, cells, p = x1, c1, np.arange(x1.shape[0])
    phi = torch.empty_like(phi1)
    phi[torch.as_tensor(p, device=phi1.device)] = phi1
    x = x.astype(x0.dtype)
    m = F.Mesh(x, cells, dtype)
    recs = m.tile_records()
    if relabel:
        assert sum(len(r["xend"]) for r in recs) > 0.9 * x.shape[0]
    else:   # the empty rows after the first are shifts
        iso = set(range(n0 + 1, n0 + extra))
        shifts = 0
        for (idx, rowend, _, P, _), r in zip(m.tiles(), recs):
            for l in range(P):
                if int(idx[l]) in iso and not (int(r["xmask"][l // 32]) >> (l % 32)) & 1:
                    shifts += 1
        assert shifts == extra - 1
    g = torch.as_tensor(np.random.default_rng(7).standard_normal(x.shape[0]), dtype=phi.dtype, device=DEV)
    out, tape = m.forward_tape(phi, T)
    got_g = m.backward_tape(tape, g).cpu().numpy()
    st = oracle.ring1(3, x.shape[0], cells)
    xd, pd = x.astype(np.float64), phi.cpu().numpy().astype(np.float64)
    fref, gap, _ = oracle.ftle(3, xd, pd, st, T, diagnostics=True)
    assert np.isnan(fref[p[n0:]]).all() and np.isfinite(fref[p[[b, c, d]]]).all()
    got_f = out.cpu().numpy().astype(np.float64)
    if dtype == "f64":
        check_f64("records 3D", got_f, fref, gap, T, 3)
    else:
        check_f32("records 3D", got_f, fref, gap, T)
    ref = oracle.ftle_grad(3, xd, pd, st, T, g.cpu().numpy().astype(np.float64))
    # points with an ill-defined top eigenvector (finite FTLE, nearly repeated
    # top eigenvalue) and their neighbours are excluded; NaN points are not
    bad = np.zeros(x.shape[0], bool)
    for i in np.nonzero(np.isfinite(fref) & ~(gap >= 1e-6))[0]:
        bad[i] = True
        bad[st.col[st.row_ptr[i]:st.row_ptr[i + 1]]] = True
    assert np.isfinite(got_g).all()
    err = np.abs(got_g - ref)[~bad].max() / np.abs(ref).max()
    print(f"[records 3D {dtype} relabel={relabel}] adjoint max err/scale = {err:.3e}, excluded {bad.sum()}",
          flush=True)
    assert err <= (1e-10 if dtype == "f64" else 2e-4)
    assert not bad[p[[b, c, d, nf]]].any()
    assert np.all(got_g[p[n0:nf]] == 0)


@pytest.mark.parametrize("dim,dtype", [(2, "f32"), (3, "f32"), (3, "f64")])
def test_from_csr_knn_vs_oracle(dim, dtype):
    """A caller-supplied, non-symmetric stencil (the k nearest neighbours):
    forward and adjoint (gather over the transposed stencil, sigma from the
    tape) against the oracle on the same stencil; and the cells' own stencil
    given as a list reproduces the cells mesh bit for bit."""
    from scipy.spatial import cKDTree
    x, cells, phi, T = _grad_case(dim, dtype)
    k = 6 if dim == 2 else 10
    _, nb = cKDTree(np.asarray(x, np.float64)).query(np.asarray(x, np.float64), k + 1)
    nb = np.ascontiguousarray(nb[:, 1:], dtype=np.int32).ravel()
    row_ptr = np.arange(x.shape[0] + 1, dtype=np.int64) * k
    m = F.Mesh.from_csr(x, row_ptr, nb, dtype)
    st = oracle.Stencil(row_ptr, nb)
    xd, pd = x.astype(np.float64), phi.cpu().numpy().astype(np.float64)
    fref, gap, _ = oracle.ftle(dim, xd, pd, st, T, diagnostics=True)
    g = torch.as_tensor(np.random.default_rng(8).standard_normal(x.shape[0]), dtype=phi.dtype, device=DEV)
    out, tape = m.forward_tape(phi, T)
    f = m.forward(phi, T).cpu().numpy().astype(np.float64)
    grad = m.backward_tape(tape, g).cpu().numpy()
    check = check_f64 if dtype == "f64" else check_f32
    if dtype == "f64":
        check("knn fwd", f, fref, gap, T, dim)
        check("knn tape fwd", out.cpu().numpy(), fref, gap, T, dim)
    else:
        check("knn fwd", f, fref, gap, T)
        check("knn tape fwd", out.cpu().numpy().astype(np.float64), fref, gap, T)
    ref = oracle.ftle_grad(dim, xd, pd, st, T, g.cpu().numpy().astype(np.float64))
    bad = np.zeros(x.shape[0], bool)
    for i in np.nonzero(np.isfinite(fref) & ~(gap >= 1e-6))[0]:
        bad[i] = True
        bad[st.col[st.row_ptr[i]:st.row_ptr[i + 1]]] = True
    err = np.abs(grad - ref)[~bad].max() / np.abs(ref).max()
    print(f"[knn {dim}D {dtype}] adjoint max err/scale = {err:.3e}, excluded {bad.sum()}", flush=True)
    assert err <= (1e-10 if dtype == "f64" else 2e-4)
    # the cells' stencil as a list: the same mesh
    ring = oracle.ring1(dim, x.shape[0], cells)
    mr = F.Mesh.from_csr(x, ring.row_ptr, ring.col, dtype)
    mc = F.Mesh(x, cells, dtype)
    assert torch.equal(torch.nan_to_num(mr.forward(phi, T), nan=7.0), torch.nan_to_num(mc.forward(phi, T), nan=7.0))


def test_adjoint_fd_16cubed_f64():
    """GPU float64 adjoint against central differences (h = 1e-6) of the oracle's FTLE."""
    x, cells, phi, T = _grad_case(3, "f64", 16)
    m = F.Mesh(x, cells, "f64")
    w = np.random.default_rng(6).standard_normal(x.shape[0])
    g = torch.as_tensor(w, device=DEV)
    grad = m.backward(phi, T, g).cpu().numpy()
    st = oracle.ring1(3, x.shape[0], cells)
    ph = phi.cpu().numpy().copy()
    _, gap, _ = oracle.ftle(3, x, ph, st, T, diagnostics=True)
    rng = np.random.default_rng(1)
    h = 1e-6
    gmax = np.abs(grad).max()
    checked = 0
    for j in rng.choice(x.shape[0], 300, replace=False):
        aff = np.concatenate([[j], st.col[st.row_ptr[j]:st.row_ptr[j + 1]]]).astype(np.int64)
        if np.any(gap[aff] < 1e-4):
            continue
        for c in range(3):
            old = ph[j, c]
            ph[j, c] = old + h
            lp = np.dot(w[aff], oracle.ftle(3, x, ph, st, T, sel=aff))
            ph[j, c] = old - h
            lm = np.dot(w[aff], oracle.ftle(3, x, ph, st, T, sel=aff))
            ph[j, c] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - grad[j, c]) <= 1e-6 * gmax + 1e-5 * abs(grad[j, c]), (j, c, fd, grad[j, c])
            checked += 1
    assert checked >= 600


def test_diff_3d_96_identities_and_autograd():
    w = configs.diff_3d(DEV)
    m = F.Mesh(w.coords, w.cells, "f32")
    flow = w.flow.to(DEV).clone().requires_grad_(True)
    wt = torch.as_tensor(w.extra["weights"], dtype=torch.float32, device=DEV)
    f = F.ftle(m, flow, w.T)
    loss = (wt * f).sum()
    loss.backward()
    g = flow.grad.double()
    phi = w.flow.to(DEV).double()
    fin = torch.isfinite(f.detach())
    scale = g.abs().sum().item()
    s0 = g.sum(0).abs().max().item() / scale
    s1 = abs((g * phi).sum().item() - wt.double()[fin].sum().item() / w.T) / (g * phi).abs().sum().item()
    S = g.T @ phi
    s2 = (S - S.T).abs().max().item() / (g.abs().sum(1) * phi.abs().sum(1)).sum().item()
    print(f"[diff 96^3 identities] translation {s0:.2e} scaling {s1:.2e} rotation {s2:.2e}", flush=True)
    assert s0 < 1e-5 and s1 < 1e-4 and s2 < 1e-5
    # autograd path == explicit tape path == oracle (sampled)
    out, tape = m.forward_tape(w.flow.to(DEV).contiguous(), w.T)
    assert torch.equal(out, f.detach())
    g2 = m.backward_tape(tape, wt)
    assert torch.equal(g2, flow.grad)
    st = oracle.ring1(3, w.n, w.cells)
    ref = oracle.ftle_grad(3, w.coords.astype(np.float64), w.flow_numpy().astype(np.float64), st, w.T,
                           w.extra["weights"].astype(np.float32).astype(np.float64))
    err = np.abs(flow.grad.cpu().numpy() - ref).max() / np.abs(ref).max()
    print(f"[diff 96^3 adjoint vs oracle] max err/scale = {err:.3e}", flush=True)
    assert err <= 2e-4


# ---------------------------------------------------------------------------
# batched
# ---------------------------------------------------------------------------

def test_batched_matches_forward_bitwise_and_replays():
    ws = configs.batched_2d(DEV, count=10, seed=3, lo=64, hi=400)
    ms = [F.Mesh(w.coords, w.cells, "f32") for w in ws]
    fl = [w.flow.to(DEV).contiguous() for w in ws]
    Ts = [w.T for w in ws]
    outs = F.batched(ms, fl, Ts)
    singles = [m.forward(f, T) for m, f, T in zip(ms, fl, Ts)]
    for o, s in zip(outs, singles):
        assert torch.equal(o, s)
    print("batched config:", F.batched_config(ms), flush=True)
    # replay with new flow maps and times (graph arguments updated)
    fl2 = [torch.flip(f, dims=[0]).contiguous() for f in fl]
    Ts2 = [-2.0 * T for T in Ts]
    for rep in range(3):
        outs2 = F.batched(ms, fl2, Ts2)
        torch.cuda.synchronize()
        for m, o, f, T in zip(ms, outs2, fl2, Ts2):
            assert torch.equal(o, m.forward(f, T))
    # a prepared call gives the same results and can be replayed
    call = F.BatchedCall(ms, fl2, Ts2)
    for rep in range(2):
        outs3 = call()
        torch.cuda.synchronize()
        for o2, o3 in zip(outs2, outs3):
            assert torch.equal(o2, o3)
    # against the oracle for a few meshes
    for k in (0, 4, 9):
        ref, gap, _ = ref_ftle(ws[k])
        check_f32(f"batched mesh {k}", outs[k].cpu().numpy().astype(np.float64), ref, gap, ws[k].T)


def test_batched_3d_and_f64_match_forward():
    """Batched launches of 3D float32 meshes and of 2D float64 meshes give the
    single-mesh forward's results bit for bit (same tile body, other launch)."""
    groups = [
        [configs.abc3d(n, T, "f32", DEV) for n, T in ((10, 10.0), (17, 6.0), (13, -8.0))],
        [configs.tri2d(n, m, s, t0, T, "f64", DEV) for n, m, s, t0, T in ((30, 20, 1, 0.0, 15.0), (41, 41, 2, 3.0, 7.5))],
    ]
    for ws in groups:
        ms = [F.Mesh(w.coords, w.cells, w.dtype) for w in ws]
        fl = [w.flow.to(DEV).contiguous() for w in ws]
        outs = F.batched(ms, fl, [w.T for w in ws])
        torch.cuda.synchronize()
        for m, o, f, w in zip(ms, outs, fl, ws):
            single = m.forward(f, w.T)
            assert torch.equal(torch.nan_to_num(o, nan=7.0), torch.nan_to_num(single, nan=7.0)), w.name


def test_batched_full_48():
    ws = configs.batched_2d(DEV)
    ms = [F.Mesh(w.coords, w.cells, "f32") for w in ws]
    fl = [w.flow.to(DEV).contiguous() for w in ws]
    outs = F.batched(ms, fl, [w.T for w in ws])
    for k in range(0, 48, 7):
        assert torch.equal(outs[k], ms[k].forward(fl[k], ws[k].T))
    for k in (1, 20):
        sel = _sample(ws[k].n, min(ws[k].n - 200, 5000), k)
        ref, gap, _ = ref_ftle(ws[k], sel=sel)
        check_f32(f"batched48 mesh {k}", outs[k].cpu().numpy().astype(np.float64)[sel], ref, gap, ws[k].T)


@pytest.mark.gpu
def test_wide_offsets_match_default():
    """The 64-bit offset kernels (the path taken when a mesh's per-point arrays
    reach 4 GiB) give bit-identical results to the default 32-bit ones, for the
    forward, tape forward, adjoint (RING1 and AXIS) and batched launches, in
    float32 and float64."""
    cases = [configs.tri2d(37, 29, 11, 0.0, 15.0, "f32", DEV),
             configs.abc3d(12, 10.0, "f32", DEV),
             configs.abc3d(9, 10.0, "f64", DEV)]

    def run(w, stencil):
        m = F.Mesh(w.coords, w.cells, w.dtype, stencil=stencil, tile_log2=6)
        fl = w.flow.to(DEV).contiguous()
        f = m.forward(fl, w.T)
        tape = torch.empty(m.tape_bytes() // fl.element_size(), dtype=fl.dtype, device=DEV)
        ft, _ = m.forward_tape(fl, w.T, tape=tape)
        g = torch.linspace(-1.0, 1.0, w.n, dtype=fl.dtype, device=DEV)
        gr = m.backward_tape(tape, g)
        torch.cuda.synchronize()
        return [f, ft, gr]

    try:
        for w in cases:
            for stencil in ("ring1", "axis"):
                F.force_wide_offsets(False)
                ref = run(w, stencil)
                F.force_wide_offsets(True)
                got = run(w, stencil)
                for a, b in zip(ref, got):
                    assert torch.equal(torch.nan_to_num(a, nan=7.0), torch.nan_to_num(b, nan=7.0)), (w.name, stencil)
        # batched: fresh meshes, so that the plan is built with the wide kernels
        w2 = [configs.tri2d(n, n, s, 1.0, 10.0, "f32", DEV) for n, s in ((20, 1), (45, 2), (33, 3))]
        fl = [w.flow.to(DEV).contiguous() for w in w2]
        F.force_wide_offsets(False)
        ref = F.batched([F.Mesh(w.coords, w.cells, "f32") for w in w2], fl, [w.T for w in w2])
        F.force_wide_offsets(True)
        got = F.batched([F.Mesh(w.coords, w.cells, "f32") for w in w2], fl, [w.T for w in w2])
        torch.cuda.synchronize()
        for a, b in zip(ref, got):
            assert torch.equal(torch.nan_to_num(a, nan=7.0), torch.nan_to_num(b, nan=7.0))
    finally:
        F.force_wide_offsets(False)
