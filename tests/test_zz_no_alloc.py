"""The allocation-free adjoint (ftle_backward_noalloc) through the C ABI,
against ftle_backward on the same inputs: bit for bit, on two calls in a row,
the second with a smaller mesh than the first (the shared scratch then still
holds the first call's tape beyond the second's points)."""
import numpy as np
import pytest
import torch

import paper_2408_02758_amd as F
from workloads import configs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _case(w, seed):
    m = F.Mesh(w.coords, w.cells, w.dtype)
    fl = w.flow.to(DEV).contiguous()
    g = torch.as_tensor(np.random.default_rng(seed).standard_normal(w.n), dtype=fl.dtype, device=DEV)
    return m, fl, g, w.T


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_backward_noalloc_matches_backward(dtype):
    big = _case(configs.abc3d(30 if dtype == "f32" else 20, 10.0, dtype, DEV), 1)
    small = _case(configs.abc3d(11, 6.0, dtype, DEV), 2)
    assert small[0].n < big[0].n
    # two calls in a row, no synchronisation between them
    outs = [m.backward_noalloc(fl, T, g, torch.empty_like(fl)) for m, fl, g, T in (big, small)]
    torch.cuda.synchronize()
    for (m, fl, g, T), got in zip((big, small), outs):
        ref = m.backward(fl, T, g)
        torch.cuda.synchronize()
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref)
    # then a 2D mesh
    m2, fl2, g2, T2 = _case(configs.tri2d(61, 47, seed=3, t0=0.0, T=9.0, dtype=dtype, device=DEV), 3)
    got2 = m2.backward_noalloc(fl2, T2, g2, torch.empty_like(fl2))
    assert torch.equal(got2, m2.backward(fl2, T2, g2))


def test_backward_noalloc_replayed_from_a_captured_graph():
    """The callers it is for: captured once into a HIP graph (no allocation
    happens inside), replayed three times with eager work and synchronisation
    between the replays, each replay equal to ftle_backward bit for bit."""
    m, fl, g, T = _case(configs.abc3d(14, 8.0, "f32", DEV), 4)
    out = torch.empty_like(fl)
    ref = m.backward(fl, T, g)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        m.backward_noalloc(fl, T, g, out, stream=side)   # first use on this device, outside the capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        m.backward_noalloc(fl, T, g, out, stream=side)
    torch.cuda.synchronize()
    for k in range(3):
        out.fill_(float("nan"))
        scratch_user = m.backward_noalloc(fl * 1.01, T, g, torch.empty_like(fl))   # the shared scratch rewritten
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {k}"
        assert not torch.equal(scratch_user, ref)
