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
