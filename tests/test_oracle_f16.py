"""Pins of the oracle's half-precision flow-map storage (encode_flow_f16,
decode_flow_f16) against the IEEE 754 binary16 format written out: values
built from sign, exponent and significand, halfway cases, overflow."""
import numpy as np

import oracle


def f16(sign, exp, frac):
    """The binary16 number (-1)^sign 2^(exp-15) (1 + frac/1024), normal range."""
    return (-1.0) ** sign * 2.0 ** (exp - 15) * (1 + frac / 1024.0)


def test_exact_displacements_round_trip():
    rng = np.random.default_rng(3)
    d = np.array([f16(int(s), int(e), int(f)) for s, e, f in
                  zip(rng.integers(0, 2, 200), rng.integers(5, 20, 200), rng.integers(0, 1024, 200))])
    x = rng.integers(-8, 8, 200).astype(np.float64) * 0.5     # x + d exact in float32
    d2, x2 = d.reshape(-1, 2), x.reshape(-1, 2)
    enc = oracle.encode_flow_f16(x2, x2 + d2)
    assert enc.dtype == np.float16
    assert np.array_equal(enc.astype(np.float64), d2)
    assert np.array_equal(oracle.decode_flow_f16(x2, enc).astype(np.float64), x2 + d2)


def test_halfway_cases_round_to_even():
    # binary16 spacing in [1, 2) is 2^-10; the halfway points 1 + (2k+1) 2^-11
    one = np.zeros((1, 2))
    for k in range(6):
        v = 1 + (2 * k + 1) * 2.0 ** -11
        lo, hi = 1 + k * 2.0 ** -10, 1 + (k + 1) * 2.0 ** -10
        even = lo if k % 2 == 0 else hi
        got = oracle.encode_flow_f16(one, np.full((1, 2), v)).astype(np.float64)
        assert np.all(got == even), (k, got, even)
    # just above halfway rounds up
    v = 1 + 2.0 ** -11 + 2.0 ** -20
    assert np.all(oracle.encode_flow_f16(one, np.full((1, 2), v)).astype(np.float64) == 1 + 2.0 ** -10)


def test_relative_error_bound_and_overflow():
    rng = np.random.default_rng(5)
    x = rng.uniform(0, 2, (5000, 2)).astype(np.float32)
    phi = (x + rng.uniform(-1.5, 1.5, (5000, 2))).astype(np.float32)
    # the float32 difference rounds by <= 2^-24 relative, binary16 then by
    # <= 2^-11 relative (normal range) or 2^-25 absolute (subnormal range)
    d = phi.astype(np.float64) - x.astype(np.float64)
    enc = oracle.encode_flow_f16(x, phi).astype(np.float64)
    small = np.abs(d) < 2.0 ** -14
    assert np.all(np.abs(enc - d)[~small] <= (2.0 ** -11 + 2.0 ** -23) * np.abs(d)[~small])
    assert np.all(np.abs(enc - d)[small] <= 2.0 ** -25)
    big = oracle.encode_flow_f16(np.zeros((1, 2)), np.array([[70000.0, -65520.0]]))
    assert np.isinf(big).all() and big[0, 0] > 0 and big[0, 1] < 0
    assert oracle.encode_flow_f16(np.zeros((1, 2)), np.array([[65504.0, 65519.0]])).astype(np.float64).tolist() == \
        [[65504.0, 65504.0]]


# ---------------------------------------------------------------------------
# the stated error bound of a stored flow map (flow_error_f16 and
# ftle_perturbation_bound): pinned by perturbations drawn inside it and by
# the storage's own rounding
# ---------------------------------------------------------------------------
def _smooth_case(dim, seed):
    from workloads import meshes
    x, cells = meshes.jittered_tri_grid(20, 15, seed=seed) if dim == 2 else meshes.kuhn_tet_grid(6)
    g = np.random.default_rng(seed)
    a = g.normal(size=(dim, dim)) * 0.4
    phi = x + np.sin(x @ a) * 0.3
    return x, phi, oracle.ring1(dim, x.shape[0], cells)


def test_perturbation_bound_holds_and_is_not_vacuous():
    """Flow maps perturbed by at most delta_j per component (uniform and
    extreme-sign draws) never move the oracle's FTLE past the bound, and the
    worst draw comes within a factor 20 of it; delta = 0 gives 0."""
    for dim in (2, 3):
        x, phi, st = _smooth_case(dim, 3 + dim)
        T = 2.5
        g = np.random.default_rng(dim)
        delta = g.uniform(0.2e-4, 1e-4, x.shape[0])
        bd = oracle.ftle_perturbation_bound(dim, x, phi, st, T, delta)
        f0 = oracle.ftle(dim, x, phi, st, T)
        fin = np.isfinite(f0)
        assert np.array_equal(np.isnan(bd), np.isnan(f0)) and np.isfinite(bd[fin]).all()
        worst = 0.0
        for k in range(24):
            e = g.uniform(-1.0, 1.0, size=phi.shape)
            if k % 2:
                e = np.sign(e)
            f1 = oracle.ftle(dim, x, phi + e * delta[:, None], st, T)
            diff = np.abs(f1 - f0)[fin]
            assert np.all(diff <= bd[fin] * (1 + 1e-9) + 1e-14), (dim, k)
            worst = max(worst, float((diff / bd[fin]).max()))
        assert worst > 0.05, worst
        z = oracle.ftle_perturbation_bound(dim, x, phi, st, T, np.zeros(x.shape[0]))
        assert np.all(z[fin] == 0.0)


def test_f16_storage_error_and_ftle_within_the_bound():
    """flow_error_f16 bounds the decoded map's error at every point (normal,
    subnormal and large displacements), and on a 128^2 double-gyre map the FTLE
    of the decoded map stays within ftle_perturbation_bound of the float32
    map's at every point."""
    g = np.random.default_rng(5)
    x = g.uniform(-3, 3, size=(20000, 2)).astype(np.float32)
    d = np.concatenate([g.normal(size=(10000, 2)) * 10.0 ** g.uniform(-9, 3, size=(10000, 1)),
                        g.normal(size=(10000, 2)) * 1e-6])
    p = (x.astype(np.float64) + d).astype(np.float32)
    dec = oracle.decode_flow_f16(x, oracle.encode_flow_f16(x, p)).astype(np.float64)
    err = np.abs(dec - p.astype(np.float64)).max(axis=1)
    bound = oracle.flow_error_f16(x, p)
    assert np.all(err <= bound)
    assert (err / bound).max() > 0.3   # the bound is nearly attained
    from workloads import configs
    w = configs.tri2d(128, 128, seed=2, t0=0.0, T=15.0, dtype="f32")
    st = oracle.ring1(2, w.n, w.cells)
    x32 = w.coords.astype(np.float32)
    p32 = w.flow_numpy().astype(np.float32)
    pd = oracle.decode_flow_f16(x32, oracle.encode_flow_f16(x32, p32))
    f0 = oracle.ftle(2, x32.astype(np.float64), p32.astype(np.float64), st, w.T)
    f1 = oracle.ftle(2, x32.astype(np.float64), pd.astype(np.float64), st, w.T)
    bd = oracle.ftle_perturbation_bound(2, x32, p32, st, w.T, oracle.flow_error_f16(x32, p32))
    fin = np.isfinite(f0) & np.isfinite(f1)
    assert np.all(np.abs(f1 - f0)[fin] <= bd[fin])
