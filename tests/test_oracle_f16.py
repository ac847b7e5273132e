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
