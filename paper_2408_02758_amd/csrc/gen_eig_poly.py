"""Coefficients of the float32 3x3 eigenvalue step in ftle_device_math.h.

The largest eigenvalue of a symmetric 3x3 tensor is q + 2 p c, where c is
the largest root of 4 c^3 - 3 c = r, i.e. c = cos(acos(r) / 3) (the
trigonometric solution of the characteristic cubic).  With s = sqrt((1+r)/2)
this is c(s) = cos((2/3) acos(s)), an analytic function on [0, 1] (c(0) = 1/2,
c(1) = 1).  This script fits it by least squares in the Chebyshev basis on
[0, 1] (degree 7, 400001 samples) and prints the monomial coefficients for a
Horner evaluation in float32 (max error about 1.2e-7 in c).
"""
import numpy as np


def coefficients(deg: int = 7):
    s = np.linspace(0.0, 1.0, 400001)
    c = np.cos(2.0 / 3.0 * np.arccos(s))
    fit = np.polynomial.chebyshev.Chebyshev.fit(s, c, deg, domain=[0, 1])
    poly = fit.convert(kind=np.polynomial.Polynomial, domain=[0, 1], window=[0, 1])
    return poly.coef, float(np.max(np.abs(poly(s) - c)))


if __name__ == "__main__":
    coef, err = coefficients()
    print(f"// max |error| in float64: {err:.2e}")
    for k, a in enumerate(coef):
        print(f"constexpr float kEigC{k} = {a:.9e}f;")
