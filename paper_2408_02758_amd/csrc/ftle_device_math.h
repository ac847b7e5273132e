// Device helpers shared by the FTLE kernels (ftle_kernels.hip, ftle_ell.hip):
// the XCD-aware workgroup order, precision-explicit arithmetic, the rank
// threshold of the least-squares solve, and the closed-form largest
// eigenvalue of a symmetric 3x3 tensor with its float64 recompute.  Device
// code only; every function has internal linkage, so each translation unit
// has its own copy.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace ftle {
namespace {

// Workgroup id -> tile.  The hardware deals consecutive ids round-robin to
// the 8 XCDs; this gives XCD x the contiguous tile range
// [x*q + min(x, r), ...) with q = n / 8, r = n % 8 (a bijection on [0, n)).
__device__ inline int xcd_tile(int bid, int n)
{
    constexpr int kXcd = 8;
    const int x = bid % kXcd, s = bid / kXcd;
    const int q = n / kXcd, r = n % kXcd;
    return x * q + min(x, r) + s;
}

// Precision-explicit math (no silent promotion of float code to double).
// The float versions use the hardware reciprocal, square root and base-2
// logarithm (about 1 ulp): the Jacobian and eigenvalue they feed already
// carry O(10) ulp of accumulated rounding.
__device__ inline float drcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ inline double drcp(double v) { return 1.0 / v; }
__device__ inline float dsqrt(float v) { return __builtin_amdgcn_sqrtf(v); }
__device__ inline double dsqrt(double v) { return sqrt(v); }
__device__ inline double dacos(double v) { return acos(v); }
__device__ inline double dcos(double v) { return cos(v); }
__device__ inline float dfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double dfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ inline float dmin(float a, float b) { return fminf(a, b); }
__device__ inline double dmin(double a, double b) { return fmin(a, b); }
__device__ inline float dmax(float a, float b) { return fmaxf(a, b); }
__device__ inline double dmax(double a, double b) { return fmax(a, b); }

// ln(v) * scale.  Float: v_log_f32 (log2) on v pre-scaled out of the
// subnormal range, times scale * ln 2.
__device__ inline float log_scaled(float v, float scale)
{
    const bool tiny = v < 1.17549435e-38f;
    const float l2 = __builtin_amdgcn_logf(tiny ? v * 4294967296.0f : v) - (tiny ? 32.0f : 0.0f);
    return l2 * (scale * 0.693147180559945309f);
}
__device__ inline double log_scaled(double v, double scale) { return log(v) * scale; }

template <typename T> __device__ inline T quiet_nan();
template <> __device__ inline float quiet_nan<float>() { return __builtin_nanf(""); }
template <> __device__ inline double quiet_nan<double>() { return __builtin_nan(""); }

// Rank threshold of the least-squares solve: the stencil is rank deficient
// when det M <= tau (tr M / D)^D (this also covers fewer than D neighbours,
// whose M is singular).  float32 cannot resolve an exactly singular M below a
// few ulps of (tr M / D)^D, hence the looser float threshold.
template <typename T> __device__ inline T rank_tau();
template <> __device__ inline float rank_tau<float>() { return 1e-5f; }
template <> __device__ inline double rank_tau<double>() { return 1e-12; }


// ---------------------------------------------------------------------------
// Largest eigenvalue of a symmetric 3x3 tensor, closed form: with
// q = tr C / 3, p = sqrt(|C - qI|_F^2 / 6), r = det((C - qI)/p) / 2 in [-1, 1],
// lambda_max = q + 2 p c, where c = cos(acos(r)/3) is the largest root of
// 4c^3 - 3c = r (trigonometric solution of the characteristic cubic; O. K.
// Smith, CACM 4(4):168, 1961).  r is returned so that the caller can detect
// r -> -1 (top pair nearly equal), where c'(r) is unbounded.
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void cubic_qpr(T c00, T c01, T c02, T c11, T c12, T c22, T& q, T& p, T& r)
{
    q = (c00 + c11 + c22) * T(1.0 / 3.0);
    const T b00 = c00 - q, b11 = c11 - q, b22 = c22 - q;
    const T p2 = (b00 * b00 + b11 * b11 + b22 * b22 + T(2) * (c01 * c01 + c02 * c02 + c12 * c12)) *
                 T(1.0 / 6.0);
    if (!(p2 > T(0))) {
        p = T(0);
        r = T(1);
        return;
    }
    p = dsqrt(p2);
    const T ip = drcp(p);
    const T n00 = b00 * ip, n11 = b11 * ip, n22 = b22 * ip;
    const T n01 = c01 * ip, n02 = c02 * ip, n12 = c12 * ip;
    r = T(0.5) * (n00 * (n11 * n22 - n12 * n12) - n01 * (n01 * n22 - n12 * n02) +
                  n02 * (n01 * n12 - n11 * n02));
    r = dmin(dmax(r, T(-1)), T(1));
}

__device__ inline double lam_max3_trig(double c00, double c01, double c02, double c11, double c12, double c22,
                                       double& r)
{
    double q, p;
    cubic_qpr<double>(c00, c01, c02, c11, c12, c22, q, p, r);
    return q + 2.0 * p * dcos(dacos(r) * (1.0 / 3.0));
}

// float: c = cos(acos(r)/3) = P7(s), s = sqrt((1 + r)/2), with P7 a degree-7
// least-squares fit of cos((2/3) acos(s)) on [0, 1] (csrc/gen_eig_poly.py;
// error 1.2e-7 in float32 Horner form).
__device__ inline float lam_max3_poly(float c00, float c01, float c02, float c11, float c12, float c22, float& r)
{
    float q, p;
    cubic_qpr<float>(c00, c01, c02, c11, c12, c22, q, p, r);
    const float s = dsqrt(dmax(0.5f * (1.0f + r), 0.0f));
    float c = 1.138295594e-03f;
    c = dfma(c, s, -6.106058646e-03f);
    c = dfma(c, s, 1.603621716e-02f);
    c = dfma(c, s, -3.019834156e-02f);
    c = dfma(c, s, 5.281414940e-02f);
    c = dfma(c, s, -1.110301883e-01f);
    c = dfma(c, s, 5.773459112e-01f);
    c = dfma(c, s, 5.000000579e-01f);
    return dfma(2.0f * p, c, q);
}

// The float64 recompute of lambda_max from a float32 Jacobian: C = J^T J and
// the trigonometric formula in double.  Out of line: it runs for a handful of
// points per launch and would otherwise raise the register budget of every
// lane.
__device__ __noinline__ float lam_max3_f64_from_J(float j00, float j01, float j02, float j10, float j11,
                                                  float j12, float j20, float j21, float j22)
{
    const double e00 = j00, e01 = j01, e02 = j02, e10 = j10, e11 = j11, e12 = j12;
    const double e20 = j20, e21 = j21, e22 = j22;
    double rd;
    const double lamd = lam_max3_trig(e00 * e00 + e10 * e10 + e20 * e20, e00 * e01 + e10 * e11 + e20 * e21,
                                      e00 * e02 + e10 * e12 + e20 * e22, e01 * e01 + e11 * e11 + e21 * e21,
                                      e01 * e02 + e11 * e12 + e21 * e22, e02 * e02 + e12 * e12 + e22 * e22, rd);
    return (float)lamd;
}

}  // namespace
}  // namespace ftle
