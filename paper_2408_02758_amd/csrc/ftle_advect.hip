// Flow maps by advection on the GPU: the step before the FTLE path.  The
// paper's inputs are flow maps precomputed by an advection code (UVaFTLE,
// Section 2.2); this computes them for analytic velocity fields, one particle
// per lane, by the classical fourth-order Runge-Kutta method in float64.
//
// Flows (their definitions, not anyone's code):
//  - the double gyre of Shadden, Lekien and Marsden (Physica D 212, 2005):
//    stream function psi = A sin(pi f) sin(pi y), f = eps sin(omega t) x^2 +
//    (1 - 2 eps sin(omega t)) x, velocity (-dpsi/dy, dpsi/dx);
//  - the steady Arnold-Beltrami-Childress flow
//    (A sin z + C cos y, B sin x + A cos z, C sin y + B cos x).
//
// A particle takes max(1, ceil(|T|/dt - 1e-9)) steps of T/steps from t0; a
// particle whose duration is not finite or needs more than kMaxAdvectSteps
// steps gets NaN without stepping (the host rejects such a common T).
// The work is arithmetic (transcendentals) on registers: one 2-3 value load
// and one store per particle.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "ftle_internal.h"

namespace ftle {
namespace {

struct FlowParams {
    double a, b, c;
};

// Velocity at p, with w the double gyre's time factor sin(omega t) at the
// stage's time (the steady ABC flow ignores it).
template <int KIND>
__device__ inline void flow_velocity(const FlowParams& pr, const double* p, double w, double* v)
{
    constexpr double kPi = 3.14159265358979323846;
    if constexpr (KIND == 0) {
        double cy, sy, sf, cf;
        const double a = pr.b * w, b = 1.0 - 2.0 * pr.b * w;
        const double f = (a * p[0] + b) * p[0];
        const double dfdx = 2.0 * a * p[0] + b;
        sincospi(p[1], &sy, &cy);
        sincospi(f, &sf, &cf);
        v[0] = -kPi * pr.a * sf * cy;
        v[1] = kPi * pr.a * cf * sy * dfdx;
    } else {
        double sx, cx, sy, cy, sz, cz;
        sincos(p[0], &sx, &cx);
        sincos(p[1], &sy, &cy);
        sincos(p[2], &sz, &cz);
        v[0] = pr.a * sz + pr.c * cy;
        v[1] = pr.b * sx + pr.a * cz;
        v[2] = pr.c * sy + pr.b * cx;
    }
}

// The four stages of a step take the double gyre's time factor sin(omega t)
// at t, t + h/2 (twice) and t + h.  (sin, cos)(omega t) advance by rotations
// through the half step's angle omega h / 2, two per step, and are evaluated
// directly every kAnchor steps: a rotation with rounded coefficients moves the
// pair by a few units in the last place, so the drift stays below 10^-13,
// far under the RK4 truncation error, at two multiplies and two FMAs per
// stage time instead of a sine.
constexpr int kAnchor = 32;

template <int KIND, typename T>
__global__ void __launch_bounds__(256) advect_kernel(FlowParams pr, int64_t n, const T* __restrict__ x0,
                                                     const double* __restrict__ t0s, const double* __restrict__ Ts,
                                                     double t0, double Tall, double dt, T* __restrict__ phi)
{
    constexpr int D = KIND == 0 ? 2 : 3;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double p[D], q[D], k1[D], k2[D], k3[D], k4[D];
#pragma unroll
    for (int d = 0; d < D; ++d) p[d] = (double)x0[i * D + d];
    const double ti = t0s ? t0s[i] : t0;
    const double Ti = Ts ? Ts[i] : Tall;
    const double steps = fmax(1.0, ceil(fabs(Ti) / dt - 1e-9));
    if (!(steps <= (double)kMaxAdvectSteps)) {   // also NaN and inf
#pragma unroll
        for (int d = 0; d < D; ++d) phi[i * D + d] = (T)NAN;
        return;
    }
    const double h = Ti / steps;
    const int64_t ns = (int64_t)steps;
    double rs = 0.0, rc = 1.0, sw = 0.0, cw = 1.0;   // rotation by omega h / 2; factor pair at the step's start
    if constexpr (KIND == 0) sincos(pr.c * (0.5 * h), &rs, &rc);
    for (int64_t s = 0; s < ns; ++s) {
        double wh = 0.0, w1 = 0.0;
        if constexpr (KIND == 0) {
            if (s % kAnchor == 0) sincos(pr.c * (ti + (double)s * h), &sw, &cw);
            const double sh = sw * rc + cw * rs, chf = cw * rc - sw * rs;
            const double s1 = sh * rc + chf * rs, c1 = chf * rc - sh * rs;
            wh = sh;
            w1 = s1;
            flow_velocity<KIND>(pr, p, sw, k1);
            sw = s1;
            cw = c1;
        } else {
            flow_velocity<KIND>(pr, p, 0.0, k1);
        }
#pragma unroll
        for (int d = 0; d < D; ++d) q[d] = p[d] + 0.5 * h * k1[d];
        flow_velocity<KIND>(pr, q, wh, k2);
#pragma unroll
        for (int d = 0; d < D; ++d) q[d] = p[d] + 0.5 * h * k2[d];
        flow_velocity<KIND>(pr, q, wh, k3);
#pragma unroll
        for (int d = 0; d < D; ++d) q[d] = p[d] + h * k3[d];
        flow_velocity<KIND>(pr, q, w1, k4);
#pragma unroll
        for (int d = 0; d < D; ++d) p[d] += h / 6.0 * (k1[d] + 2.0 * k2[d] + 2.0 * k3[d] + k4[d]);
    }
#pragma unroll
    for (int d = 0; d < D; ++d) phi[i * D + d] = (T)p[d];
}

template <int KIND, typename T>
hipError_t advect_launch(const FlowParams& pr, int64_t n, const void* x0, const double* t0s, const double* Ts,
                         double t0, double T_, double dt, void* phi, hipStream_t stream)
{
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL((advect_kernel<KIND, T>), dim3((unsigned)blocks), dim3(256), 0, stream, pr, n,
                       static_cast<const T*>(x0), t0s, Ts, t0, T_, dt, static_cast<T*>(phi));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_advect(int kind, const double* params, bool f64, int64_t n, const void* x0, const double* t0s,
                         const double* Ts, double t0, double T, double dt, void* phi, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const FlowParams pr{params[0], params[1], params[2]};
    if (kind == 0)
        return f64 ? advect_launch<0, double>(pr, n, x0, t0s, Ts, t0, T, dt, phi, stream)
                   : advect_launch<0, float>(pr, n, x0, t0s, Ts, t0, T, dt, phi, stream);
    return f64 ? advect_launch<1, double>(pr, n, x0, t0s, Ts, t0, T, dt, phi, stream)
               : advect_launch<1, float>(pr, n, x0, t0s, Ts, t0, T, dt, phi, stream);
}

}  // namespace ftle
