// Flow maps by RK4 advection in a velocity field sampled on a regular grid,
// the form simulation output comes in (the paper's inputs are flow maps
// precomputed from such data, Section 2.2): nodes origin + i spacing per
// axis (x fastest), slices at t_first + k t_step.  The velocity is
// multilinear in space (bilinear in 2D, trilinear in 3D) and linear in time;
// a point outside the grid's box (a time outside the slices) takes the value
// at the nearest point of the box (the nearest slice).  One particle per
// lane, the classical fourth-order Runge-Kutta method in float64 with the
// steps of the analytic flows (ftle_advect.hip).
//
// Read plainly, every evaluation gathers its cell's corner values in two
// slices (64 bytes per particle in 2D) lane by lane, and those gathers bound
// the kernel.  A particle moves less than a cell per step and stays between
// the same two slices for many steps, so each lane keeps its current cell's
// interpolant in registers (float64 polynomial coefficients, slice 0 and the
// change to slice 1) and reads the field only when its cell or slice pair
// changes; an evaluation is then 2^D fused multiply-adds per component for
// the time and 2^D - 1 for the cell.  Against the definition's weighted sum
// of corner values, this and the reciprocal spacings reorder the arithmetic
// at the level of a rounding.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "ftle_internal.h"

namespace ftle {
namespace {

// The field's constants in the form the kernel uses them: reciprocal
// spacings (a multiply in place of a divide; the cell and fraction then
// differ from a divide's by at most a rounding, and the interpolant is
// continuous across cell faces) and strides in elements.
struct GridArgs {
    double origin[3], inv_spacing[3], top[3];   // top: shape - 1
    int cmax[3];                                 // the last cell: shape - 2 (shapes below 2^31)
    int64_t stride[3];                           // elements between nodes along x, y, z
    int64_t slice;                               // elements between slices
    double t_first, inv_t_step, t_top;           // t_top: nt - 1
    int kmax;                                    // nt - 2 (nt below 2^31)
    int two;                                     // more than one slice
};

// The pair of slices bracketing time t: the first one's index and the
// second one's weight (the nearest slice outside the sampled times).
struct SliceWeights {
    int k;
    double w;
};

__device__ inline SliceWeights slice_weights(const GridArgs& g, double t)
{
    SliceWeights r{0, 0.0};
    if (g.two) {
        double s = (t - g.t_first) * g.inv_t_step;
        s = (s > 0.0) ? s : 0.0;   // also NaN
        s = (s > g.t_top) ? g.t_top : s;
        int k = (int)s;            // 0 <= s < 2^31: truncation is the floor
        k = (k > g.kmax) ? g.kmax : k;
        r.k = k;
        r.w = s - (double)k;
    }
    return r;
}

// A lane's current cell and slice pair, with the interpolant read for it.
// In a cell the multilinear interpolant of one component is the polynomial
// sum over corner sets m of a_m prod_{d in m} f_d in the cell fractions f;
// between two slices it is a0 + w (a1 - a0) coefficient by coefficient.  The
// cache holds a0 and a1 - a0 per component, in float64.
template <int D>
struct CellCache {
    static constexpr int kCorners = 1 << D;
    int cell[D];
    int k;
    double a0[D][kCorners], da[D][kCorners];
};

// A cell's corner values (corner m = x bit | y bit << 1 [| z bit << 2]) into
// the polynomial's coefficients: along each axis, the upper corners' values
// less the lower ones'.
template <int D>
__device__ inline void corners_to_coefficients(double* a)
{
#pragma unroll
    for (int d = 0; d < D; ++d)
#pragma unroll
        for (int m = 0; m < (1 << D); ++m)
            if (m & (1 << d)) a[m] -= a[m ^ (1 << d)];
}

// Multilinear velocity at p between the slices of sw, reading the field only
// when p's cell or the slice pair differs from the cached one.
template <int D, bool TWO, typename V>
__device__ inline void grid_velocity(const GridArgs& g, const V* __restrict__ vel, const double* p,
                                     const SliceWeights& sw, CellCache<D>& cc, double* v)
{
    constexpr int kCorners = CellCache<D>::kCorners;
    double f[3] = {0.0, 0.0, 0.0};
    int c[3] = {0, 0, 0};
    bool miss = sw.k != cc.k;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double u = (p[d] - g.origin[d]) * g.inv_spacing[d];
        u = (u > 0.0) ? u : 0.0;   // also NaN
        u = (u > g.top[d]) ? g.top[d] : u;
        int cd = (int)u;           // 0 <= u < 2^31: truncation is the floor
        cd = (cd > g.cmax[d]) ? g.cmax[d] : cd;
        f[d] = u - (double)cd;
        c[d] = cd;
        miss |= cd != cc.cell[d];
    }
    if (miss) {
        int64_t base = (int64_t)sw.k * g.slice;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            base += (int64_t)c[d] * g.stride[d];
            cc.cell[d] = c[d];
        }
        cc.k = sw.k;
        // each cell row along x: the two x neighbours' components, 2 D
        // consecutive values of the field
        int64_t row[kCorners / 2];
#pragma unroll
        for (int r = 0; r < kCorners / 2; ++r)
            row[r] = base + ((r & 1) ? g.stride[1] : 0) + ((D == 3 && (r & 2)) ? g.stride[2] : 0);
#pragma unroll
        for (int r = 0; r < kCorners / 2; ++r)
#pragma unroll
            for (int e = 0; e < 2 * D; ++e) cc.a0[e % D][2 * r + e / D] = (double)vel[row[r] + e];
        if (TWO) {
#pragma unroll
            for (int r = 0; r < kCorners / 2; ++r)
#pragma unroll
                for (int e = 0; e < 2 * D; ++e) cc.da[e % D][2 * r + e / D] = (double)vel[row[r] + g.slice + e];
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            corners_to_coefficients<D>(cc.a0[d]);
            if (TWO) {
                corners_to_coefficients<D>(cc.da[d]);
#pragma unroll
                for (int m = 0; m < kCorners; ++m) cc.da[d][m] -= cc.a0[d][m];
            }
        }
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double a[kCorners];
#pragma unroll
        for (int m = 0; m < kCorners; ++m) a[m] = TWO ? cc.a0[d][m] + sw.w * cc.da[d][m] : cc.a0[d][m];
        // the polynomial in f, the highest axis folded first
#pragma unroll
        for (int e = D - 1; e >= 0; --e)
#pragma unroll
            for (int m = 0; m < kCorners; ++m)
                if (!(m & (1 << e)) && m < (1 << e)) a[m] += f[e] * a[m | (1 << e)];
        v[d] = a[0];
    }
}

template <int D, bool TWO, typename T, typename V>
__global__ void __launch_bounds__(256) advect_grid_kernel(GridArgs g, const V* __restrict__ vel, int64_t n,
                                                          const T* __restrict__ x0, const double* __restrict__ t0s,
                                                          const double* __restrict__ Ts, double t0, double Tall,
                                                          double dt, T* __restrict__ phi)
{
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
    CellCache<D> cc;
    cc.k = -1;   // no cell read yet
#pragma unroll
    for (int d = 0; d < D; ++d) cc.cell[d] = -1;
    for (int64_t s = 0; s < ns; ++s) {
        const double t = ti + (double)s * h;
        const SliceWeights w0 = slice_weights(g, t), wh = slice_weights(g, t + 0.5 * h),
                           w1 = slice_weights(g, t + h);
        grid_velocity<D, TWO>(g, vel, p, w0, cc, k1);
#pragma unroll
        for (int d = 0; d < D; ++d) q[d] = p[d] + 0.5 * h * k1[d];
        grid_velocity<D, TWO>(g, vel, q, wh, cc, k2);
#pragma unroll
        for (int d = 0; d < D; ++d) q[d] = p[d] + 0.5 * h * k2[d];
        grid_velocity<D, TWO>(g, vel, q, wh, cc, k3);
#pragma unroll
        for (int d = 0; d < D; ++d) q[d] = p[d] + h * k3[d];
        grid_velocity<D, TWO>(g, vel, q, w1, cc, k4);
#pragma unroll
        for (int d = 0; d < D; ++d) p[d] += h / 6.0 * (k1[d] + 2.0 * k2[d] + 2.0 * k3[d] + k4[d]);
    }
#pragma unroll
    for (int d = 0; d < D; ++d) phi[i * D + d] = (T)p[d];
}

template <int D, typename T, typename V>
hipError_t advect_grid_launch(const GridField& g, const void* vel, int64_t n, const void* x0, const double* t0s,
                              const double* Ts, double t0, double T_, double dt, void* phi, hipStream_t stream)
{
    GridArgs a{};
    int64_t stride = D;
    for (int d = 0; d < D; ++d) {
        a.origin[d] = g.origin[d];
        a.inv_spacing[d] = 1.0 / g.spacing[d];
        a.top[d] = (double)(g.shape[d] - 1);
        a.cmax[d] = (int)(g.shape[d] - 2);
        a.stride[d] = stride;
        stride *= g.shape[d];
    }
    a.slice = stride;
    a.t_first = g.t_first;
    a.two = g.nt > 1;
    a.inv_t_step = a.two ? 1.0 / g.t_step : 0.0;
    a.t_top = (double)(g.nt - 1);
    a.kmax = (int)(g.nt - 2);
    const int64_t blocks = (n + 255) / 256;
    auto kernel = a.two ? advect_grid_kernel<D, true, T, V> : advect_grid_kernel<D, false, T, V>;
    hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(256), 0, stream, a,
                       static_cast<const V*>(vel), n, static_cast<const T*>(x0), t0s, Ts, t0, T_, dt,
                       static_cast<T*>(phi));
    return hipGetLastError();
}

}  // namespace

hipError_t launch_advect_grid(int dim, const GridField& g, const void* vel, bool vel_f64, bool f64, int64_t n,
                              const void* x0, const double* t0s, const double* Ts, double t0, double T, double dt,
                              void* phi, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
#define FTLE_GRID(D, TT, VV) advect_grid_launch<D, TT, VV>(g, vel, n, x0, t0s, Ts, t0, T, dt, phi, stream)
    if (dim == 2) {
        if (f64) return vel_f64 ? FTLE_GRID(2, double, double) : FTLE_GRID(2, double, float);
        return vel_f64 ? FTLE_GRID(2, float, double) : FTLE_GRID(2, float, float);
    }
    if (f64) return vel_f64 ? FTLE_GRID(3, double, double) : FTLE_GRID(3, double, float);
    return vel_f64 ? FTLE_GRID(3, float, double) : FTLE_GRID(3, float, float);
#undef FTLE_GRID
}

}  // namespace ftle
