// The paper's own neighbour list as the kernel reads it (Section 2.2): per
// point exactly 2*dim 32-bit indices, one per signed axis direction
// (-x, +x, -y, +y[, -z, +z]), -1 where that side has no neighbour, in the
// caller's point order, with no row pointers (Table 1: 128 / 192 index bits
// per point).  Two kernels stream it:
//
//  - ftle_axis_ell builds the list on the GPU from a one-ring CSR: for each
//    side, the neighbour on that side with the largest cosine to the axis,
//    ties to the smaller index (the list the paper precomputes on the host);
//  - ftle_forward_ell computes the FTLE of every point from the list, one
//    lane per point: the least-squares Jacobian over the present slots, the
//    Cauchy-Green tensor, its largest eigenvalue and the logarithm, in
//    registers.  "direct": every neighbour's coordinates and flow map are
//    gathered from global memory, the paper's layout without reuse (what the
//    caches catch is all the reuse there is); "staged": a workgroup first
//    copies its own block of consecutive points into LDS with coalesced
//    loads and takes neighbours inside the block from there.
//
// Unlike the tiled kernels (ftle_kernels.hip) nothing is reordered: lane i
// handles caller point i, so neighbours are close in memory only as far as
// the caller's numbering makes them so.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ftle_device_math.h"
#include "ftle_internal.h"

namespace ftle {
namespace {

template <int D, typename T> struct Pt;
template <typename T> struct Pt<2, T> { T v[2]; };
template <typename T> struct Pt<3, T> { T v[3]; };

template <int D, typename T>
__device__ inline Pt<D, T> load_pt(const T* __restrict__ a, int64_t i)
{
    Pt<D, T> p;
#pragma unroll
    for (int d = 0; d < D; ++d) p.v[d] = a[i * D + d];
    return p;
}

// The 2*dim indices of point i (2D: one 16-byte load; 3D: three 8-byte loads).
template <int D>
__device__ inline void load_slots(const int32_t* __restrict__ ell, int64_t i, int32_t (&s)[2 * D])
{
    if constexpr (D == 2) {
        const int4 v = reinterpret_cast<const int4*>(ell)[i];
        s[0] = v.x, s[1] = v.y, s[2] = v.z, s[3] = v.w;
    } else {
        const int2* r = reinterpret_cast<const int2*>(ell + i * 6);
        const int2 a = r[0], b = r[1], c = r[2];
        s[0] = a.x, s[1] = a.y, s[2] = b.x, s[3] = b.y, s[4] = c.x, s[5] = c.y;
    }
}

// FTLE of one point from its least-squares sums: M (symmetric, upper
// triangle) and B = sum dphi dx^T.  NaN when M fails the rank test.
__device__ inline float ell_epilogue2(float m00, float m01, float m11, float b00, float b01, float b10, float b11,
                                      float inv2T)
{
    const float det = m00 * m11 - m01 * m01;
    const float trh = (m00 + m11) * 0.5f;
    const bool ok = det > rank_tau<float>() * trh * trh;
    const float id = drcp(det);
    const float j00 = (b00 * m11 - b01 * m01) * id, j01 = (b01 * m00 - b00 * m01) * id;
    const float j10 = (b10 * m11 - b11 * m01) * id, j11 = (b11 * m00 - b10 * m01) * id;
    const float c00 = j00 * j00 + j10 * j10, c01 = j00 * j01 + j10 * j11, c11 = j01 * j01 + j11 * j11;
    const float mm = (c00 + c11) * 0.5f, dd = (c00 - c11) * 0.5f;
    const float lam = mm + dsqrt(dd * dd + c01 * c01);
    return ok ? log_scaled(lam, inv2T) : quiet_nan<float>();
}
__device__ inline double ell_epilogue2(double m00, double m01, double m11, double b00, double b01, double b10,
                                       double b11, double inv2T)
{
    const double det = m00 * m11 - m01 * m01;
    const double trh = (m00 + m11) * 0.5;
    const bool ok = det > rank_tau<double>() * trh * trh;
    const double id = 1.0 / det;
    const double j00 = (b00 * m11 - b01 * m01) * id, j01 = (b01 * m00 - b00 * m01) * id;
    const double j10 = (b10 * m11 - b11 * m01) * id, j11 = (b11 * m00 - b10 * m01) * id;
    const double c00 = j00 * j00 + j10 * j10, c01 = j00 * j01 + j10 * j11, c11 = j01 * j01 + j11 * j11;
    const double mm = (c00 + c11) * 0.5, dd = (c00 - c11) * 0.5;
    const double lam = mm + sqrt(dd * dd + c01 * c01);
    return ok ? log_scaled(lam, inv2T) : quiet_nan<double>();
}

template <typename T>
__device__ inline T ell_epilogue3(const T (&m)[6], const T (&b)[9], T inv2T, float eig_tau, uint32_t& redone)
{
    const T m00 = m[0], m01 = m[1], m02 = m[2], m11 = m[3], m12 = m[4], m22 = m[5];
    const T a00 = m11 * m22 - m12 * m12, a01 = m02 * m12 - m01 * m22, a02 = m01 * m12 - m02 * m11;
    const T a11 = m00 * m22 - m02 * m02, a12 = m01 * m02 - m00 * m12, a22 = m00 * m11 - m01 * m01;
    const T det = m00 * a00 + m01 * a01 + m02 * a02;
    const T tr3 = (m00 + m11 + m22) * T(1.0 / 3.0);
    const bool ok = det > rank_tau<T>() * tr3 * tr3 * tr3;
    const T id = drcp(det);
    T j[9];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const T b0 = b[3 * r], b1 = b[3 * r + 1], b2 = b[3 * r + 2];
        j[3 * r] = (b0 * a00 + b1 * a01 + b2 * a02) * id;
        j[3 * r + 1] = (b0 * a01 + b1 * a11 + b2 * a12) * id;
        j[3 * r + 2] = (b0 * a02 + b1 * a12 + b2 * a22) * id;
    }
    const T c00 = j[0] * j[0] + j[3] * j[3] + j[6] * j[6];
    const T c01 = j[0] * j[1] + j[3] * j[4] + j[6] * j[7];
    const T c02 = j[0] * j[2] + j[3] * j[5] + j[6] * j[8];
    const T c11 = j[1] * j[1] + j[4] * j[4] + j[7] * j[7];
    const T c12 = j[1] * j[2] + j[4] * j[5] + j[7] * j[8];
    const T c22 = j[2] * j[2] + j[5] * j[5] + j[8] * j[8];
    T r, lam;
    if constexpr (sizeof(T) == 4) {
        lam = lam_max3_poly(c00, c01, c02, c11, c12, c22, r);
        if (ok && (r + 1.0f < eig_tau)) {   // top pair nearly equal: float64 from J
            lam = lam_max3_f64_from_J(j[0], j[1], j[2], j[3], j[4], j[5], j[6], j[7], j[8]);
            ++redone;
        }
    } else {
        lam = lam_max3_trig(c00, c01, c02, c11, c12, c22, r);
    }
    return ok ? log_scaled(lam, inv2T) : quiet_nan<T>();
}

// One lane per caller point.  Workgroups take blocks of B consecutive
// points, XCD by XCD in contiguous ranges (xcd_tile), so that a point's
// neighbours in the caller's numbering (the next grid line or plane) are
// mostly in the same XCD's L2.  Slots outside [0, n) (the list's -1) and the
// point itself are replaced by the point itself, whose differences are exact
// zeros: every lane issues all its loads at once, with no branch between
// them.  STAGED: the block's points are first copied to LDS (x then phi, D
// values each) and a neighbour inside the block is read there (the global
// load then reads the lane's own point, already in cache).  (Two or four
// points per lane, to keep more loads in flight, measured no faster.)
template <int D, typename T, bool STAGED, int B>
__global__ void __launch_bounds__(B) ell_kernel(const T* __restrict__ x, const T* __restrict__ flow,
                                                  const int32_t* __restrict__ ell, int64_t n, T inv2T,
                                                  T* __restrict__ out, float eig_tau, unsigned long long* hits)
{
    extern __shared__ __align__(16) unsigned char ell_lds[];
    T* sx = reinterpret_cast<T*>(ell_lds);   // STAGED: [B][D] coordinates, then [B][D] flow map
    T* sf = sx + B * D;
    const int tid = (int)threadIdx.x;
    const int64_t b0 = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * B;
    const int64_t i = b0 + tid;
    if constexpr (STAGED) {
        // coalesced copy of the block's coordinates and flow map
        const int64_t cnt = (n - b0 < B ? n - b0 : B) * D;
        for (int k = tid; k < cnt; k += B) {
            sx[k] = x[b0 * D + k];
            sf[k] = flow[b0 * D + k];
        }
        __syncthreads();
    }
    if (i >= n) return;
    const Pt<D, T> xi = load_pt<D, T>(x, i), fi = load_pt<D, T>(flow, i);
    int32_t s[2 * D];
    load_slots<D>(ell, i, s);
    Pt<D, T> xj[2 * D], fj[2 * D];
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) {
        const int64_t j = ((uint64_t)(int64_t)s[k] < (uint64_t)n) ? (int64_t)s[k] : i;
        if constexpr (STAGED) {
            const uint64_t o = (uint64_t)(j - b0);
            const bool in = o < (uint64_t)B;
            const int64_t g = in ? i : j;
            const uint32_t l = in ? (uint32_t)o : (uint32_t)tid;
            const Pt<D, T> xg = load_pt<D, T>(x, g), fg = load_pt<D, T>(flow, g);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                xj[k].v[d] = in ? sx[l * D + d] : xg.v[d];
                fj[k].v[d] = in ? sf[l * D + d] : fg.v[d];
            }
        } else {
            xj[k] = load_pt<D, T>(x, j);
            fj[k] = load_pt<D, T>(flow, j);
        }
    }
    T f;
    if constexpr (D == 2) {
        T m00 = 0, m01 = 0, m11 = 0, b00 = 0, b01 = 0, b10 = 0, b11 = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const T dx0 = xj[k].v[0] - xi.v[0], dx1 = xj[k].v[1] - xi.v[1];
            const T df0 = fj[k].v[0] - fi.v[0], df1 = fj[k].v[1] - fi.v[1];
            m00 = dfma(dx0, dx0, m00);
            m01 = dfma(dx0, dx1, m01);
            m11 = dfma(dx1, dx1, m11);
            b00 = dfma(df0, dx0, b00);
            b01 = dfma(df0, dx1, b01);
            b10 = dfma(df1, dx0, b10);
            b11 = dfma(df1, dx1, b11);
        }
        f = ell_epilogue2(m00, m01, m11, b00, b01, b10, b11, inv2T);
    } else {
        T m[6] = {0, 0, 0, 0, 0, 0};
        T b[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            T dx[3], df[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                dx[d] = xj[k].v[d] - xi.v[d];
                df[d] = fj[k].v[d] - fi.v[d];
            }
            m[0] = dfma(dx[0], dx[0], m[0]);
            m[1] = dfma(dx[0], dx[1], m[1]);
            m[2] = dfma(dx[0], dx[2], m[2]);
            m[3] = dfma(dx[1], dx[1], m[3]);
            m[4] = dfma(dx[1], dx[2], m[4]);
            m[5] = dfma(dx[2], dx[2], m[5]);
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) b[3 * r + c] = dfma(df[r], dx[c], b[3 * r + c]);
        }
        uint32_t redone = 0;
        f = ell_epilogue3<T>(m, b, inv2T, eig_tau, redone);
        if (hits && redone) atomicAdd(hits, (unsigned long long)redone);
    }
    out[i] = f;
}

// The paper's list from a one-ring CSR, one lane per point, in float64 with
// no contraction of products into FMAs (so that every comparison is the one
// a plain float64 evaluation of the same formula makes).
template <int D, typename T>
__global__ void __launch_bounds__(256) axis_ell_kernel(const T* __restrict__ x, const int64_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col, int64_t n,
                                                         int32_t* __restrict__ ell)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * blockDim.x + threadIdx.x;   // XCD-contiguous
    if (i >= n) return;
    double xi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) xi[d] = (double)x[i * D + d];
    const int64_t p0 = row_ptr[i], p1 = row_ptr[i + 1];
    int32_t best_j[2 * D];
    double best_c[2 * D];
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) {
        best_j[k] = -1;
        best_c[k] = 0.0;
    }
    for (int64_t p = p0; p < p1; ++p) {
        const int32_t j = col[p];
        if ((uint64_t)(int64_t)j >= (uint64_t)n || j == i) continue;   // not a neighbour
        double dx[D];
        double nrm2 = 0.0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            dx[d] = (double)x[(int64_t)j * D + d] - xi[d];
            nrm2 = nrm2 + dx[d] * dx[d];
        }
        const double nrm = sqrt(nrm2);
#pragma unroll
        for (int d = 0; d < D; ++d)
#pragma unroll
            for (int sg = 0; sg < 2; ++sg) {
                const double along = sg ? dx[d] : -dx[d];
                if (!(along > 0.0)) continue;
                const double c = along / nrm;
                const int k = 2 * d + sg;
                if (best_j[k] < 0 || c > best_c[k]) {   // rows ascend: ties keep the smaller index
                    best_c[k] = c;
                    best_j[k] = j;
                }
            }
    }
    if constexpr (D == 2) {
        reinterpret_cast<int4*>(ell)[i] = int4{best_j[0], best_j[1], best_j[2], best_j[3]};
    } else {
        int2* r = reinterpret_cast<int2*>(ell + i * 6);
        r[0] = int2{best_j[0], best_j[1]};
        r[1] = int2{best_j[2], best_j[3]};
        r[2] = int2{best_j[4], best_j[5]};
    }
}

template <int D, typename T>
hipError_t ell_launch(bool staged, const void* x, const void* flow, const int32_t* ell, int64_t n, double inv2T,
                      void* out, double eig_tau, unsigned long long* hits, hipStream_t stream)
{
    constexpr int B = 256;
    const dim3 grid((unsigned)((n + B - 1) / B)), blk(B);
    const T* xp = static_cast<const T*>(x);
    const T* fp = static_cast<const T*>(flow);
    T* op = static_cast<T*>(out);
    if (staged)
        hipLaunchKernelGGL((ell_kernel<D, T, true, B>), grid, blk, 2 * D * B * sizeof(T), stream, xp, fp, ell, n,
                           (T)inv2T, op, (float)eig_tau, hits);
    else
        hipLaunchKernelGGL((ell_kernel<D, T, false, B>), grid, blk, 0, stream, xp, fp, ell, n, (T)inv2T, op,
                           (float)eig_tau, hits);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_forward_ell(int dim, bool f64, bool staged, const void* x, const void* flow, const int32_t* ell,
                              int64_t n, double inv2T, void* out, double eig_tau, unsigned long long* hits,
                              hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    if (dim == 2)
        return f64 ? ell_launch<2, double>(staged, x, flow, ell, n, inv2T, out, eig_tau, hits, stream)
                   : ell_launch<2, float>(staged, x, flow, ell, n, inv2T, out, eig_tau, hits, stream);
    return f64 ? ell_launch<3, double>(staged, x, flow, ell, n, inv2T, out, eig_tau, hits, stream)
               : ell_launch<3, float>(staged, x, flow, ell, n, inv2T, out, eig_tau, hits, stream);
}

hipError_t launch_axis_ell(int dim, bool f64, const void* x, const int64_t* row_ptr, const int32_t* col, int64_t n,
                           int32_t* ell, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256)), blk(256);
#define FTLE_AXIS_LAUNCH(D, T)                                                                                    \
    hipLaunchKernelGGL((axis_ell_kernel<D, T>), grid, blk, 0, stream, static_cast<const T*>(x), row_ptr, col, n, \
                       ell)
    if (dim == 2) {
        if (f64)
            FTLE_AXIS_LAUNCH(2, double);
        else
            FTLE_AXIS_LAUNCH(2, float);
    } else {
        if (f64)
            FTLE_AXIS_LAUNCH(3, double);
        else
            FTLE_AXIS_LAUNCH(3, float);
    }
#undef FTLE_AXIS_LAUNCH
    return hipGetLastError();
}

}  // namespace ftle
