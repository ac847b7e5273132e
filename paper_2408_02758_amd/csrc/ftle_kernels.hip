// HIP kernels of the FTLE library (gfx950 / CDNA4, wave64).
//
// Per mesh point i (the per-point FTLE kernel of UVaFTLE, Section 2 of de
// Castro et al.; Table 1 sizes its core):
//   M = sum_j dx dx^T,  B = sum_j dphi dx^T   (j over the stencil S(i),
//   dx = x_j - x_i, dphi = phi_j - phi_i), J = B M^{-1},
//   C = J^T J, lambda = lambda_max(C), FTLE = ln(lambda) / (2 |T|).
//
// Design for the MI355X memory system:
//  - The paper finds the gather of neighbour data to be the bottleneck
//    (Section 2.2: irregular accesses with little reuse).  Here points are in
//    Morton order and cut into tiles; a workgroup stages its tile's points
//    and their one-ring halo (coordinates and flow map) into LDS with
//    batched gathers, so each value comes from HBM about once, and the
//    stencil walk reads LDS only.
//  - The neighbour list (Section 2.2: precomputed on the host, read in a
//    fixed order) is stored per tile, compressed (ftle_internal.h): the
//    staged points' caller indices as runs of consecutive indices, and the
//    stencil as 10-bit indices of the neighbours' staged slots, three per
//    32-bit word, kept only for rows that are not the previous row shifted
//    by one slot.  The record is copied to LDS whole and decoded there.
//    Rows are padded to a multiple of three with the point itself (which
//    adds exact zeros), so the walk reads three neighbours per 32-bit LDS
//    load with no per-entry select.
//  - A lane computes one point at a time (a workgroup of B lanes walks its
//    tile's P points in steps of B); Jacobian, tensor, eigenvalue and
//    logarithm stay in registers.  No MFMA: per point the work is a few
//    dozen multiply-adds over a gathered stencil, not a dense contraction.
//  - Consecutive workgroup ids land on different XCDs; tiles are remapped so
//    that each XCD walks a contiguous stretch of the Morton order and halo
//    reuse happens in its own L2.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include <cmath>
#include <cstdint>
#include <type_traits>
#include <atomic>

#include "ftle_device_math.h"
#include "ftle_internal.h"

namespace ftle {
namespace {

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------
template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };
template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };
template <typename T> using vec2_t = typename Vec2<T>::type;
template <typename T> using vec4_t = typename Vec4<T>::type;

template <typename T> struct Packed3 { T a, b, c; };

// LDS by byte address.  No kernel here declares static LDS: all of it is the
// dynamic allocation, which then starts at LDS address 0, so staged data have
// plain 32-bit addresses whose constant parts fold into the instruction's
// offset field.  Vectors move as native (ext_vector_type) vectors.
template <typename T, int N> using native_vec = T __attribute__((ext_vector_type(N)));
template <typename V> struct LdsIo {   // scalars
    __device__ static V ld(uint32_t a) { return *(const __attribute__((address_space(3))) V*)(size_t)a; }
    __device__ static void st(uint32_t a, const V v) { *(__attribute__((address_space(3))) V*)(size_t)a = v; }
};
template <typename T> struct LdsIo<HIP_vector_type<T, 2>> {
    using N = native_vec<T, 2>;
    __device__ static HIP_vector_type<T, 2> ld(uint32_t a)
    {
        const N v = *(const __attribute__((address_space(3))) N*)(size_t)a;
        return HIP_vector_type<T, 2>{v[0], v[1]};
    }
    __device__ static void st(uint32_t a, const HIP_vector_type<T, 2> v)
    {
        *(__attribute__((address_space(3))) N*)(size_t)a = N{v.x, v.y};
    }
};
template <typename T> struct LdsIo<HIP_vector_type<T, 4>> {
    using N = native_vec<T, 4>;
    __device__ static HIP_vector_type<T, 4> ld(uint32_t a)
    {
        const N v = *(const __attribute__((address_space(3))) N*)(size_t)a;
        return HIP_vector_type<T, 4>{v[0], v[1], v[2], v[3]};
    }
    __device__ static void st(uint32_t a, const HIP_vector_type<T, 4> v)
    {
        *(__attribute__((address_space(3))) N*)(size_t)a = N{v.x, v.y, v.z, v.w};
    }
};
template <typename V> __device__ inline V lds_ld(uint32_t a) { return LdsIo<V>::ld(a); }
template <typename V> __device__ inline void lds_st(uint32_t a, const V v) { LdsIo<V>::st(a, v); }

// ---------------------------------------------------------------------------
// Staged points in LDS, from the launch's base address lds0; staged slot l
// (l is the stencil's local index), e = sizeof(T):
//   forward 2D: (x0, x1, phi0, phi1) at 4e l
//   forward 3D: (x0, x1), (x2, phi0), (phi1, phi2) at 2e l + {0, 1, 2} F,
//               F = 2e kMaxStaged (a fixed stride: one address per neighbour
//               reaches all three through the instruction's offset field)
//   adjoint 2D: (x0, x1, w0, w1) (h0, h1, -, -) at 8e l
//   adjoint 3D: (x0, x1, x2, h0), (h1, h2, w0, w1) at 4e l + {0, 1} A and
//               w2 at 2 A + e l, A = 4e bwd3_capacity
// so that 16-byte reads are 16-byte aligned and neighbouring points sit in
// neighbouring banks.  A copy of the tile's record follows.
// ---------------------------------------------------------------------------
template <int D, typename T> struct Layout {
    static constexpr uint32_t e = sizeof(T);
    static constexpr uint32_t unit = (D == 2 ? 4 : 2) * e;
    static constexpr uint32_t stride = kMaxStaged * 2 * e;   // 3D forward: array stride
    static constexpr uint32_t bunit = 4 * e;                                   // 3D adjoint: slot of the 4-value arrays
    static constexpr uint32_t bstride = (uint32_t)bwd3_capacity(e == 8) * bunit;   // and their stride
    // LDS address of the record copy after the staged points
    static __device__ uint32_t fwd_rec(uint32_t lds0, int S) { return lds0 + (uint32_t)fwd_points_bytes(D, e == 8, S); }
    static __device__ uint32_t bwd_rec(uint32_t lds0, int S) { return lds0 + (uint32_t)bwd_points_bytes(D, e == 8, S); }
};

// Copy of a tile's record (n16 chunks of 16 bytes) into LDS as a direct
// global -> LDS transfer
// (global_load_lds_dwordx4): each wave moves 64 consecutive 16-byte chunks to
// consecutive LDS chunks without passing through registers, so the copy stays
// in flight while the wave issues other instructions.  The caller waits
// (vmcnt 0) and synchronises the workgroup before reading dst.
template <int B>
__device__ inline void dma_record(const uint4* __restrict__ src, uint32_t dst, int n16, int tid)
{
    const int lane = tid & 63;
    for (int c0 = tid - lane; c0 < n16; c0 += B) {   // wave-uniform chunk base
        if (c0 + lane < n16)
            __builtin_amdgcn_global_load_lds(src + c0 + lane,
                                             (__attribute__((address_space(3))) void*)(size_t)(dst + 16u * c0), 16, 0, 0);
    }
}

// Element `i` of an array of records of `bytes` bytes, addressed with a 32-bit
// byte offset from a uniform base (one shift per access) unless WIDE.
template <bool WIDE, typename V, typename P>
__device__ inline V rec_at(const P* base, uint32_t i, uint32_t bytes)
{
    if constexpr (WIDE)
        return *reinterpret_cast<const V*>(reinterpret_cast<const unsigned char*>(base) + (uint64_t)i * bytes);
    else
        return *reinterpret_cast<const V*>(reinterpret_cast<const unsigned char*>(base) + i * bytes);
}
template <bool WIDE, typename V, typename P>
__device__ inline void rec_put(P* base, uint32_t i, uint32_t bytes, const V v)
{
    if constexpr (WIDE)
        *reinterpret_cast<V*>(reinterpret_cast<unsigned char*>(base) + (uint64_t)i * bytes) = v;
    else
        *reinterpret_cast<V*>(reinterpret_cast<unsigned char*>(base) + i * bytes) = v;
}

// Walk of one row of the padded stencil, WPS words (3 WPS neighbours) per
// step: the words' LDS loads, then the neighbours' slot loads, then the
// arithmetic; a final single word.  visit(pad, l...) gets the local indices
// and the padding count of the step's last word (its bits 30-31): a zero
// constant except for the row's last word, visited first when PAD and as the
// final single word otherwise.
template <int K> using IntK = std::integral_constant<int, K>;

template <int WPS, bool PAD, typename F>
__device__ inline void walk_row(uint32_t words, int s, int e, F&& visit)
{
    // one bit-field extract per entry; written as an instruction because the
    // compiler otherwise merges the extract into the caller's address scaling
    // as shift, mask and add (three operations instead of extract + shift-add)
    auto ix = [](uint32_t w, auto k) {
        uint32_t r;
        asm("v_bfe_u32 %0, %1, %2, 10" : "=v"(r) : "v"(w), "i"(10 * decltype(k)::value));
        return r;
    };
    using Zero = std::integral_constant<uint32_t, 0>;
    uint32_t a = words + 4u * s;   // the loop runs on the LDS address
    uint32_t end = words + 4u * e;
    if constexpr (PAD) {
        // the row's last word first, with its padding count (no other word
        // holds padding); an empty row visits a placeholder word of three
        // slot-0 entries, all padding (pad 3; its reads stay inside the
        // staged points).  Unconditional, so that the accumulators enter the
        // loop as values, not as constants the compiler materialises on both
        // of its edges.
        const bool any = e > s;
        end -= any ? 4u : 0u;
        const uint32_t w0 = any ? lds_ld<uint32_t>(end) : 0u;
        visit(any ? w0 >> 30 : 3u, ix(w0, IntK<0>{}), ix(w0, IntK<1>{}), ix(w0, IntK<2>{}));
    }
    if constexpr (WPS == 2) {
        for (; a + 8u <= end; a += 8u) {
            const uint32_t w0 = lds_ld<uint32_t>(a), w1 = lds_ld<uint32_t>(a + 4u);
            visit(Zero{}, ix(w0, IntK<0>{}), ix(w0, IntK<1>{}), ix(w0, IntK<2>{}), ix(w1, IntK<0>{}),
                  ix(w1, IntK<1>{}), ix(w1, IntK<2>{}));
        }
    }
    for (; a < end; a += 4u) {
        const uint32_t w0 = lds_ld<uint32_t>(a);
        if constexpr (PAD) {
            visit(Zero{}, ix(w0, IntK<0>{}), ix(w0, IntK<1>{}), ix(w0, IntK<2>{}));
        } else {
            // with two words a step this single word, when there is one, is
            // the row's last: its padding is skipped when the active lanes'
            // rows all end in padding there (the 2D rows of 7 and 8 entries)
            // (at most 2 padding entries: the first entry is always live)
            visit(min(w0 >> 30, 2u), ix(w0, IntK<0>{}), ix(w0, IntK<1>{}), ix(w0, IntK<2>{}));
        }
    }
}

// Entry k of the N a walk step visits holds a neighbour, not the row's
// padding (the last pad entries of the row's last word; pad 3: all of an
// empty row's placeholder word).  The padding's
// arithmetic is skipped by a branch that whole waves take when their rows
// end alike (in 3D: 14 neighbours, one padding entry).
template <int N, typename P> __device__ inline bool entry_live(int k, P pad)
{
    return k < N - 3 || (uint32_t)(N - k) > (uint32_t)pad;
}

// Decoding of a tile record held in LDS at address rec (layout R).
// Caller index of staged slot l: its run is the last one starting at or
// before l.
__device__ inline uint32_t slot_point(uint32_t rec, const RecLayout& R, int l)
{
    const int g = l >> 5;
    const uint32_t m = lds_ld<uint32_t>(rec + R.smask + 4u * g) & (0xffffffffu >> (31 - (l & 31)));
    const int r = (int)lds_ld<uint16_t>(rec + R.spre + 2u * g) + __popc(m) - 1;
    return lds_ld<uint32_t>(rec + R.runs + 4u * r) + (uint32_t)l;
}

// Row of own slot l: the words [s, e) of its anchor (the last explicit row
// a <= l) and the shift l - a that every entry takes.
struct RowRef {
    int s, e, shift;
};
__device__ inline RowRef row_ref(uint32_t rec, const RecLayout& R, int l)
{
    const int q = l >> 5;
    const uint32_t m = lds_ld<uint32_t>(rec + R.xmask + 4u * q) & (0xffffffffu >> (31 - (l & 31)));
    const int pre = lds_ld<uint16_t>(rec + R.xpre + 2u * q);
    const int last = lds_ld<uint16_t>(rec + R.xlast + 2u * q);
    const int a = m ? (q << 5) + 31 - __clz((int)m) : last;
    const int k = pre + __popc(m) - 1;   // explicit row number of a
    const int s = k ? lds_ld<uint16_t>(rec + R.xend + 2u * (k - 1)) : 0;
    const int e = lds_ld<uint16_t>(rec + R.xend + 2u * k);
    return RowRef{s, e, l - a};
}

// ---------------------------------------------------------------------------
// Staging of the tile's points (own + halo) into their LDS slots, once the
// record is in LDS.  One round stages K slots per thread: K caller indices
// decoded from the record, then the 2K gathers (coordinates and flow map),
// then the K LDS stores.  K is a compile-time constant and the loads and
// stores are unconditional, so the compiler counts outstanding loads exactly:
// one gather round trip per round.  (With loads under per-slot branches it
// must wait for all outstanding loads before each gather.)  Lanes past the
// last slot S-1 load slot S-1's point and store the same values to it again.
// ---------------------------------------------------------------------------
template <int D, typename T, int B, bool WIDE, int K>
__device__ inline void fwd_stage(uint32_t rec, const RecLayout& R, const T* __restrict__ x,
                                 const T* __restrict__ flow, int S, int r0, uint32_t lds0, int tid)
{
    using V2 = vec2_t<T>;
    using V4 = vec4_t<T>;
    using L = Layout<D, T>;
    const int base = r0 + tid;
    uint32_t u[K];
#pragma unroll
    for (int k = 0; k < K; ++k) u[k] = slot_point(rec, R, min(base + k * B, S - 1));
    if constexpr (D == 2) {
        V2 xv[K], fv[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            xv[k] = rec_at<WIDE, V2>(x, u[k], sizeof(V2));
            fv[k] = rec_at<WIDE, V2>(flow, u[k], sizeof(V2));
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t o = (uint32_t)min(base + k * B, S - 1) * L::unit;
            lds_st(lds0 + o, V4{xv[k].x, xv[k].y, fv[k].x, fv[k].y});
        }
    } else {
        Packed3<T> xv[K], fv[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            xv[k] = rec_at<WIDE, Packed3<T>>(x, u[k], sizeof(Packed3<T>));
            fv[k] = rec_at<WIDE, Packed3<T>>(flow, u[k], sizeof(Packed3<T>));
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t o = lds0 + (uint32_t)min(base + k * B, S - 1) * L::unit;
            lds_st(o, V2{xv[k].a, xv[k].b});
            lds_st(o + L::stride, V2{xv[k].c, fv[k].a});
            lds_st(o + 2 * L::stride, V2{fv[k].b, fv[k].c});
        }
    }
}


// Rounds over S staged slots: full rounds of kMaxK slots per thread, then one
// round of the K (1..kMaxK) the rest needs.  K is workgroup-uniform, so the
// switch is a scalar branch and each case is straight-line code.
constexpr int kMaxK = 4;
template <int B, typename F>
__device__ inline void stage_points(int S, F&& round)
{
    int r0 = 0;
    for (; S - r0 > kMaxK * B; r0 += kMaxK * B) round(IntK<kMaxK>{}, r0);
    switch ((S - r0 + B - 1) / B) {
    case 1: round(IntK<1>{}, r0); break;
    case 2: round(IntK<2>{}, r0); break;
    case 3: round(IntK<3>{}, r0); break;
    default: round(IntK<4>{}, r0); break;
    }
}

// ---------------------------------------------------------------------------
// One tile of the forward pass.  OUT: write FTLE.  TAPE: write the adjoint
// tape: p = J v / (|T| lambda) and h = M^{-1} v, with v the unit top
// eigenvector of C (TAPE 1), and also sigma = h . sum_j dx (TAPE 2; with a
// symmetric stencil the adjoint forms sigma itself).
// ---------------------------------------------------------------------------
// Staging of a forward tile by the workgroup's B threads (tid in [0, B)) into
// the LDS region at lds0: the record straight to LDS, then the staged points
// in rounds of K slots per thread (fwd_stage).  The caller waits (vmcnt 0)
// and synchronises before the compute.
template <int D, typename T, int B, bool WIDE>
__device__ __forceinline__ void fwd_stage_tile(const TileMeta m, const uint4* __restrict__ rec,
                                               const T* __restrict__ x, const T* __restrict__ flow,
                                               const uint32_t lds0, const int tid)
{
    using L = Layout<D, T>;
    const int S = (int)m.P + (int)m.H;
    const RecLayout R = rec_layout(m);
    const uint32_t recl = L::fwd_rec(lds0, S);   // LDS address of the record
    dma_record<B>(rec + m.rec_off, recl, (int)(R.bytes / 16), tid);
    __builtin_amdgcn_s_waitcnt(0);   // this wave's part of the record has landed in LDS
    __syncthreads();
    stage_points<B>(S, [&](auto kc, int r0) {
        fwd_stage<D, T, B, WIDE, decltype(kc)::value>(recl, R, x, flow, S, r0, lds0, tid);
    });
}

// The compute of a staged forward tile by B threads (tid in [0, B)).
template <int D, typename T, bool OUT, int TAPE, int B, bool WIDE>
__device__ __forceinline__ void fwd_compute_tile(const TileMeta m, const T* __restrict__ minv, const T inv2T,
                                                 T* __restrict__ out, T* __restrict__ tape, const int64_t n,
                                                 const float eig_tau, unsigned long long* hits, const uint32_t lds0,
                                                 const int tid)
{
    using V2 = vec2_t<T>;
    using V4 = vec4_t<T>;
    using L = Layout<D, T>;
    const int P = (int)m.P;
    const int S = P + (int)m.H;
    const RecLayout R = rec_layout(m);
    const uint32_t recl = L::fwd_rec(lds0, S);   // LDS address of the record
    const uint32_t words = recl;
    uint32_t redone = 0;   // points of this lane that took the float64 recompute
    for (int l = tid; l < P; l += B) {
        const RowRef row = row_ref(recl, R, l);
        const int s = row.s, e = row.e;
        const uint32_t sh = (uint32_t)row.shift * L::unit;   // the row's entries are its anchor's plus shift
        uint32_t u;   // caller index of slot l, decoded after the walk (one register less in it)
        const uint32_t oself = (uint32_t)l * L::unit;
        T f;
        if constexpr (D == 2) {
            const V4 c0 = lds_ld<V4>(lds0 + oself);
            T m00 = 0, m01 = 0, m11 = 0, b00 = 0, b01 = 0, b10 = 0, b11 = 0, s0 = 0, s1 = 0;
            auto acc = [&](const V4 q) {
                const T dx0 = q.x - c0.x, dx1 = q.y - c0.y;
                const T df0 = q.z - c0.z, df1 = q.w - c0.w;
                m00 = dfma(dx0, dx0, m00);
                m01 = dfma(dx0, dx1, m01);
                m11 = dfma(dx1, dx1, m11);
                b00 = dfma(df0, dx0, b00);
                b01 = dfma(df0, dx1, b01);
                b10 = dfma(df1, dx0, b10);
                b11 = dfma(df1, dx1, b11);
                if constexpr (TAPE == 2) {
                    s0 += dx0;
                    s1 += dx1;
                }
            };
            const uint32_t b0 = lds0 + sh;
            auto at = [&](uint32_t j) { return lds_ld<V4>(b0 + j * L::unit); };
            walk_row<2, false>(words, s, e, [&](auto pad, auto... o) {
                constexpr int N = sizeof...(o);
                const V4 q[] = {at(o)...};
#pragma unroll
                for (int k = 0; k < N; ++k)
                    if (entry_live<N>(k, pad)) acc(q[k]);
            });
            u = slot_point(recl, R, l);
            const T det = m00 * m11 - m01 * m01;
            const T trh = (m00 + m11) * T(0.5);
            const bool ok = det > rank_tau<T>() * trh * trh;
            const T id = drcp(det);
            const T j00 = (b00 * m11 - b01 * m01) * id, j01 = (b01 * m00 - b00 * m01) * id;
            const T j10 = (b10 * m11 - b11 * m01) * id, j11 = (b11 * m00 - b10 * m01) * id;
            const T c00 = j00 * j00 + j10 * j10, c01 = j00 * j01 + j10 * j11, c11 = j01 * j01 + j11 * j11;
            const T mm = (c00 + c11) * T(0.5), dd = (c00 - c11) * T(0.5);
            const T hh = dsqrt(dd * dd + c01 * c01);
            const T lam = mm + hh;
            f = ok ? log_scaled(lam, inv2T) : quiet_nan<T>();
            if constexpr (TAPE) {
                T v0 = (dd >= T(0)) ? dd + hh : c01;
                T v1 = (dd >= T(0)) ? c01 : hh - dd;
                const T nv2 = v0 * v0 + v1 * v1;
                if (nv2 > T(0)) {
                    const T iv = drcp(dsqrt(nv2));
                    v0 *= iv;
                    v1 *= iv;
                } else {
                    v0 = T(1);
                    v1 = T(0);
                }
                const bool use = ok && (lam > T(0)) && isfinite(f);
                // a point without a usable FTLE (rank-deficient stencil, non-
                // finite values) puts zeros on the tape: selects, not products
                // with zero, since J may hold NaN there
                const T sc = T(2) * inv2T * drcp(lam);
                const T p0 = use ? (j00 * v0 + j01 * v1) * sc : T(0), p1 = use ? (j10 * v0 + j11 * v1) * sc : T(0);
                const T h0 = use ? (m11 * v0 - m01 * v1) * id : T(0);
                const T h1 = use ? (m00 * v1 - m01 * v0) * id : T(0);
                rec_put<WIDE>(tape, u, sizeof(V4), V4{p0, p1, h0, h1});
                if constexpr (TAPE == 2) rec_put<WIDE>(tape + (size_t)n * 4, u, sizeof(T), h0 * s0 + h1 * s1);
            }
        } else {
            // The tape kernels take M^-1 from the mesh (host-computed in float64
            // from the coordinates alone; NaN where M is rank deficient) and
            // accumulate B only: 6 FMAs per neighbour and the adjugate fewer.
            // The plain forward forms M itself, which measured faster where
            // the launch is bound by memory as much as by arithmetic.
            constexpr bool kMinv = TAPE != 0;
            Packed3<T> ia{}, ib{};
            auto load_minv = [&] {
                u = slot_point(recl, R, l);
                ia = rec_at<WIDE, Packed3<T>>(minv, 2 * u, sizeof(Packed3<T>));
                ib = rec_at<WIDE, Packed3<T>>(minv, 2 * u + 1, sizeof(Packed3<T>));
            };
            // loaded before the walk, after it when the walk also sums the
            // differences (registers)
            if constexpr (TAPE == 1) load_minv();
            const V2 ca = lds_ld<V2>(lds0 + oself), cb = lds_ld<V2>(lds0 + oself + L::stride);
            const V2 cc = lds_ld<V2>(lds0 + oself + 2 * L::stride);
            T m00 = 0, m01 = 0, m02 = 0, m11 = 0, m12 = 0, m22 = 0;
            T b00 = 0, b01 = 0, b02 = 0, b10 = 0, b11 = 0, b12 = 0, b20 = 0, b21 = 0, b22 = 0;
            T s0 = 0, s1 = 0, s2 = 0;
            struct Q {
                V2 a, b, c;
            };
            auto acc = [&](const Q q) {
                const T dx0 = q.a.x - ca.x, dx1 = q.a.y - ca.y, dx2 = q.b.x - cb.x;
                const T df0 = q.b.y - cb.y, df1 = q.c.x - cc.x, df2 = q.c.y - cc.y;
                if constexpr (!kMinv) {
                    m00 = dfma(dx0, dx0, m00);
                    m01 = dfma(dx0, dx1, m01);
                    m02 = dfma(dx0, dx2, m02);
                    m11 = dfma(dx1, dx1, m11);
                    m12 = dfma(dx1, dx2, m12);
                    m22 = dfma(dx2, dx2, m22);
                }
                b00 = dfma(df0, dx0, b00);
                b01 = dfma(df0, dx1, b01);
                b02 = dfma(df0, dx2, b02);
                b10 = dfma(df1, dx0, b10);
                b11 = dfma(df1, dx1, b11);
                b12 = dfma(df1, dx2, b12);
                b20 = dfma(df2, dx0, b20);
                b21 = dfma(df2, dx1, b21);
                b22 = dfma(df2, dx2, b22);
                if constexpr (TAPE == 2) {
                    s0 += dx0;
                    s1 += dx1;
                    s2 += dx2;
                }
            };
            // one address per neighbour; the other two arrays at fixed offsets
            const uint32_t b0 = lds0 + sh;
            auto at = [&](uint32_t j) {
                const uint32_t t = b0 + j * L::unit;
                return Q{lds_ld<V2>(t), lds_ld<V2>(t + L::stride), lds_ld<V2>(t + 2 * L::stride)};
            };
            walk_row<1, true>(words, s, e, [&](auto pad, auto... o) {
                constexpr int N = sizeof...(o);
                const Q q[] = {at(o)...};
#pragma unroll
                for (int k = 0; k < N; ++k)
                    if (entry_live<N>(k, pad)) acc(q[k]);
            });
            if constexpr (TAPE == 2) load_minv();
            if constexpr (!kMinv) u = slot_point(recl, R, l);
            // M^-1 = A id: A the adjugate of M (symmetric) and id = 1 / det M,
            // or A = M^-1 itself and id = 1
            T a00, a01, a02, a11, a12, a22, id;
            bool ok;
            if constexpr (kMinv) {
                a00 = ia.a, a01 = ia.b, a02 = ia.c, a11 = ib.a, a12 = ib.b, a22 = ib.c;
                id = T(1);
                ok = !isnan(a00);
            } else {
                a00 = m11 * m22 - m12 * m12, a01 = m02 * m12 - m01 * m22, a02 = m01 * m12 - m02 * m11;
                a11 = m00 * m22 - m02 * m02, a12 = m01 * m02 - m00 * m12, a22 = m00 * m11 - m01 * m01;
                const T det = m00 * a00 + m01 * a01 + m02 * a02;
                const T tr3 = (m00 + m11 + m22) * T(1.0 / 3.0);
                ok = det > rank_tau<T>() * tr3 * tr3 * tr3;
                id = drcp(det);
            }
            const T j00 = (b00 * a00 + b01 * a01 + b02 * a02) * id;
            const T j01 = (b00 * a01 + b01 * a11 + b02 * a12) * id;
            const T j02 = (b00 * a02 + b01 * a12 + b02 * a22) * id;
            const T j10 = (b10 * a00 + b11 * a01 + b12 * a02) * id;
            const T j11 = (b10 * a01 + b11 * a11 + b12 * a12) * id;
            const T j12 = (b10 * a02 + b11 * a12 + b12 * a22) * id;
            const T j20 = (b20 * a00 + b21 * a01 + b22 * a02) * id;
            const T j21 = (b20 * a01 + b21 * a11 + b22 * a12) * id;
            const T j22 = (b20 * a02 + b21 * a12 + b22 * a22) * id;
            const T c00 = j00 * j00 + j10 * j10 + j20 * j20;
            const T c01 = j00 * j01 + j10 * j11 + j20 * j21;
            const T c02 = j00 * j02 + j10 * j12 + j20 * j22;
            const T c11 = j01 * j01 + j11 * j11 + j21 * j21;
            const T c12 = j01 * j02 + j11 * j12 + j21 * j22;
            const T c22 = j02 * j02 + j12 * j12 + j22 * j22;
            T r, lam;
            if constexpr (sizeof(T) == 4) {
                lam = lam_max3_poly(c00, c01, c02, c11, c12, c22, r);
                // Top pair nearly equal: c'(r) amplifies float rounding in r;
                // redo the tensor and the eigenvalue in double from J.
                const bool redo = ok && (r + 1.0f < eig_tau);   // (r + 1: no loop-invariant register)
                if (redo) {
                    lam = lam_max3_f64_from_J(j00, j01, j02, j10, j11, j12, j20, j21, j22);
                    ++redone;
                }
            } else {
                lam = lam_max3_trig(c00, c01, c02, c11, c12, c22, r);
            }
            f = ok ? log_scaled(lam, inv2T) : quiet_nan<T>();
            if constexpr (TAPE) {
                // unit top eigenvector: the largest cross product of two rows of C - lambda I
                const T r00 = c00 - lam, r11 = c11 - lam, r22 = c22 - lam;
                const T xa0 = c01 * c12 - c02 * r11, xa1 = c02 * c01 - r00 * c12, xa2 = r00 * r11 - c01 * c01;
                const T xb0 = c01 * r22 - c02 * c12, xb1 = c02 * c02 - r00 * r22, xb2 = r00 * c12 - c01 * c02;
                const T xc0 = r11 * r22 - c12 * c12, xc1 = c12 * c02 - c01 * r22, xc2 = c01 * c12 - r11 * c02;
                const T na = xa0 * xa0 + xa1 * xa1 + xa2 * xa2;
                const T nb = xb0 * xb0 + xb1 * xb1 + xb2 * xb2;
                const T nc = xc0 * xc0 + xc1 * xc1 + xc2 * xc2;
                T v0 = xa0, v1 = xa1, v2 = xa2, nv = na;
                if (nb > nv) { v0 = xb0; v1 = xb1; v2 = xb2; nv = nb; }
                if (nc > nv) { v0 = xc0; v1 = xc1; v2 = xc2; nv = nc; }
                if (nv > T(0)) {
                    const T iv = drcp(dsqrt(nv));
                    v0 *= iv; v1 *= iv; v2 *= iv;
                } else {
                    v0 = T(1); v1 = T(0); v2 = T(0);
                }
                const bool use = ok && (lam > T(0)) && isfinite(f);
                // a point without a usable FTLE (rank-deficient stencil, non-
                // finite values) puts zeros on the tape: selects, not products
                // with zero, since J and v may hold NaN there
                const T sc = T(2) * inv2T * drcp(lam);
                const T h0 = use ? (a00 * v0 + a01 * v1 + a02 * v2) * id : T(0);
                const T h1 = use ? (a01 * v0 + a11 * v1 + a12 * v2) * id : T(0);
                const T h2 = use ? (a02 * v0 + a12 * v1 + a22 * v2) * id : T(0);
                rec_put<WIDE>(tape, 2 * u, sizeof(Packed3<T>),
                              Packed3<T>{use ? (j00 * v0 + j01 * v1 + j02 * v2) * sc : T(0),
                                         use ? (j10 * v0 + j11 * v1 + j12 * v2) * sc : T(0),
                                         use ? (j20 * v0 + j21 * v1 + j22 * v2) * sc : T(0)});
                rec_put<WIDE>(tape, 2 * u + 1, sizeof(Packed3<T>), Packed3<T>{h0, h1, h2});
                if constexpr (TAPE == 2) rec_put<WIDE>(tape + (size_t)n * 6, u, sizeof(T), h0 * s0 + h1 * s1 + h2 * s2);
            }
        }
        if constexpr (OUT) rec_put<WIDE>(out, u, sizeof(T), f);
    }
    if (hits && redone) atomicAdd(hits, (unsigned long long)redone);   // rare: nearly equal top pairs
}

// One tile of the forward pass by the whole workgroup of B threads.
template <int D, typename T, bool OUT, int TAPE, int B, bool WIDE>
__device__ __forceinline__ void fwd_tile(const TileMeta m, const uint4* __restrict__ rec,
                                         const T* __restrict__ x, const T* __restrict__ minv,
                                         const T* __restrict__ flow, const T inv2T, T* __restrict__ out,
                                         T* __restrict__ tape, const int64_t n, const float eig_tau,
                                         unsigned long long* hits, const uint32_t lds0)
{
    fwd_stage_tile<D, T, B, WIDE>(m, rec, x, flow, lds0, (int)threadIdx.x);
    __builtin_amdgcn_s_waitcnt(0);   // the staging loads have landed in LDS
    __syncthreads();
    fwd_compute_tile<D, T, OUT, TAPE, B, WIDE>(m, minv, inv2T, out, tape, n, eig_tau, hits, lds0, (int)threadIdx.x);
}

// float: at most 64 VGPRs (8 waves per SIMD), so that the LDS, not the
// registers, bounds the workgroups per CU; the tape variant needs the hint.
template <int D, typename T, bool OUT, int TAPE, int B, bool WIDE>
__global__ void __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 8 : 1)))
fwd_kernel(const TileMeta* __restrict__ meta, const uint4* __restrict__ rec, int n_tiles, const T* __restrict__ x,
           const T* __restrict__ minv, const T* __restrict__ flow, T inv2T, T* __restrict__ out, T* __restrict__ tape,
           int64_t n, float eig_tau, unsigned long long* hits)
{
    const int t = xcd_tile(blockIdx.x, n_tiles);
    fwd_tile<D, T, OUT, TAPE, B, WIDE>(meta[t], rec, x, minv, flow, inv2T, out, tape, n, eig_tau, hits, 0u);
}

// ---------------------------------------------------------------------------
// Adjoint gather.  With w_k = g_k p_k (p, h, sigma from the tape):
//   dL/dphi_j = sum_{i : j in S(i)} w_i (h_i . (x_j - x_i))  -  g_j sigma_j p_j
// The tile set here is the one of the transposed stencil S^T (equal to S for
// the symmetric one-ring stencil).  Points with non-finite g add nothing.
// ---------------------------------------------------------------------------
// Adjoint staging round (as fwd_stage): slot l holds x, h and w = g p of its
// point (g non-finite -> 0).
template <int D, typename T, int B, bool WIDE, int K>
__device__ inline void bwd_stage(uint32_t rec, const RecLayout& R, const T* __restrict__ x,
                                 const T* __restrict__ tape, const T* __restrict__ g, int S, int r0,
                                 uint32_t lds0, int tid)
{
    using V2 = vec2_t<T>;
    using V4 = vec4_t<T>;
    using L = Layout<D, T>;
    const int base = r0 + tid;
    uint32_t u[K];
#pragma unroll
    for (int k = 0; k < K; ++k) u[k] = slot_point(rec, R, min(base + k * B, S - 1));
    T gu[K];
    if constexpr (D == 2) {
        V2 xv[K];
        V4 tv[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            gu[k] = rec_at<WIDE, T>(g, u[k], sizeof(T));
            xv[k] = rec_at<WIDE, V2>(x, u[k], sizeof(V2));
            tv[k] = rec_at<WIDE, V4>(tape, u[k], sizeof(V4));
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t o = (uint32_t)min(base + k * B, S - 1) * L::unit;
            const T gg = isfinite(gu[k]) ? gu[k] : T(0);
            lds_st(lds0 + 2 * o, V4{xv[k].x, xv[k].y, gg * tv[k].x, gg * tv[k].y});
            lds_st(lds0 + 2 * o + 4 * sizeof(T), V2{tv[k].z, tv[k].w});
        }
    } else {
        Packed3<T> xv[K], pv[K], hv[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            gu[k] = rec_at<WIDE, T>(g, u[k], sizeof(T));
            xv[k] = rec_at<WIDE, Packed3<T>>(x, u[k], sizeof(Packed3<T>));
            pv[k] = rec_at<WIDE, Packed3<T>>(tape, 2 * u[k], sizeof(Packed3<T>));
            hv[k] = rec_at<WIDE, Packed3<T>>(tape, 2 * u[k] + 1, sizeof(Packed3<T>));
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t sl = (uint32_t)min(base + k * B, S - 1);
            const uint32_t o = lds0 + sl * L::bunit;
            const T gg = isfinite(gu[k]) ? gu[k] : T(0);
            lds_st(o, V4{xv[k].a, xv[k].b, xv[k].c, hv[k].a});
            lds_st(o + L::bstride, V4{hv[k].b, hv[k].c, gg * pv[k].a, gg * pv[k].b});
            lds_st(lds0 + 2 * L::bstride + sl * sizeof(T), gg * pv[k].c);
        }
    }
}

// Staging of an adjoint tile by B threads (tid in [0, B)) into the LDS region
// at lds0 (as fwd_stage_tile).
template <int D, typename T, int B, bool WIDE>
__device__ __forceinline__ void bwd_stage_tile(const TileMeta m, const uint4* __restrict__ rec,
                                               const T* __restrict__ x, const T* __restrict__ tape,
                                               const T* __restrict__ g, const uint32_t lds0, const int tid)
{
    using L = Layout<D, T>;
    const int S = (int)m.P + (int)m.H;
    const RecLayout R = rec_layout(m);
    const uint32_t recl = L::bwd_rec(lds0, S);   // LDS address of the record
    dma_record<B>(rec + m.rec_off, recl, (int)(R.bytes / 16), tid);
    __builtin_amdgcn_s_waitcnt(0);   // this wave's part of the record has landed in LDS
    __syncthreads();
    stage_points<B>(S, [&](auto kc, int r0) {
        bwd_stage<D, T, B, WIDE, decltype(kc)::value>(recl, R, x, tape, g, S, r0, lds0, tid);
    });
}

// The gather of a staged adjoint tile by B threads (tid in [0, B)).
// SIG: sigma_j from the tape (non-symmetric stencil).  Otherwise S^T = S, the
// walk visits exactly the stencil of j, and sigma_j = h_j . sum_i (x_i - x_j)
// is formed from the same differences.
template <int D, typename T, int B, bool WIDE, bool SIG>
__device__ __forceinline__ void bwd_compute_tile(const TileMeta m, const T* __restrict__ tape, const int64_t n,
                                                 T* __restrict__ grad, const uint32_t lds0, const int tid)
{
    using V2 = vec2_t<T>;
    using V4 = vec4_t<T>;
    using L = Layout<D, T>;
    const int P = (int)m.P;
    const int S = P + (int)m.H;
    const RecLayout R = rec_layout(m);
    const uint32_t recl = L::bwd_rec(lds0, S);   // LDS address of the record
    const uint32_t words = recl;
    // 2D: the slot array at lds0; 3D: the two 4-value arrays, then w2
    const uint32_t c0 = lds0, cw = lds0 + 2 * L::bstride;
    for (int l = tid; l < P; l += B) {
        const RowRef row = row_ref(recl, R, l);
        const int s = row.s, e = row.e;
        const uint32_t sh = (uint32_t)row.shift * L::unit;   // the row's entries are its anchor's plus shift
        const uint32_t u = slot_point(recl, R, l);
        T sig = T(0);
        if constexpr (SIG) sig = rec_at<WIDE, T>(tape + (size_t)n * (2 * D), u, sizeof(T));
        const uint32_t oself = (uint32_t)l * L::unit;
        if constexpr (D == 2) {
            const V4 cj = lds_ld<V4>(c0 + 2 * oself);
            T a0 = 0, a1 = 0, s0 = 0, s1 = 0;
            struct Q {
                V4 a;
                V2 h;
            };
            const uint32_t b0 = c0 + 2 * sh;
            auto at = [&](uint32_t j) {
                const uint32_t o = j * L::unit;
                return Q{lds_ld<V4>(b0 + 2 * o), lds_ld<V2>(b0 + 2 * o + 4 * sizeof(T))};
            };
            walk_row<1, true>(words, s, e, [&](auto pad, auto... o) {
                constexpr int N = sizeof...(o);
                const Q q[] = {at(o)...};
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    if (!entry_live<N>(k, pad)) continue;
                    const Q& v = q[k];
                    const T d0 = cj.x - v.a.x, d1 = cj.y - v.a.y;
                    const T t = v.h.x * d0 + v.h.y * d1;
                    a0 = dfma(v.a.z, t, a0);
                    a1 = dfma(v.a.w, t, a1);
                    if constexpr (!SIG) {
                        s0 += d0;
                        s1 += d1;
                    }
                }
            });
            if constexpr (!SIG) {
                const V2 hj = lds_ld<V2>(c0 + 2 * oself + 4 * sizeof(T));
                sig = -(hj.x * s0 + hj.y * s1);
            }
            rec_put<WIDE>(grad, u, sizeof(V2), V2{a0 - sig * cj.z, a1 - sig * cj.w});
        } else {
            const V4 cj = lds_ld<V4>(lds0 + (uint32_t)l * L::bunit);
            const V4 cb = lds_ld<V4>(lds0 + (uint32_t)l * L::bunit + L::bstride);
            const T cw2 = lds_ld<T>(cw + (uint32_t)l * sizeof(T));
            T a0 = 0, a1 = 0, a2 = 0, s0 = 0, s1 = 0, s2 = 0;
            struct Q {
                V4 a, b;
                T c;
            };
            // per neighbour one address into the 4-value arrays (the second at
            // a fixed offset) and one into w2
            const uint32_t bq = lds0 + (uint32_t)row.shift * L::bunit, bw = cw + (uint32_t)row.shift * sizeof(T);
            auto at = [&](uint32_t j) {
                const uint32_t t = bq + j * L::bunit;
                return Q{lds_ld<V4>(t), lds_ld<V4>(t + L::bstride), lds_ld<T>(bw + j * sizeof(T))};
            };
            walk_row<1, true>(words, s, e, [&](auto pad, auto... o) {
                constexpr int N = sizeof...(o);
                const Q q[] = {at(o)...};
#pragma unroll
                for (int k = 0; k < N; ++k) {
                    if (!entry_live<N>(k, pad)) continue;
                    const Q& v = q[k];
                    const T d0 = cj.x - v.a.x, d1 = cj.y - v.a.y, d2 = cj.z - v.a.z;
                    const T t = v.a.w * d0 + v.b.x * d1 + v.b.y * d2;
                    a0 = dfma(v.b.z, t, a0);
                    a1 = dfma(v.b.w, t, a1);
                    a2 = dfma(v.c, t, a2);
                    if constexpr (!SIG) {
                        s0 += d0;
                        s1 += d1;
                        s2 += d2;
                    }
                }
            });
            if constexpr (!SIG) sig = -(cj.w * s0 + cb.x * s1 + cb.y * s2);
            rec_put<WIDE>(grad, u, sizeof(Packed3<T>), Packed3<T>{a0 - sig * cb.z, a1 - sig * cb.w, a2 - sig * cw2});
        }
    }
}

template <int D, typename T, int B, bool WIDE, bool SIG>
__global__ void __launch_bounds__(B) bwd_kernel(const TileMeta* __restrict__ meta, const uint4* __restrict__ rec,
                                                  int n_tiles, const T* __restrict__ x, const T* __restrict__ tape,
                                                  int64_t n, const T* __restrict__ g, T* __restrict__ grad)
{
    const TileMeta m = meta[xcd_tile(blockIdx.x, n_tiles)];
    bwd_stage_tile<D, T, B, WIDE>(m, rec, x, tape, g, 0u, (int)threadIdx.x);
    __builtin_amdgcn_s_waitcnt(0);   // the staging loads have landed in LDS
    __syncthreads();
    bwd_compute_tile<D, T, B, WIDE, SIG>(m, tape, n, grad, 0u, (int)threadIdx.x);
}

// ---------------------------------------------------------------------------
// Batched forward over (mesh, tile) work items, running the same tile body as
// fwd_kernel (results are bit-identical).  Two launch forms:
//  - persistent (tiles_per_pop > 0): a resident grid drains an atomic queue,
//    each workgroup taking tiles_per_pop consecutive items per pop; queue[0]
//    is the next item, queue[1] counts finished workgroups, and the last
//    workgroup to finish zeroes both for the next launch;
//  - flat (tiles_per_pop == 0): one workgroup per item (grid = n_items).
// ---------------------------------------------------------------------------
template <int D, typename T, int B, bool WIDE>
__global__ void __launch_bounds__(B) batched_kernel(const BatchItem* __restrict__ items, int n_items,
                                                      int tiles_per_pop, unsigned* queue,
                                                      BatchCall call, float eig_tau)
{
    // (the call's arrays are indexed here, in the kernel body, so that they
    // are read from the kernel arguments and never copied)
    if (tiles_per_pop == 0) {
        // flat launch: one work item per workgroup, dealt XCD-contiguously
        const BatchItem it = items[xcd_tile(blockIdx.x, n_items)];
        fwd_tile<D, T, true, 0, B, WIDE>(it.meta, it.rec, static_cast<const T*>(it.x), nullptr,
                                             static_cast<const T*>(call.flow[it.mesh]), (T)call.inv2T[it.mesh],
                                             static_cast<T*>(call.out[it.mesh]), nullptr, 0, eig_tau, it.fp64_hits,
                                             kBatchedLdsHead);
        return;
    }
    for (;;) {
        if (threadIdx.x == 0) lds_st(0u, (int)atomicAdd(&queue[0], (unsigned)tiles_per_pop));
        __syncthreads();
        const int base = lds_ld<int>(0u);
        __syncthreads();
        if (base >= n_items) break;
        const int lim = min(base + tiles_per_pop, n_items);
        for (int i = base; i < lim; ++i) {
            const BatchItem it = items[i];
            fwd_tile<D, T, true, 0, B, WIDE>(it.meta, it.rec, static_cast<const T*>(it.x), nullptr,
                                                 static_cast<const T*>(call.flow[it.mesh]), (T)call.inv2T[it.mesh],
                                                 static_cast<T*>(call.out[it.mesh]), nullptr, 0, eig_tau,
                                                 it.fp64_hits, kBatchedLdsHead);
            __syncthreads();
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned done = atomicAdd(&queue[1], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&queue[0], 0u);
            atomicExch(&queue[1], 0u);
            __threadfence();
        }
    }
}

template <int D, typename T>
size_t fwd_lds(const DevTiles& t)
{
    return fwd_points_bytes(D, sizeof(T) == 8, t.max_staged) + (size_t)t.max_rec;
}
template <int D, typename T>
size_t bwd_lds(const DevTiles& t)
{
    return bwd_points_bytes(D, sizeof(T) == 8, t.max_staged) + (size_t)t.max_rec;
}

template <int D, typename T, int B, bool WIDE>
hipError_t fwd_launch_b(const DevTiles& tiles, const void* x, const void* flow, double inv2T, void* out,
                        void* tape, bool tape_sigma, int64_t n, double eig_tau, unsigned long long* hits,
                        hipStream_t stream)
{
    const size_t lds = fwd_lds<D, T>(tiles);
    const dim3 grid(tiles.n_tiles), blk(B);
    const T* xp = static_cast<const T*>(x);
    const T* fp = static_cast<const T*>(flow);
    T* op = static_cast<T*>(out);
    T* tp = static_cast<T*>(tape);
#define FTLE_FWD_LAUNCH(OUT, TAPE)                                                                              \
    hipLaunchKernelGGL((fwd_kernel<D, T, OUT, TAPE, B, WIDE>), grid, blk, lds, stream, tiles.meta, tiles.rec,   \
                       tiles.n_tiles, xp, static_cast<const T*>(tiles.minv), fp, (T)inv2T, op, tp, n,             \
                       (float)eig_tau, hits)
    if (!tape)
        FTLE_FWD_LAUNCH(true, 0);
    else if (out && tape_sigma)
        FTLE_FWD_LAUNCH(true, 2);
    else if (out)
        FTLE_FWD_LAUNCH(true, 1);
    else if (tape_sigma)
        FTLE_FWD_LAUNCH(false, 2);
    else
        FTLE_FWD_LAUNCH(false, 1);
#undef FTLE_FWD_LAUNCH
    return hipGetLastError();
}

template <int D, typename T, int B, bool WIDE>
hipError_t bwd_launch_b(const DevTiles& tiles, const void* x, const void* tape, bool tape_sigma, int64_t n,
                        const void* g, void* grad, hipStream_t stream)
{
    const size_t lds = bwd_lds<D, T>(tiles);
    if (tape_sigma)
        hipLaunchKernelGGL((bwd_kernel<D, T, B, WIDE, true>), dim3(tiles.n_tiles), dim3(B), lds, stream, tiles.meta,
                           tiles.rec, tiles.n_tiles, static_cast<const T*>(x), static_cast<const T*>(tape), n,
                           static_cast<const T*>(g), static_cast<T*>(grad));
    else
        hipLaunchKernelGGL((bwd_kernel<D, T, B, WIDE, false>), dim3(tiles.n_tiles), dim3(B), lds, stream, tiles.meta,
                           tiles.rec, tiles.n_tiles, static_cast<const T*>(x), static_cast<const T*>(tape), n,
                           static_cast<const T*>(g), static_cast<T*>(grad));
    return hipGetLastError();
}

// 32-bit byte offsets reach every array of an n-point mesh when the largest
// per-point record (the 3D tape's 2*dim values) times n stays below 4 GiB.
std::atomic<bool> g_force_wide{false};

template <typename T>
bool needs_wide(int dim, int64_t n)
{
    if (g_force_wide.load(std::memory_order_relaxed)) return true;
    return (uint64_t)n * (uint64_t)(2 * dim) * sizeof(T) >= (1ull << 32);
}

template <int D, typename T, bool WIDE>
hipError_t fwd_launch_w(const DevTiles& tiles, const void* x, const void* flow, double inv2T, void* out,
                        void* tape, bool ts, int64_t n, double eig_tau, unsigned long long* hits, int block,
                        hipStream_t stream)
{
    switch (block) {
    case 128: return fwd_launch_b<D, T, 128, WIDE>(tiles, x, flow, inv2T, out, tape, ts, n, eig_tau, hits, stream);
    case 256: return fwd_launch_b<D, T, 256, WIDE>(tiles, x, flow, inv2T, out, tape, ts, n, eig_tau, hits, stream);
    case 512: return fwd_launch_b<D, T, 512, WIDE>(tiles, x, flow, inv2T, out, tape, ts, n, eig_tau, hits, stream);
    default: return hipErrorInvalidValue;
    }
}

template <int D, typename T>
hipError_t fwd_launch(const DevTiles& tiles, const void* x, const void* flow, double inv2T, void* out,
                      void* tape, bool ts, int64_t n, double eig_tau, unsigned long long* hits, int block,
                      hipStream_t stream)
{
    if (needs_wide<T>(D, n))
        return fwd_launch_w<D, T, true>(tiles, x, flow, inv2T, out, tape, ts, n, eig_tau, hits, block, stream);
    return fwd_launch_w<D, T, false>(tiles, x, flow, inv2T, out, tape, ts, n, eig_tau, hits, block, stream);
}

template <int D, typename T>
hipError_t bwd_launch(const DevTiles& tiles, const void* x, const void* tape, bool ts, int64_t n, const void* g,
                      void* grad, int block, hipStream_t stream)
{
    const bool wide = needs_wide<T>(D, n);
    switch (block) {
    case 128:
        return wide ? bwd_launch_b<D, T, 128, true>(tiles, x, tape, ts, n, g, grad, stream)
                    : bwd_launch_b<D, T, 128, false>(tiles, x, tape, ts, n, g, grad, stream);
    case 256:
        return wide ? bwd_launch_b<D, T, 256, true>(tiles, x, tape, ts, n, g, grad, stream)
                    : bwd_launch_b<D, T, 256, false>(tiles, x, tape, ts, n, g, grad, stream);
    case 512:
        return wide ? bwd_launch_b<D, T, 512, true>(tiles, x, tape, ts, n, g, grad, stream)
                    : bwd_launch_b<D, T, 512, false>(tiles, x, tape, ts, n, g, grad, stream);
    default: return hipErrorInvalidValue;
    }
}

struct BatchArgs {
    const BatchItem* items;
    int n_items;
    int tiles_per_pop;
    unsigned* queue;
    BatchCall call;
    float eig_tau;
};

}  // namespace

size_t fwd_lds_bytes(int dim, bool f64, const DevTiles& t)
{
    if (dim == 2) return f64 ? fwd_lds<2, double>(t) : fwd_lds<2, float>(t);
    return f64 ? fwd_lds<3, double>(t) : fwd_lds<3, float>(t);
}

size_t bwd_lds_bytes(int dim, bool f64, const DevTiles& t)
{
    if (dim == 2) return f64 ? bwd_lds<2, double>(t) : bwd_lds<2, float>(t);
    return f64 ? bwd_lds<3, double>(t) : bwd_lds<3, float>(t);
}

hipError_t launch_forward(int dim, bool f64, const DevTiles& tiles, const void* x, const void* flow,
                          double inv2T, void* out, void* tape, bool tape_sigma, int64_t n, double eig_tau,
                          unsigned long long* hits, int block, hipStream_t stream)
{
    if (tiles.n_tiles == 0) return hipSuccess;
    const bool ts = tape_sigma;
    if (dim == 2)
        return f64 ? fwd_launch<2, double>(tiles, x, flow, inv2T, out, tape, ts, n, eig_tau, hits, block, stream)
                   : fwd_launch<2, float>(tiles, x, flow, inv2T, out, tape, ts, n, eig_tau, hits, block, stream);
    return f64 ? fwd_launch<3, double>(tiles, x, flow, inv2T, out, tape, ts, n, eig_tau, hits, block, stream)
               : fwd_launch<3, float>(tiles, x, flow, inv2T, out, tape, ts, n, eig_tau, hits, block, stream);
}

// ---------------------------------------------------------------------------
// Half-precision flow-map storage (2D meshes, float32 arithmetic).  The flow
// map is held as the displacement d = phi - x, rounded to binary16: 4 bytes
// per point instead of 8.  The staging decodes phi' = x + d in float32 (one
// rounding); from there the tile runs the float32 forward unchanged, so the
// result is the float32 FTLE of the decoded map phi'.
// ---------------------------------------------------------------------------
template <int B, int K>
__device__ inline void fwd16_stage(uint32_t rec, const RecLayout& R, const float* __restrict__ x,
                                   const __half2* __restrict__ d, int S, int r0, int tid)
{
    using L = Layout<2, float>;
    const int base = r0 + tid;
    uint32_t u[K];
#pragma unroll
    for (int k = 0; k < K; ++k) u[k] = slot_point(rec, R, min(base + k * B, S - 1));
    float2 xv[K];
    __half2 dv[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        xv[k] = rec_at<false, float2>(x, u[k], sizeof(float2));
        dv[k] = rec_at<false, __half2>(d, u[k], sizeof(__half2));
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float2 dd = __half22float2(dv[k]);
        const uint32_t o = (uint32_t)min(base + k * B, S - 1) * L::unit;
        lds_st(o, float4{xv[k].x, xv[k].y, xv[k].x + dd.x, xv[k].y + dd.y});
    }
}

template <int B>
__global__ void __launch_bounds__(B) __attribute__((amdgpu_waves_per_eu(8)))
fwd16_kernel(const TileMeta* __restrict__ meta, const uint4* __restrict__ rec, int n_tiles, const float* __restrict__ x,
             const __half2* __restrict__ d, float inv2T, float* __restrict__ out, int64_t n, float eig_tau,
             unsigned long long* hits)
{
    using L = Layout<2, float>;
    const TileMeta m = meta[xcd_tile(blockIdx.x, n_tiles)];
    const int S = (int)m.P + (int)m.H;
    const RecLayout R = rec_layout(m);
    const uint32_t recl = L::fwd_rec(0u, S);
    const int tid = (int)threadIdx.x;
    dma_record<B>(rec + m.rec_off, recl, (int)(R.bytes / 16), tid);
    __builtin_amdgcn_s_waitcnt(0);   // this wave's part of the record has landed in LDS
    __syncthreads();
    stage_points<B>(S, [&](auto kc, int r0) { fwd16_stage<B, decltype(kc)::value>(recl, R, x, d, S, r0, tid); });
    __builtin_amdgcn_s_waitcnt(0);   // the staging loads have landed in LDS
    __syncthreads();
    fwd_compute_tile<2, float, true, 0, B, false>(m, nullptr, inv2T, out, nullptr, n, eig_tau, hits, 0u, tid);
}

// d = binary16(phi - x), the float32 difference rounded to nearest even.
__global__ void __launch_bounds__(256) encode16_kernel(const float2* __restrict__ x, const float2* __restrict__ phi,
                                                       __half2* __restrict__ d, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float2 a = x[i], b = phi[i];
    d[i] = __floats2half2_rn(b.x - a.x, b.y - a.y);
}

hipError_t launch_forward_f16(const DevTiles& tiles, const void* x, const void* delta, double inv2T, void* out,
                              int64_t n, double eig_tau, unsigned long long* hits, int block, hipStream_t stream)
{
    if (tiles.n_tiles == 0) return hipSuccess;
    const size_t lds = fwd_lds<2, float>(tiles);
    const float* xp = static_cast<const float*>(x);
    const __half2* dp = static_cast<const __half2*>(delta);
    float* op = static_cast<float*>(out);
#define FTLE_FWD16_LAUNCH(BB)                                                                                    \
    hipLaunchKernelGGL((fwd16_kernel<BB>), dim3(tiles.n_tiles), dim3(BB), lds, stream, tiles.meta, tiles.rec,    \
                       tiles.n_tiles, xp, dp, (float)inv2T, op, n, (float)eig_tau, hits)
    switch (block) {
    case 128: FTLE_FWD16_LAUNCH(128); break;
    case 512: FTLE_FWD16_LAUNCH(512); break;
    default: FTLE_FWD16_LAUNCH(256); break;
    }
#undef FTLE_FWD16_LAUNCH
    return hipGetLastError();
}

hipError_t launch_encode_f16(const void* x, const void* flow, void* delta, int64_t n, hipStream_t stream)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(encode16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                       static_cast<const float2*>(x), static_cast<const float2*>(flow), static_cast<__half2*>(delta),
                       n);
    return hipGetLastError();
}

hipError_t launch_backward_gather(int dim, bool f64, const DevTiles& tiles, const void* x,
                                  const void* tape, bool tape_sigma, int64_t n, const void* g, void* grad,
                                  int block, hipStream_t stream)
{
    if (tiles.n_tiles == 0) return hipSuccess;
    const bool ts = tape_sigma;
    if (dim == 2)
        return f64 ? bwd_launch<2, double>(tiles, x, tape, ts, n, g, grad, block, stream)
                   : bwd_launch<2, float>(tiles, x, tape, ts, n, g, grad, block, stream);
    return f64 ? bwd_launch<3, double>(tiles, x, tape, ts, n, g, grad, block, stream)
               : bwd_launch<3, float>(tiles, x, tape, ts, n, g, grad, block, stream);
}

template <int D, typename T, bool WIDE>
const void* batched_symbol_b(int block)
{
    switch (block) {
    case 128: return reinterpret_cast<const void*>(&batched_kernel<D, T, 128, WIDE>);
    case 256: return reinterpret_cast<const void*>(&batched_kernel<D, T, 256, WIDE>);
    case 512: return reinterpret_cast<const void*>(&batched_kernel<D, T, 512, WIDE>);
    default: return nullptr;
    }
}

const void* batched_kernel_symbol(int dim, bool f64, int block, bool wide)
{
    if (dim == 2) {
        if (f64) return wide ? batched_symbol_b<2, double, true>(block) : batched_symbol_b<2, double, false>(block);
        return wide ? batched_symbol_b<2, float, true>(block) : batched_symbol_b<2, float, false>(block);
    }
    if (f64) return wide ? batched_symbol_b<3, double, true>(block) : batched_symbol_b<3, double, false>(block);
    return wide ? batched_symbol_b<3, float, true>(block) : batched_symbol_b<3, float, false>(block);
}

void set_force_wide(bool on) { g_force_wide.store(on, std::memory_order_relaxed); }

bool batched_needs_wide(int dim, bool f64, int64_t max_points)
{
    return f64 ? needs_wide<double>(dim, max_points) : needs_wide<float>(dim, max_points);
}

size_t batched_kernel_arg_storage() { return sizeof(BatchArgs); }

void batched_kernel_args(const BatchItem* items, int n_items, int tiles_per_pop, unsigned* queue,
                         const BatchCall& call, double eig_tau, void* storage, void** args)
{
    BatchArgs* a = static_cast<BatchArgs*>(storage);
    a->items = items;
    a->n_items = n_items;
    a->tiles_per_pop = tiles_per_pop;
    a->queue = queue;
    a->call = call;
    a->eig_tau = (float)eig_tau;
    args[0] = &a->items;
    args[1] = &a->n_items;
    args[2] = &a->tiles_per_pop;
    args[3] = &a->queue;
    args[4] = &a->call;
    args[5] = &a->eig_tau;
}

hipError_t launch_batched(int dim, bool f64, bool wide, const BatchItem* items, int n_items, int tiles_per_pop,
                          unsigned* queue, const BatchCall& call, size_t lds, double eig_tau, int block, int grid,
                          hipStream_t stream)
{
    const void* k = batched_kernel_symbol(dim, f64, block, wide);
    if (!k) return hipErrorInvalidValue;
    BatchArgs storage;
    void* args[6];
    batched_kernel_args(items, n_items, tiles_per_pop, queue, call, eig_tau, &storage, args);
    return hipLaunchKernel(k, dim3(grid), dim3(block), args, lds, stream);
}

}  // namespace ftle
