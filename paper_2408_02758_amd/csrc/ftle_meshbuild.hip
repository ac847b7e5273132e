// The whole mesh build on the GPU (ftle_create_mesh_device and
// ftle_create_mesh_device_from_csr): the Morton order of the points, the
// stencil over Morton positions (the one-ring stencil from the cells, the
// axis stencil from it, or a caller's list moved to Morton positions), its
// transpose when it is not symmetric, the tile cut and the compressed tile
// records, and (3D) the inverse normal matrices.  The host-side builder in ftle_host.cpp
// does the same on the CPU, following Section 2.2 (neighbours determined
// once, before the FTLE kernels); the Conclusions name moving that step to
// the accelerator as future work.  Every kernel here reproduces the host's
// result exactly (integer work, and float64 arithmetic evaluated in the same
// order without contraction), so that meshes built either way are the same
// byte for byte.
//
//   bbox_partial    per-workgroup bounds of the coordinates (and whether all
//                   are finite), reduced on the host
//   morton_keys     each point's interleaved code, quantised as the host
//                   quantises it
//   radix_hist / radix_scatter
//                   a stable LSD radix sort of (code, point) pairs, 8 bits a
//                   pass: per-tile digit counts, their scan (digit-major, so
//                   that equal digits keep tile order), then each key's place
//                   from its tile's offset plus its rank among equal digits
//                   before it (wave ballots; waves and rounds in order)
//   check_relabel   cells validated (index range, repeated points) and
//                   renumbered to Morton positions
//   tile_extent     for candidate Morton ranges: halo points and stencil words
//   tile_record     the record of each tile (the layout in ftle_internal.h):
//                   own points and halo in caller order, index runs, rows as
//                   sorted local slots, shift rows; a first pass sizes the
//                   records, a second writes them
//   normal_inverse  the 3D normal matrix inverse per point (float64)
//   axis_slots / axis_fill
//                   the axis stencil from the one-ring rows, then its CSR
//   csr_in_count / csr_in_fill
//                   a caller's list checked, moved to Morton positions, sorted
//   transpose_count / transpose_fill / sort_rows / csr_compare
//                   the transpose for the adjoint's tiles, and the test
//                   whether it equals the stencil
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "ftle_device_math.h"
#include "ftle_internal.h"

namespace ftle {
namespace {

inline unsigned blocks_of(int64_t m, int per) { return (unsigned)((m + per - 1) / per); }

// ---------------------------------------------------------------------------
// bounds and Morton codes
// ---------------------------------------------------------------------------
template <int D, typename T>
__global__ void __launch_bounds__(256) bbox_partial(const T* __restrict__ x, int64_t n, double* __restrict__ part,
                                                    unsigned long long* __restrict__ first_bad)
{
    __shared__ double slo[D][256], shi[D][256];
    const int t = (int)threadIdx.x;
    double lo[D], hi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        lo[d] = INFINITY;
        hi[d] = -INFINITY;
    }
    int64_t bad = -1;
    for (int64_t i = (int64_t)blockIdx.x * 256 + t; i < n; i += (int64_t)gridDim.x * 256)
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const double v = (double)x[i * D + d];
            if (!isfinite(v) && bad < 0) bad = i;
            lo[d] = fmin(lo[d], v);
            hi[d] = fmax(hi[d], v);
        }
    if (bad >= 0) atomicMin(first_bad, (unsigned long long)bad);
#pragma unroll
    for (int d = 0; d < D; ++d) {
        slo[d][t] = lo[d];
        shi[d][t] = hi[d];
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s)
#pragma unroll
            for (int d = 0; d < D; ++d) {
                slo[d][t] = fmin(slo[d][t], slo[d][t + s]);
                shi[d][t] = fmax(shi[d][t], shi[d][t + s]);
            }
        __syncthreads();
    }
    if (t == 0)
#pragma unroll
        for (int d = 0; d < D; ++d) {
            part[blockIdx.x * 2 * D + d] = slo[d][0];
            part[blockIdx.x * 2 * D + D + d] = shi[d][0];
        }
}

// sample k: points k*stride and k*stride + 1 (the caller-order axis test)
template <int D, typename T>
__global__ void __launch_bounds__(256) gather_pairs(const T* __restrict__ x, int64_t m, int64_t stride,
                                                    double* __restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= m) return;
    const int64_t i = k * stride;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        out[k * 2 * D + d] = (double)x[i * D + d];
        out[k * 2 * D + D + d] = (double)x[(i + 1) * D + d];
    }
}

__device__ inline uint64_t spread2(uint64_t v)
{
    v &= 0xffffffffULL;
    v = (v | (v << 16)) & 0x0000ffff0000ffffULL;
    v = (v | (v << 8)) & 0x00ff00ff00ff00ffULL;
    v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0fULL;
    v = (v | (v << 2)) & 0x3333333333333333ULL;
    v = (v | (v << 1)) & 0x5555555555555555ULL;
    return v;
}

__device__ inline uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffULL;
    v = (v | (v << 32)) & 0x001f00000000ffffULL;
    v = (v | (v << 16)) & 0x001f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

template <int D, typename T>
__global__ void __launch_bounds__(256) morton_keys(const T* __restrict__ x, int64_t n, MortonParams mp,
                                                   uint64_t* __restrict__ key, uint32_t* __restrict__ val)
{
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    uint64_t code = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const double t = floor((((double)x[i * D + d] - mp.lo[d]) / mp.unit[d] + 0.2) * mp.scale);
        uint64_t q = (uint64_t)fmin(mp.qmax, fmax(0.0, t));
        if (mp.fast >= 0 && d != mp.fast) q <<= mp.shift_bits;
        code |= (D == 2 ? spread2(q) : spread3(q)) << d;
    }
    key[i] = code;
    val[i] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// stable LSD radix sort, 8 bits a pass, tiles of kRadixTile keys
// ---------------------------------------------------------------------------
constexpr int kRadixThreads = 256, kRadixRounds = 16, kRadixTile = kRadixThreads * kRadixRounds;

// hist[digit * n_tiles + tile] = keys of the tile with that digit
__global__ void __launch_bounds__(kRadixThreads) radix_hist(const uint64_t* __restrict__ key, int64_t n, int shift,
                                                            uint32_t n_tiles, uint32_t* __restrict__ hist)
{
    __shared__ uint32_t h[256];
    const int t = (int)threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    for (int j = 0; j < kRadixRounds; ++j) {
        const int64_t i = base + j * kRadixThreads + t;
        if (i < n) atomicAdd(&h[(key[i] >> shift) & 255], 1u);
    }
    __syncthreads();
    hist[(int64_t)t * n_tiles + blockIdx.x] = h[t];
}

// keys of the tile in index order, a round of 256 at a time: the place of a
// key is its digit's offset for the tile, plus the tile's earlier keys of
// that digit, plus those of earlier waves of the round, plus its rank in its
// wave (lanes below it with the same digit, from ballots bit by bit)
__global__ void __launch_bounds__(kRadixThreads) radix_scatter(const uint64_t* __restrict__ key,
                                                               const uint32_t* __restrict__ val, int64_t n, int shift,
                                                               uint32_t n_tiles, const uint32_t* __restrict__ off,
                                                               uint64_t* __restrict__ key2, uint32_t* __restrict__ val2)
{
    constexpr int kWaves = kRadixThreads / 64;
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[kWaves][256];
    const int t = (int)threadIdx.x, lane = t & 63, wave = t >> 6;
    run[t] = off[(int64_t)t * n_tiles + blockIdx.x];
    for (int w = 0; w < kWaves; ++w) wcnt[w][t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kRadixTile;
    const uint64_t below = (1ull << lane) - 1;
    for (int j = 0; j < kRadixRounds; ++j) {
        const int64_t i = base + j * kRadixThreads + t;
        const bool live = i < n;
        const uint64_t k = live ? key[i] : 0;
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        uint64_t same = __ballot(live);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            same &= bit ? m : ~m;
        }
        if (!live) same = 0;
        const uint32_t rank = (uint32_t)__popcll(same & below);
        if (live && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(same);
        __syncthreads();
        if (live) {
            uint32_t before = run[d];
            for (int w = 0; w < wave; ++w) before += wcnt[w][d];
            const uint32_t p = before + rank;
            key2[p] = k;
            val2[p] = val[i];
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kWaves; ++w) {
            add += wcnt[w][t];
            wcnt[w][t] = 0;
        }
        run[t] += add;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) iota_u32(uint32_t* __restrict__ v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) v[i] = (uint32_t)i;
}

__global__ void __launch_bounds__(256) invert_perm(const uint32_t* __restrict__ perm, int64_t n,
                                                   int32_t* __restrict__ inv)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r < n) inv[perm[r]] = (int32_t)r;
}

// cells validated (an index outside [0, n): flag 1; a point repeated in a
// cell: flag 2; the lowest such cell in *first) and renumbered
template <int K>
__global__ void __launch_bounds__(256) check_relabel(const int32_t* __restrict__ cells, int64_t n_cells, int64_t n,
                                                     const int32_t* __restrict__ inv, int32_t* __restrict__ mc,
                                                     int* __restrict__ flag, unsigned long long* __restrict__ first)
{
    const int64_t c = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * 256 + threadIdx.x;
    if (c >= n_cells) return;
    int32_t v[K];
#pragma unroll
    for (int a = 0; a < K; ++a) v[a] = cells[c * K + a];
    int kind = 0;
#pragma unroll
    for (int a = 0; a < K; ++a) {
        if ((uint64_t)(int64_t)v[a] >= (uint64_t)n) kind = 1;
#pragma unroll
        for (int q = 0; q < a; ++q)
            if (kind == 0 && v[q] == v[a]) kind = 2;
    }
    if (kind) {
        atomicOr(flag, kind);
        atomicMin(first, (unsigned long long)c);
        return;
    }
#pragma unroll
    for (int a = 0; a < K; ++a) mc[c * K + a] = inv[v[a]];
}

// ---------------------------------------------------------------------------
// tiles.  Shared by both kernels: the halo of Morton range [b, e) (the
// stencil's neighbours outside it), gathered in an LDS hash set of Morton
// positions (open addressing).
// ---------------------------------------------------------------------------
constexpr int kTileThreads = 256;
constexpr int kHashSlots = 2 * kMaxStaged;   // at most kMaxStaged keys are ever kept
constexpr int kChunk = 4;                    // stencil entries a lane loads at once
constexpr int kRowScratch = 32;              // row entries a lane sorts in LDS (longer rows: in global memory)

__device__ inline uint32_t tile_hash(int32_t v) { return ((uint32_t)v * 2654435761u) >> 21; }   // 11 bits

// Insert every outside neighbour of rows [b, e); keys[] = -1 before.  Returns
// (to every lane) the number of distinct keys, or kMaxStaged + 1 when more
// would be needed.  hlist gets the keys in insertion order.
__device__ inline int gather_halo(const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col, int64_t b,
                                  int64_t e, int32_t* keys, int32_t* hlist, int* count, int t)
{
    static_assert(kHashSlots == 1 << 11, "tile_hash gives 11 bits");
    for (int64_t r = b + t; r < e; r += kTileThreads) {
        if (__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) > kMaxStaged) break;
        const int64_t p0 = row_ptr[r], p1 = row_ptr[r + 1];
        // kChunk entries loaded together, then inserted (a load past the row
        // end repeats its last entry, which is then found already inserted)
        for (int64_t p = p0; p < p1; p += kChunk) {
            int32_t cs[kChunk];
#pragma unroll
            for (int q = 0; q < kChunk; ++q) cs[q] = col[min(p + q, p1 - 1)];
#pragma unroll
            for (int q = 0; q < kChunk; ++q) {
                const int32_t c = cs[q];
                if (c >= b && c < e) continue;
                uint32_t h = tile_hash(c);
                for (int probe = 0; probe < kHashSlots; ++probe, h = (h + 1) & (kHashSlots - 1)) {
                    const int32_t k = atomicCAS(&keys[h], -1, c);
                    if (k == -1) {
                        const int at = atomicAdd(count, 1);
                        if (at < kMaxStaged) hlist[at] = c;
                        break;
                    }
                    if (k == c) break;
                }
            }
        }
    }
    __syncthreads();
    const int cnt = *count;
    return cnt > kMaxStaged ? kMaxStaged + 1 : cnt;
}

__device__ inline int lookup_halo(const int32_t* keys, const uint16_t* slot, int32_t c)
{
    uint32_t h = tile_hash(c);
    while (keys[h] != c) h = (h + 1) & (kHashSlots - 1);
    return slot[h];
}

// For each candidate range: its halo size (kMaxStaged + 1 when over) and its
// stencil words (rows padded to multiples of 3).
__global__ void __launch_bounds__(kTileThreads) tile_extent(const int64_t* __restrict__ row_ptr,
                                                            const int32_t* __restrict__ col,
                                                            const int64_t* __restrict__ ranges,
                                                            uint32_t* __restrict__ halo_words)
{
    __shared__ int32_t keys[kHashSlots];
    __shared__ int32_t hlist[kMaxStaged];
    __shared__ int count;
    __shared__ unsigned long long words;
    const int t = (int)threadIdx.x;
    const int tb = xcd_tile((int)blockIdx.x, (int)gridDim.x);   // XCD-contiguous ranges
    const int64_t b = ranges[2 * tb], e = ranges[2 * tb + 1];
    for (int i = t; i < kHashSlots; i += kTileThreads) keys[i] = -1;
    if (t == 0) {
        count = 0;
        words = 0;
    }
    __syncthreads();
    unsigned long long w = 0;
    for (int64_t r = b + t; r < e; r += kTileThreads) w += (uint64_t)((row_ptr[r + 1] - row_ptr[r] + 2) / 3);
    atomicAdd(&words, w);
    int H = kMaxStaged + 1;
    if (e - b <= kMaxStaged) H = gather_halo(row_ptr, col, b, e, keys, hlist, &count, t);
    __syncthreads();
    if (t == 0) {
        halo_words[2 * tb] = (uint32_t)H;
        halo_words[2 * tb + 1] = (uint32_t)(words > 0xffffffffull ? 0xffffffffull : words);
    }
}

// In-LDS bitonic sort of m (<= 1024) 64-bit keys, padded with ~0 to a power of two.
__device__ inline void bitonic_sort64(uint64_t* s, int m, int t)
{
    int p2 = 1;
    while (p2 < m) p2 <<= 1;
    for (int i = m + t; i < p2; i += kTileThreads) s[i] = ~0ull;
    __syncthreads();
    for (int size = 2; size <= p2; size <<= 1)
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = t; i < p2; i += kTileThreads) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const uint64_t a = s[i], c = s[j];
                    if ((a > c) == up) {
                        s[i] = c;
                        s[j] = a;
                    }
                }
            }
            __syncthreads();
        }
}

// Block-wide exclusive sum of per-lane values; returns the lane's prefix and
// leaves the total in *total.
__device__ inline uint32_t block_excl(uint32_t v, uint32_t* s, uint32_t* total, int t)
{
    s[t] = v;
    __syncthreads();
    for (int off = 1; off < kTileThreads; off <<= 1) {
        const uint32_t u = t >= off ? s[t - off] : 0u;
        __syncthreads();
        s[t] += u;
        __syncthreads();
    }
    const uint32_t incl = s[t];
    if (t == kTileThreads - 1) *total = incl;
    __syncthreads();
    return incl - v;
}

// One tile per workgroup.  WRITE = false: the record's counts go to
// counts[4 t] = {nw, nr, nx, nwf}, and each row (its neighbours' slots,
// ascending, padded with the point's own slot) to rowbuf from row_base[t].
// WRITE = true: the record is written at rec + 16 meta[t].rec_off, the rows
// read back from rowbuf.
template <bool WRITE>
__global__ void __launch_bounds__(kTileThreads) tile_record(const int64_t* __restrict__ row_ptr,
                                                            const int32_t* __restrict__ col,
                                                            const uint32_t* __restrict__ perm,
                                                            const int64_t* __restrict__ ranges,
                                                            const int64_t* __restrict__ row_base,
                                                            uint16_t* __restrict__ rowbuf,
                                                            uint32_t* __restrict__ counts,
                                                            const TileMeta* __restrict__ meta,
                                                            unsigned char* __restrict__ rec)
{
    // srt (sort keys: (caller index << 32) | payload) and hlist (halo in
    // insertion order) until the halo is sorted, then each lane's row scratch
    __shared__ __align__(16) unsigned char ubuf[kRowScratch * kTileThreads * 2];
    static_assert(sizeof(ubuf) >= kMaxStaged * 12, "srt and hlist fit the shared buffer");
    uint64_t* srt = reinterpret_cast<uint64_t*>(ubuf);
    int32_t* hlist = reinterpret_cast<int32_t*>(ubuf + 8 * kMaxStaged);
    uint16_t* rscr = reinterpret_cast<uint16_t*>(ubuf);   // entry k of lane t's row at rscr[k * kTileThreads + t]
    __shared__ int32_t keys[kHashSlots];            // halo hash set (Morton positions)
    __shared__ uint16_t hslot[kHashSlots];          // their slots
    __shared__ uint32_t caller[kMaxStaged];         // caller index of each staged slot
    __shared__ uint16_t own_slot[kMaxStaged];       // slot of own point b + i
    __shared__ int32_t order[kMaxStaged];           // Morton position of own slot l
    __shared__ uint32_t scan_s[kTileThreads];
    __shared__ uint32_t total;
    __shared__ int count;
    __shared__ uint32_t rowoff[kMaxStaged + 1];     // row l's first entry in the tile's row buffer
    __shared__ uint8_t expl[kMaxStaged];
    __shared__ uint8_t start[kMaxStaged];
    __shared__ uint32_t gmask[kMaxStaged / 32];    // the record's 32-slot group masks
    const int t = (int)threadIdx.x;
    const int tb = xcd_tile((int)blockIdx.x, (int)gridDim.x);   // XCD-contiguous tiles
    const int64_t b = ranges[2 * tb], e = ranges[2 * tb + 1];
    const int P = (int)(e - b);
    for (int i = t; i < kHashSlots; i += kTileThreads) keys[i] = -1;
    if (t == 0) count = 0;
    __syncthreads();
    // own points in caller order
    for (int i = t; i < P; i += kTileThreads) srt[i] = ((uint64_t)perm[b + i] << 32) | (uint32_t)i;
    bitonic_sort64(srt, P, t);
    for (int l = t; l < P; l += kTileThreads) {
        const int i = (int)(srt[l] & 0xffffffffu);
        order[l] = (int32_t)(b + i);
        own_slot[i] = (uint16_t)l;
        caller[l] = (uint32_t)(srt[l] >> 32);
    }
    __syncthreads();
    // the halo in caller order (the extents admitted only tiles with P + H <= kMaxStaged)
    const int H = gather_halo(row_ptr, col, b, e, keys, hlist, &count, t);
    if (P + H > kMaxStaged) {
        if (!WRITE && t == 0)
            for (int q = 0; q < 4; ++q) counts[4 * tb + q] = ~0u;
        return;
    }
    for (int h = t; h < H; h += kTileThreads) srt[h] = ((uint64_t)perm[hlist[h]] << 32) | (uint32_t)hlist[h];
    bitonic_sort64(srt, H, t);
    for (int h = t; h < H; h += kTileThreads) {
        const int32_t c = (int32_t)(srt[h] & 0xffffffffu);
        caller[P + h] = (uint32_t)(srt[h] >> 32);
        uint32_t q = tile_hash(c);
        while (keys[q] != c) q = (q + 1) & (kHashSlots - 1);
        hslot[q] = (uint16_t)(P + h);
    }
    __syncthreads();
    const int S = P + H;
    const TileMeta m = WRITE ? meta[tb] : TileMeta{};
    const RecLayout R = WRITE ? rec_layout(m) : RecLayout{};
    unsigned char* out = WRITE ? rec + (size_t)16 * m.rec_off : nullptr;
    // runs of consecutive caller indices
    for (int l = t; l < S; l += kTileThreads) start[l] = (l == 0 || caller[l] != caller[l - 1] + 1u) ? 1 : 0;
    __syncthreads();
    {
        // lane t takes slots [t*cs, (t+1)*cs)
        const int cs = (S + kTileThreads - 1) / kTileThreads;
        uint32_t c = 0;
        for (int l = t * cs; l < min(S, (t + 1) * cs); ++l) c += start[l];
        uint32_t k = block_excl(c, scan_s, &total, t);
        if (WRITE)
            for (int l = t * cs; l < min(S, (t + 1) * cs); ++l)
                if (start[l]) reinterpret_cast<uint32_t*>(out + R.runs)[k++] = caller[l] - (uint32_t)l;
    }
    const uint32_t nr = total;
    if (WRITE) {
        // group masks by one lane each, then their prefix counts by one lane
        for (int g = t; g < (S + 31) / 32; g += kTileThreads) {
            uint32_t mask = 0;
            for (int i = 0; i < 32 && 32 * g + i < S; ++i) mask |= (uint32_t)start[32 * g + i] << i;
            gmask[g] = mask;
        }
        __syncthreads();
        if (t == 0) {
            uint32_t before = 0;
            for (int g = 0; g < (S + 31) / 32; ++g) {
                reinterpret_cast<uint32_t*>(out + R.smask)[g] = gmask[g];
                reinterpret_cast<uint16_t*>(out + R.spre)[g] = (uint16_t)before;
                before += (uint32_t)__popc(gmask[g]);
            }
        }
        __syncthreads();
    }
    // rows: padded lengths and their offsets
    {
        const int cs = (P + kTileThreads - 1) / kTileThreads;
        uint32_t c = 0;
        for (int l = t * cs; l < min(P, (t + 1) * cs); ++l) {
            const int64_t r = order[l];
            c += (uint32_t)((row_ptr[r + 1] - row_ptr[r] + 2) / 3 * 3);
        }
        uint32_t o = block_excl(c, scan_s, &total, t);
        for (int l = t * cs; l < min(P, (t + 1) * cs); ++l) {
            rowoff[l] = o;
            const int64_t r = order[l];
            o += (uint32_t)((row_ptr[r + 1] - row_ptr[r] + 2) / 3 * 3);
        }
        if (t == 0) rowoff[P] = total;
    }
    __syncthreads();
    const uint32_t nwf = rowoff[P] / 3;
    uint16_t* rows = rowbuf + row_base[tb];
    if (!WRITE) {
        // each row: its neighbours' slots, insertion-sorted, then the padding
        for (int l = t; l < P; l += kTileThreads) {
            const int64_t r = order[l];
            uint16_t* row = rows + rowoff[l];
            const int padded = (int)(rowoff[l + 1] - rowoff[l]);
            // sorted in the lane's LDS scratch when it fits, else in place
            const bool scratch = padded <= kRowScratch;
            uint16_t* srow = scratch ? rscr + t : row;
            const int step = scratch ? kTileThreads : 1;
            int len = 0;
            const int64_t p0 = row_ptr[r], p1 = row_ptr[r + 1];
            for (int64_t p = p0; p < p1; p += kChunk) {
                int32_t cs[kChunk];
#pragma unroll
                for (int q = 0; q < kChunk; ++q) cs[q] = col[min(p + q, p1 - 1)];
                for (int q = 0; q < kChunk && p + q < p1; ++q) {
                    const int32_t c = cs[q];
                    const uint16_t s = (c >= b && c < e) ? own_slot[c - b] : (uint16_t)lookup_halo(keys, hslot, c);
                    int k = len;
                    while (k > 0 && srow[(k - 1) * step] > s) {
                        srow[k * step] = srow[(k - 1) * step];
                        --k;
                    }
                    srow[k * step] = s;
                    ++len;
                }
            }
            if (scratch)
                for (int k = 0; k < len; ++k) row[k] = srow[k * step];
            for (int k = len; k < padded; ++k) row[k] = (uint16_t)l;
        }
        __syncthreads();
    }
    // explicit rows: not the previous row with every entry plus one
    for (int l = t; l < P; l += kTileThreads) {
        bool shift = false;
        if (l > 0 && rowoff[l + 1] - rowoff[l] == rowoff[l] - rowoff[l - 1]) {
            shift = true;
            for (uint32_t k = 0; shift && k < rowoff[l + 1] - rowoff[l]; ++k)
                shift = rows[rowoff[l] + k] == (uint16_t)(rows[rowoff[l - 1] + k] + 1);
        }
        expl[l] = shift ? 0 : 1;
    }
    __syncthreads();
    // explicit rows' numbers and word offsets
    uint32_t nx, nw;
    {
        const int cs = (P + kTileThreads - 1) / kTileThreads;
        uint32_t c = 0, cw = 0;
        for (int l = t * cs; l < min(P, (t + 1) * cs); ++l)
            if (expl[l]) {
                ++c;
                cw += (rowoff[l + 1] - rowoff[l]) / 3;
            }
        uint32_t kx = block_excl(c, scan_s, &total, t);
        nx = total;
        uint32_t kw = block_excl(cw, scan_s, &total, t);
        nw = total;
        if (WRITE) {
            uint32_t* wd = reinterpret_cast<uint32_t*>(out);
            uint16_t* xend = reinterpret_cast<uint16_t*>(out + R.xend);
            for (int l = t * cs; l < min(P, (t + 1) * cs); ++l) {
                if (!expl[l]) continue;
                const uint32_t len = rowoff[l + 1] - rowoff[l];
                const uint16_t* row = rows + rowoff[l];
                const uint32_t pad = len ? (len - (uint32_t)(row_ptr[order[l] + 1] - row_ptr[order[l]])) : 0;
                for (uint32_t k = 0; k < len; k += 3) {
                    uint32_t word = (uint32_t)row[k] | (uint32_t)row[k + 1] << 10 | (uint32_t)row[k + 2] << 20;
                    if (k + 3 == len) word |= pad << 30;
                    wd[kw++] = word;
                }
                xend[kx++] = (uint16_t)kw;
            }
        }
    }
    if (WRITE) {
        for (int q = t; q < (P + 31) / 32; q += kTileThreads) {
            uint32_t mask = 0;
            for (int i = 0; i < 32 && 32 * q + i < P; ++i) mask |= (uint32_t)expl[32 * q + i] << i;
            gmask[q] = mask;
        }
        __syncthreads();
        if (t == 0) {
            uint32_t before = 0, last = 0;   // explicit rows before group q, and the last of them
            for (int q = 0; q < (P + 31) / 32; ++q) {
                const uint32_t mask = gmask[q];
                reinterpret_cast<uint32_t*>(out + R.xmask)[q] = mask;
                reinterpret_cast<uint16_t*>(out + R.xpre)[q] = (uint16_t)before;
                reinterpret_cast<uint16_t*>(out + R.xlast)[q] = (uint16_t)last;
                before += (uint32_t)__popc(mask);
                if (mask) last = 32u * (uint32_t)q + 31u - (uint32_t)__clz(mask);
            }
        }
    } else if (t == 0) {
        counts[4 * tb] = nw;
        counts[4 * tb + 1] = nr;
        counts[4 * tb + 2] = nx;
        counts[4 * tb + 3] = nwf;
    }
}

// The float64 inverse of each point's normal matrix M = sum (x_j - x_i)(x_j - x_i)^T
// over its row (Morton positions), in caller order, NaN where the rank test fails.
template <typename T>
__global__ void __launch_bounds__(256) normal_inverse(const int64_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col,
                                                      const uint32_t* __restrict__ perm, const T* __restrict__ x,
                                                      int64_t n, double tau, T* __restrict__ out)
{
#pragma clang fp contract(off)
    const int64_t r = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * 256 + threadIdx.x;
    if (r >= n) return;
    const int64_t i = perm[r];
    const double xi0 = (double)x[i * 3], xi1 = (double)x[i * 3 + 1], xi2 = (double)x[i * 3 + 2];
    double m00 = 0, m01 = 0, m02 = 0, m11 = 0, m12 = 0, m22 = 0;
    for (int64_t p = row_ptr[r]; p < row_ptr[r + 1]; ++p) {
        const int64_t j = perm[col[p]];
        const double d0 = (double)x[j * 3] - xi0, d1 = (double)x[j * 3 + 1] - xi1, d2 = (double)x[j * 3 + 2] - xi2;
        m00 += d0 * d0;
        m01 += d0 * d1;
        m02 += d0 * d2;
        m11 += d1 * d1;
        m12 += d1 * d2;
        m22 += d2 * d2;
    }
    const double a00 = m11 * m22 - m12 * m12, a01 = m02 * m12 - m01 * m22, a02 = m01 * m12 - m02 * m11;
    const double a11 = m00 * m22 - m02 * m02, a12 = m01 * m02 - m00 * m12, a22 = m00 * m11 - m01 * m01;
    const double det = m00 * a00 + m01 * a01 + m02 * a02;
    const double tr3 = (m00 + m11 + m22) / 3.0;
    double v[6] = {a00 / det, a01 / det, a02 / det, a11 / det, a12 / det, a22 / det};
    if (!(det > tau * tr3 * tr3 * tr3))
        for (double& q : v) q = __builtin_nan("");
#pragma unroll
    for (int k = 0; k < 6; ++k) out[i * 6 + k] = (T)v[k];
}

// ---------------------------------------------------------------------------
// The axis stencil over Morton positions (FTLE_STENCIL_AXIS), as the host
// builds it: per signed axis direction the one-ring neighbour on that side
// with the largest cosine to the axis (float64, no contraction, ties to the
// smaller caller index), in slot order (-x, +x, -y, +y[, -z, +z]), absent
// sides dropped, a neighbour chosen twice listed twice.
// ---------------------------------------------------------------------------
template <int D, typename T>
__global__ void __launch_bounds__(256) axis_slots(const T* __restrict__ x, const uint32_t* __restrict__ perm,
                                                  const int64_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                                  int64_t n, int32_t* __restrict__ slots, uint32_t* __restrict__ cnt)
{
#pragma clang fp contract(off)
    const int64_t r = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * 256 + threadIdx.x;
    if (r >= n) return;
    const int64_t i = perm[r];
    double xi[D];
#pragma unroll
    for (int d = 0; d < D; ++d) xi[d] = (double)x[i * D + d];
    int32_t best[2 * D];
    uint32_t best_u[2 * D];
    double best_c[2 * D];
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) {
        best[k] = -1;
        best_u[k] = 0;
        best_c[k] = 0.0;
    }
    for (int64_t p = row_ptr[r]; p < row_ptr[r + 1]; ++p) {
        const int32_t c = col[p];
        const uint32_t j = perm[c];
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
                const double cs = along / nrm;
                const int k = 2 * d + sg;
                if (best[k] < 0 || cs > best_c[k] || (cs == best_c[k] && j < best_u[k])) {
                    best_c[k] = cs;
                    best[k] = c;
                    best_u[k] = j;
                }
            }
    }
    uint32_t m = 0;
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) {
        slots[r * 2 * D + k] = best[k];
        m += best[k] >= 0 ? 1u : 0u;
    }
    cnt[r] = m;
}

template <int D>
__global__ void __launch_bounds__(256) axis_fill(const int32_t* __restrict__ slots, const int64_t* __restrict__ row_ptr,
                                                 int64_t n, int32_t* __restrict__ col)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    int64_t q = row_ptr[r];
#pragma unroll
    for (int k = 0; k < 2 * D; ++k) {
        const int32_t c = slots[r * 2 * D + k];
        if (c >= 0) col[q++] = c;
    }
}

// Transpose of a CSR over Morton positions: column counts, then (after their
// scan) each entry placed by an atomic cursor, then each row sorted (rows
// ascend, as the host's counting transpose leaves them).
__global__ void __launch_bounds__(256) transpose_count(const int32_t* __restrict__ col, int64_t nnz,
                                                       uint32_t* __restrict__ tcnt)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p < nnz) atomicAdd(&tcnt[col[p]], 1u);
}

__global__ void __launch_bounds__(256) transpose_fill(const int64_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col, int64_t n,
                                                      const int64_t* __restrict__ trp, uint32_t* __restrict__ cur,
                                                      int32_t* __restrict__ tcol)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    for (int64_t p = row_ptr[r]; p < row_ptr[r + 1]; ++p) {
        const int32_t c = col[p];
        tcol[trp[c] + atomicAdd(&cur[c], 1u)] = (int32_t)r;
    }
}

__global__ void __launch_bounds__(256) sort_rows(const int64_t* __restrict__ row_ptr, int64_t n,
                                                 int32_t* __restrict__ col)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    int32_t* row = col + row_ptr[r];
    const int64_t len = row_ptr[r + 1] - row_ptr[r];
    for (int64_t a = 1; a < len; ++a) {
        const int32_t v = row[a];
        int64_t k = a;
        while (k > 0 && row[k - 1] > v) {
            row[k] = row[k - 1];
            --k;
        }
        row[k] = v;
    }
}

// *differ = 1 where two CSRs of n rows and nnz entries differ
__global__ void __launch_bounds__(256) csr_compare(const int64_t* __restrict__ rp_a, const int32_t* __restrict__ col_a,
                                                   const int64_t* __restrict__ rp_b, const int32_t* __restrict__ col_b,
                                                   int64_t n, int64_t nnz, int* __restrict__ differ)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if ((i <= n && rp_a[i] != rp_b[i]) || (i < nnz && col_a[i] != col_b[i])) *differ = 1;
}

// ---------------------------------------------------------------------------
// A caller's CSR over caller indices moved to Morton positions: per Morton
// row r (caller row perm[r]) the entries that are neither -1 nor the point
// itself, renumbered and sorted ascending (repeats kept).  The count pass also
// checks the input: err[0] lowers to 0 for row_ptr[0] != 0 and to i + 1 for a
// row i whose end precedes its start; err[1] lowers to the position of an
// entry outside [-1, n).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) csr_in_count(const int64_t* __restrict__ row_ptr,
                                                    const int32_t* __restrict__ col, int64_t n, int64_t nnz_in,
                                                    const uint32_t* __restrict__ perm, uint32_t* __restrict__ cnt,
                                                    unsigned long long* __restrict__ err)
{
    const int64_t r = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * 256 + threadIdx.x;
    if (r >= n) return;
    if (r == 0 && row_ptr[0] != 0) atomicMin(&err[0], 0ull);
    const int64_t i = perm[r];
    const int64_t p0 = row_ptr[i], p1 = row_ptr[i + 1];
    uint32_t c = 0;
    if (p1 < p0) {
        atomicMin(&err[0], (unsigned long long)(i + 1));
    } else if (p0 >= 0 && p1 <= nnz_in) {
        for (int64_t p = p0; p < p1; ++p) {
            const int32_t v = col[p];
            if (v < -1 || v >= n)
                atomicMin(&err[1], (unsigned long long)p);
            else if (v >= 0 && v != (int32_t)i)
                ++c;
        }
    }
    cnt[r] = c;
}

__global__ void __launch_bounds__(256) csr_in_fill(const int64_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col, int64_t n,
                                                   const uint32_t* __restrict__ perm, const int32_t* __restrict__ inv,
                                                   const int64_t* __restrict__ out_rp, int32_t* __restrict__ out)
{
    const int64_t r = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * 256 + threadIdx.x;
    if (r >= n) return;
    const int64_t i = perm[r];
    int32_t* row = out + out_rp[r];
    int64_t len = 0;
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
        const int32_t v = col[p];
        if (v < 0 || v == (int32_t)i) continue;
        const int32_t u = inv[v];
        int64_t k = len;
        while (k > 0 && row[k - 1] > u) {
            row[k] = row[k - 1];
            --k;
        }
        row[k] = u;
        ++len;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers (ftle_internal.h)
// ---------------------------------------------------------------------------
hipError_t mb_bbox(int dim, bool f64, const void* x, int64_t n, double* part, int nblocks,
                   unsigned long long* first_bad, hipStream_t s)
{
#define FTLE_MB(D, T) hipLaunchKernelGGL((bbox_partial<D, T>), dim3(nblocks), dim3(256), 0, s, static_cast<const T*>(x), n, part, first_bad)
    if (dim == 2) {
        if (f64) FTLE_MB(2, double); else FTLE_MB(2, float);
    } else {
        if (f64) FTLE_MB(3, double); else FTLE_MB(3, float);
    }
#undef FTLE_MB
    return hipGetLastError();
}

hipError_t mb_gather_pairs(int dim, bool f64, const void* x, int64_t m, int64_t stride, double* out, hipStream_t s)
{
    if (m <= 0) return hipSuccess;
#define FTLE_MB(D, T) hipLaunchKernelGGL((gather_pairs<D, T>), dim3(blocks_of(m, 256)), dim3(256), 0, s, static_cast<const T*>(x), m, stride, out)
    if (dim == 2) {
        if (f64) FTLE_MB(2, double); else FTLE_MB(2, float);
    } else {
        if (f64) FTLE_MB(3, double); else FTLE_MB(3, float);
    }
#undef FTLE_MB
    return hipGetLastError();
}

hipError_t mb_morton(int dim, bool f64, const void* x, int64_t n, const MortonParams& mp, uint64_t* key,
                     uint32_t* val, hipStream_t s)
{
#define FTLE_MB(D, T) hipLaunchKernelGGL((morton_keys<D, T>), dim3(blocks_of(n, 256)), dim3(256), 0, s, static_cast<const T*>(x), n, mp, key, val)
    if (dim == 2) {
        if (f64) FTLE_MB(2, double); else FTLE_MB(2, float);
    } else {
        if (f64) FTLE_MB(3, double); else FTLE_MB(3, float);
    }
#undef FTLE_MB
    return hipGetLastError();
}

size_t mb_sort_scratch_bytes(int64_t n)
{
    const int64_t tiles = (n + kRadixTile - 1) / kRadixTile;
    const size_t h = (size_t)256 * tiles + 1;
    return 8 * (size_t)n + 4 * (size_t)n + ((4 * h + 255) & ~(size_t)255) + scan_partial_bytes((int64_t)h) + 256;
}

hipError_t mb_sort(uint64_t* key, uint32_t* val, int64_t n, int key_bits, void* scratch, uint32_t** sorted_val,
                   hipStream_t s)
{
    unsigned char* w = static_cast<unsigned char*>(scratch);
    uint64_t* key2 = reinterpret_cast<uint64_t*>(w);
    uint32_t* val2 = reinterpret_cast<uint32_t*>(w + 8 * (size_t)n);
    const int64_t tiles = (n + kRadixTile - 1) / kRadixTile;
    const int64_t h = 256 * tiles;
    uint32_t* hist = reinterpret_cast<uint32_t*>(w + 12 * (size_t)n);
    uint32_t* partial = reinterpret_cast<uint32_t*>(w + 12 * (size_t)n + ((4 * (size_t)(h + 1) + 255) & ~(size_t)255));
    hipError_t e;
    for (int shift = 0; shift < key_bits; shift += 8) {
        hipLaunchKernelGGL(radix_hist, dim3((unsigned)tiles), dim3(kRadixThreads), 0, s, key, n, shift,
                           (uint32_t)tiles, hist);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = scan_exclusive_u32(hist, h, hist, partial, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(radix_scatter, dim3((unsigned)tiles), dim3(kRadixThreads), 0, s, key, val, n, shift,
                           (uint32_t)tiles, hist, key2, val2);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        std::swap(key, key2);
        std::swap(val, val2);
    }
    *sorted_val = val;
    return hipSuccess;
}

hipError_t mb_iota(uint32_t* v, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(iota_u32, dim3(blocks_of(n, 256)), dim3(256), 0, s, v, n);
    return hipGetLastError();
}

hipError_t mb_invert(const uint32_t* perm, int64_t n, int32_t* inv, hipStream_t s)
{
    hipLaunchKernelGGL(invert_perm, dim3(blocks_of(n, 256)), dim3(256), 0, s, perm, n, inv);
    return hipGetLastError();
}

hipError_t mb_relabel(int dim, const int32_t* cells, int64_t n_cells, int64_t n, const int32_t* inv, int32_t* mc,
                      int* flag, unsigned long long* first, hipStream_t s)
{
    if (n_cells == 0) return hipSuccess;
    if (dim == 2)
        hipLaunchKernelGGL(check_relabel<3>, dim3(blocks_of(n_cells, 256)), dim3(256), 0, s, cells, n_cells, n, inv, mc,
                           flag, first);
    else
        hipLaunchKernelGGL(check_relabel<4>, dim3(blocks_of(n_cells, 256)), dim3(256), 0, s, cells, n_cells, n, inv, mc,
                           flag, first);
    return hipGetLastError();
}

hipError_t mb_tile_extent(const int64_t* row_ptr, const int32_t* col, const int64_t* ranges, int64_t n_ranges,
                          uint32_t* halo_words, hipStream_t s)
{
    if (n_ranges == 0) return hipSuccess;
    hipLaunchKernelGGL(tile_extent, dim3((unsigned)n_ranges), dim3(kTileThreads), 0, s, row_ptr, col, ranges,
                       halo_words);
    return hipGetLastError();
}

hipError_t mb_tile_record(bool write, const int64_t* row_ptr, const int32_t* col, const uint32_t* perm,
                          const int64_t* ranges, int64_t n_tiles, const int64_t* row_base, uint16_t* rowbuf,
                          uint32_t* counts, const TileMeta* meta, unsigned char* rec, hipStream_t s)
{
    if (n_tiles == 0) return hipSuccess;
    if (write)
        hipLaunchKernelGGL(tile_record<true>, dim3((unsigned)n_tiles), dim3(kTileThreads), 0, s, row_ptr, col, perm,
                           ranges, row_base, rowbuf, counts, meta, rec);
    else
        hipLaunchKernelGGL(tile_record<false>, dim3((unsigned)n_tiles), dim3(kTileThreads), 0, s, row_ptr, col, perm,
                           ranges, row_base, rowbuf, counts, meta, rec);
    return hipGetLastError();
}

hipError_t mb_normal_inverse(bool f64, const int64_t* row_ptr, const int32_t* col, const uint32_t* perm,
                             const void* x, int64_t n, void* out, hipStream_t s)
{
    if (f64)
        hipLaunchKernelGGL(normal_inverse<double>, dim3(blocks_of(n, 256)), dim3(256), 0, s, row_ptr, col, perm,
                           static_cast<const double*>(x), n, 1e-12, static_cast<double*>(out));
    else
        hipLaunchKernelGGL(normal_inverse<float>, dim3(blocks_of(n, 256)), dim3(256), 0, s, row_ptr, col, perm,
                           static_cast<const float*>(x), n, 1e-5, static_cast<float*>(out));
    return hipGetLastError();
}

hipError_t mb_axis_stencil(int dim, bool f64, const void* x, const uint32_t* perm, const int64_t* ring_rp,
                           const int32_t* ring_col, int64_t n, int32_t* slots, uint32_t* cnt, hipStream_t s)
{
    const dim3 g(blocks_of(n, 256)), b(256);
    if (dim == 2) {
        if (f64)
            hipLaunchKernelGGL((axis_slots<2, double>), g, b, 0, s, static_cast<const double*>(x), perm, ring_rp,
                               ring_col, n, slots, cnt);
        else
            hipLaunchKernelGGL((axis_slots<2, float>), g, b, 0, s, static_cast<const float*>(x), perm, ring_rp,
                               ring_col, n, slots, cnt);
    } else {
        if (f64)
            hipLaunchKernelGGL((axis_slots<3, double>), g, b, 0, s, static_cast<const double*>(x), perm, ring_rp,
                               ring_col, n, slots, cnt);
        else
            hipLaunchKernelGGL((axis_slots<3, float>), g, b, 0, s, static_cast<const float*>(x), perm, ring_rp,
                               ring_col, n, slots, cnt);
    }
    return hipGetLastError();
}

hipError_t mb_axis_fill(int dim, const int32_t* slots, const int64_t* row_ptr, int64_t n, int32_t* col, hipStream_t s)
{
    if (dim == 2)
        hipLaunchKernelGGL(axis_fill<2>, dim3(blocks_of(n, 256)), dim3(256), 0, s, slots, row_ptr, n, col);
    else
        hipLaunchKernelGGL(axis_fill<3>, dim3(blocks_of(n, 256)), dim3(256), 0, s, slots, row_ptr, n, col);
    return hipGetLastError();
}

hipError_t mb_transpose_count(const int32_t* col, int64_t nnz, uint32_t* tcnt, hipStream_t s)
{
    if (nnz == 0) return hipSuccess;
    hipLaunchKernelGGL(transpose_count, dim3(blocks_of(nnz, 256)), dim3(256), 0, s, col, nnz, tcnt);
    return hipGetLastError();
}

hipError_t mb_transpose_fill(const int64_t* row_ptr, const int32_t* col, int64_t n, const int64_t* trp, uint32_t* cur,
                             int32_t* tcol, hipStream_t s)
{
    hipLaunchKernelGGL(transpose_fill, dim3(blocks_of(n, 256)), dim3(256), 0, s, row_ptr, col, n, trp, cur, tcol);
    hipLaunchKernelGGL(sort_rows, dim3(blocks_of(n, 256)), dim3(256), 0, s, trp, n, tcol);
    return hipGetLastError();
}

hipError_t mb_csr_compare(const int64_t* rp_a, const int32_t* col_a, const int64_t* rp_b, const int32_t* col_b,
                          int64_t n, int64_t nnz, int* differ, hipStream_t s)
{
    const int64_t m = std::max<int64_t>(n + 1, nnz);
    hipLaunchKernelGGL(csr_compare, dim3(blocks_of(m, 256)), dim3(256), 0, s, rp_a, col_a, rp_b, col_b, n, nnz, differ);
    return hipGetLastError();
}

hipError_t mb_csr_in_count(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz_in, const uint32_t* perm,
                           uint32_t* cnt, unsigned long long* err, hipStream_t s)
{
    hipLaunchKernelGGL(csr_in_count, dim3(blocks_of(n, 256)), dim3(256), 0, s, row_ptr, col, n, nnz_in, perm, cnt, err);
    return hipGetLastError();
}

hipError_t mb_csr_in_fill(const int64_t* row_ptr, const int32_t* col, int64_t n, const uint32_t* perm,
                          const int32_t* inv, const int64_t* out_rp, int32_t* out, hipStream_t s)
{
    hipLaunchKernelGGL(csr_in_fill, dim3(blocks_of(n, 256)), dim3(256), 0, s, row_ptr, col, n, perm, inv, out_rp, out);
    return hipGetLastError();
}

}  // namespace ftle
