// The one-ring stencil of a cell mesh built on the GPU: the neighbour
// determination that precedes the FTLE path (Section 2.2 keeps it on the host,
// off the accelerator; the Conclusions list accelerating it as future work).
// Every point's neighbours are the other points sharing a cell with it,
// ascending, each once.  Hand-written kernels, no library sort:
//
//   1. incidence lists in one pass: each cell appends its index to the list
//      of each of its K = dim + 1 points, a list of at most 16 (triangles)
//      or 32 (tetrahedra) entries per point at a fixed place (atomic
//      cursors, one per distinct point of a workgroup, aggregated in LDS
//      first; the order inside a list does not matter; an index outside
//      [0, n) raises the error flag).  When a point has more incident cells
//      than that, or the fixed lists would not be addressable in 32 bits,
//      the lists are packed instead:
//   2. the counts (from the first pass, or from a counting pass) are scanned
//      into each point's incidence offset (scan_tiles / scan_partials /
//      add_partials: 2048-element tiles, the tiles' sums scanned by one
//      workgroup, then added back), and
//   3. a second pass appends each cell's index to its points' packed lists;
//   4. rows: one lane per point walks its incident cells and inserts their
//      other points into a short sorted list of distinct indices in LDS, each
//      one's place found by binary search (a lane's list is interleaved with
//      its workgroup's, so that a list step is one conflict-free LDS access),
//      then stores its count and the list (a fixed kRowCap slots per point in
//      the workspace); the counts are scanned into the row pointers, and a
//      copy moves the lists into place.
//      A point with more than kRowCap distinct neighbours is handed to a
//      workgroup of its own (long_rows: its candidates sorted by a bitonic
//      network in LDS, duplicates dropped by a flag scan), once to count and
//      once to write.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "ftle_device_math.h"
#include "ftle_internal.h"

namespace ftle {
namespace {

constexpr int kScanThreads = 256, kScanItems = 8, kScanTile = kScanThreads * kScanItems;
constexpr int kRowThreads = 128;   // lanes per workgroup of the row passes
constexpr int kRowCap = 32;        // distinct neighbours a lane keeps in LDS
constexpr int kLongCap = 4096;     // candidates (with repeats) of a long row
constexpr uint32_t kIncCap2 = 16, kIncCap3 = 32;   // fixed incidence list length (triangles, tetrahedra)

inline unsigned blocks_for(int64_t m, int per = 256) { return (unsigned)((m + per - 1) / per); }

// The points of cell c (tetrahedra: one 16-byte load when the array is
// 16-byte aligned, a workgroup-uniform test).
template <int K>
__device__ inline void load_cell(const int32_t* __restrict__ cells, int64_t c, int32_t (&v)[K])
{
    if (K == 4 && (reinterpret_cast<uintptr_t>(cells) & 15) == 0) {
        const int4 q = reinterpret_cast<const int4*>(cells)[c];
        v[0] = q.x, v[1] = q.y, v[2] = q.z;
        if constexpr (K == 4) v[3] = q.w;
    } else {
#pragma unroll
        for (int a = 0; a < K; ++a) v[a] = cells[c * K + a];
    }
}

// 1 and 3.  A workgroup takes kAggCells cells per lane and first gathers their
// points' occurrences in an LDS hash table (open addressing, keys inserted by
// compare-and-swap), so that each distinct point of the workgroup's cells
// costs one global atomic instead of one per occurrence: cells come in mesh
// order, and neighbouring cells share most of their points.  A point that
// finds no slot within kProbes probes goes to global memory directly.
//   kCount:  cnt[v] += occurrences of v (a cell with an index outside [0, n)
//            sets bit 1 of *err and adds nothing);
//   kPacked: each occurrence of v gets a position from cur[v] (the workgroup
//            reserves its block of positions with one atomic) and
//            inc[position] = its cell;
//   kFixed:  as kCount, and each occurrence of v also gets list position
//            k = the count before it, inc[v cap + k] = its cell while k < cap
//            (beyond it, bit 4 of *err and no store).
constexpr int kAggThreads = 256, kAggCells = 4, kAggSlots = 4096, kProbes = 32;
enum IncMode { kCount, kPacked, kFixed };

__device__ inline uint32_t agg_hash(int32_t v) { return ((uint32_t)v * 2654435761u) >> 20; }   // 12 bits

template <int K, int MODE>
__global__ void __launch_bounds__(kAggThreads) incidence_pass(const int32_t* __restrict__ cells, int64_t n_cells,
                                                              int64_t n, uint32_t* __restrict__ cnt,
                                                              int32_t* __restrict__ inc, int* __restrict__ err,
                                                              uint32_t cap)
{
    constexpr bool FILL = MODE != kCount;
    static_assert(kAggSlots == 1 << 12, "agg_hash gives 12 bits");
    __shared__ int32_t key[kAggSlots];
    __shared__ uint32_t num[kAggSlots];
    const int t = (int)threadIdx.x;
    for (int i = t; i < kAggSlots; i += kAggThreads) {
        key[i] = -1;
        num[i] = 0;
    }
    __syncthreads();
    // each XCD takes a contiguous stretch of cells (its L2 then holds their points' counters)
    const int64_t c0 = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * (kAggThreads * kAggCells);
    int slot[kAggCells][K];
    uint32_t local[kAggCells][K];
#pragma unroll
    for (int q = 0; q < kAggCells; ++q) {
        const int64_t c = c0 + q * kAggThreads + t;
        int32_t v[K];
        bool ok = c < n_cells;
        if (ok) {
            load_cell<K>(cells, c, v);
#pragma unroll
            for (int a = 0; a < K; ++a) ok &= (uint64_t)(int64_t)v[a] < (uint64_t)n;
            if (MODE != kPacked && !ok) atomicOr(err, 1);
        }
#pragma unroll
        for (int a = 0; a < K; ++a) {
            slot[q][a] = -2;   // nothing to do
            if (!ok) continue;
            uint32_t h = agg_hash(v[a]);
            int s = -1;
            for (int p = 0; p < kProbes; ++p, h = (h + 1) & (kAggSlots - 1)) {
                const int32_t k = atomicCAS(&key[h], -1, v[a]);
                if (k == -1 || k == v[a]) {
                    s = (int)h;
                    break;
                }
            }
            slot[q][a] = s;
            if (s >= 0) {
                local[q][a] = atomicAdd(&num[s], 1u);
            } else if (MODE == kPacked) {
                inc[atomicAdd(&cnt[v[a]], 1u)] = (int32_t)c;
            } else if (MODE == kFixed) {
                const uint32_t k = atomicAdd(&cnt[v[a]], 1u);
                if (k < cap)
                    inc[(uint32_t)v[a] * cap + k] = (int32_t)c;
                else
                    atomicOr(err, 4);
            } else {
                atomicAdd(&cnt[v[a]], 1u);
            }
        }
    }
    __syncthreads();
    for (int i = t; i < kAggSlots; i += kAggThreads) {
        const int32_t k = key[i];
        if (k < 0) continue;
        if (FILL)
            num[i] = atomicAdd(&cnt[k], num[i]);   // the block's first position
        else
            atomicAdd(&cnt[k], num[i]);
    }
    if constexpr (MODE == kPacked) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kAggCells; ++q)
#pragma unroll
            for (int a = 0; a < K; ++a)
                if (slot[q][a] >= 0) inc[num[slot[q][a]] + local[q][a]] = (int32_t)(c0 + q * kAggThreads + t);
    } else if constexpr (MODE == kFixed) {
        __syncthreads();
        bool over = false;
#pragma unroll
        for (int q = 0; q < kAggCells; ++q)
#pragma unroll
            for (int a = 0; a < K; ++a)
                if (slot[q][a] >= 0) {
                    const uint32_t k = num[slot[q][a]] + local[q][a];
                    if (k < cap)
                        inc[(uint32_t)key[slot[q][a]] * cap + k] = (int32_t)(c0 + q * kAggThreads + t);
                    else
                        over = true;
                }
        if (over) atomicOr(err, 4);
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan of m uint32 counts into out[0..m) (Out: uint32 or int64),
// with out[m] = the total.  scan_tiles scans each 2048-element tile and
// writes its sum to partial[tile]; scan_partials scans the partial sums in
// one workgroup (chunks of 1024 with a carry) and writes the total to
// out[m]; add_partials adds each tile's offset.
// ---------------------------------------------------------------------------
template <typename Out>
__device__ inline Out block_inclusive_scan(Out v, Out* s, int tid, int nthreads)
{
    s[tid] = v;
    __syncthreads();
    for (int off = 1; off < nthreads; off <<= 1) {
        const Out t = tid >= off ? s[tid - off] : Out(0);
        __syncthreads();
        s[tid] += t;
        __syncthreads();
    }
    return s[tid];
}

template <typename Out>
__global__ void __launch_bounds__(kScanThreads) scan_tiles(const uint32_t* in, int64_t m, Out* out,
                                                             Out* __restrict__ partial)   // in and out may coincide
{
    __shared__ Out s[kScanThreads];
    const int tid = (int)threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)tid * kScanItems;
    Out v[kScanItems], sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = base + k < m ? (Out)in[base + k] : Out(0);
        sum += v[k];
    }
    const Out incl = block_inclusive_scan<Out>(sum, s, tid, kScanThreads);
    Out run = incl - sum;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (base + k < m) out[base + k] = run;
        run += v[k];
    }
    if (tid == kScanThreads - 1) partial[blockIdx.x] = incl;
}

template <typename Out>
__global__ void __launch_bounds__(1024) scan_partials(Out* __restrict__ partial, int64_t np, Out* __restrict__ total)
{
    __shared__ Out s[1024];
    const int tid = (int)threadIdx.x;
    Out carry = 0;
    for (int64_t c0 = 0; c0 < np; c0 += 1024) {
        const int64_t i = c0 + tid;
        const Out v = i < np ? partial[i] : Out(0);
        const Out incl = block_inclusive_scan<Out>(v, s, tid, 1024);
        if (i < np) partial[i] = carry + incl - v;
        carry += s[1023];
        __syncthreads();
    }
    if (tid == 0) *total = carry;
}

template <typename Out>
__global__ void __launch_bounds__(256) add_partials(Out* __restrict__ out, int64_t m, const Out* __restrict__ partial)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) out[i] += partial[i / kScanTile];
}

template <typename Out>
hipError_t exclusive_scan(const uint32_t* in, int64_t m, Out* out, Out* partial, hipStream_t stream)
{
    const int64_t tiles = (m + kScanTile - 1) / kScanTile;
    if (tiles > 0)
        hipLaunchKernelGGL((scan_tiles<Out>), dim3((unsigned)tiles), dim3(kScanThreads), 0, stream, in, m, out,
                           partial);
    hipLaunchKernelGGL((scan_partials<Out>), dim3(1), dim3(1024), 0, stream, partial, tiles, out + m);
    if (tiles > 1)
        hipLaunchKernelGGL((add_partials<Out>), dim3(blocks_for(m)), dim3(256), 0, stream, out, m,
                           (const Out*)partial);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 4. rows.  Lane r (point r) keeps its distinct neighbours, ascending, in
// lst[k * kRowThreads + lane], k < kRowCap, then sets deg[r] to their count
// and stores them at store[k * n + r] (entry-major, so that each store
// instruction writes consecutive points).  A point with more is appended to
// longs (deg[r] = 0 until long_rows counts it).
// ---------------------------------------------------------------------------
// Point r's incidence list: inc[p0, p1).  *capp = 0: packed lists at the
// offsets off[r], off[r + 1]; otherwise fixed lists of *capp entries, off[r]
// of them used.
struct IncRange {
    uint32_t p0, p1;
};
__device__ inline IncRange inc_range(const uint32_t* __restrict__ off, uint32_t cap, int64_t r)
{
    if (cap) {
        const uint32_t p0 = (uint32_t)r * cap;
        return IncRange{p0, p0 + off[r]};
    }
    return IncRange{off[r], off[r + 1]};
}

template <int K>
__global__ void __launch_bounds__(kRowThreads) ring_rows(const int32_t* __restrict__ cells,
                                                         const int32_t* __restrict__ inc,
                                                         const uint32_t* __restrict__ off,
                                                         const uint32_t* __restrict__ capp, int64_t n,
                                                         uint32_t* __restrict__ deg, int32_t* __restrict__ store,
                                                         uint32_t* __restrict__ longs, uint32_t* __restrict__ n_long)
{
    __shared__ int32_t lst[kRowCap * kRowThreads];
    const int t = (int)threadIdx.x;
    const int64_t r = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * kRowThreads + t;   // XCD-contiguous rows
    if (r >= n) return;
    int32_t* my = lst + t;   // entry k at my[k * kRowThreads]
    int cnt = 0;
    bool over = false;
    const IncRange ir = inc_range(off, *capp, r);
    const uint32_t p0 = ir.p0, p1 = ir.p1;
    // incident cells kChunk at a time: their loads are issued together, then
    // their points are inserted (a cell past the end repeats the last one,
    // whose points are then found already listed)
    constexpr int kChunk = 4;
    for (uint32_t p = p0; p < p1 && !over; p += kChunk) {
        int32_t v[kChunk][K];
        int32_t c[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q) c[q] = inc[min(p + q, p1 - 1)];
#pragma unroll
        for (int q = 0; q < kChunk; ++q) load_cell<K>(cells, c[q], v[q]);
#pragma unroll
        for (int q = 0; q < kChunk; ++q)
#pragma unroll
            for (int a = 0; a < K; ++a) {
                const int32_t u = v[q][a];
                if (u == (int32_t)r || over) continue;
                // insertion point k: the number of listed entries below u, by
                // binary search (at most 6 steps for 32 entries)
                int k = 0, hi = cnt;
                while (k < hi) {
                    const int mid = (k + hi) >> 1;
                    if (my[mid * kRowThreads] < u)
                        k = mid + 1;
                    else
                        hi = mid;
                }
                if (k < cnt && my[k * kRowThreads] == u) continue;   // already listed
                if (cnt == kRowCap) {
                    over = true;
                    continue;
                }
                for (int j = cnt; j > k; --j) my[j * kRowThreads] = my[(j - 1) * kRowThreads];
                my[k * kRowThreads] = u;
                ++cnt;
            }
    }
    if (over) longs[atomicAdd(n_long, 1u)] = (uint32_t)r;
    deg[r] = over ? 0u : (uint32_t)cnt;
    if (!over)
        for (int k = 0; k < cnt; ++k) store[k * n + r] = my[k * kRowThreads];
}

// The stored lists into place: col[row_ptr[r] + k] = store[k * n + r] for the
// rows ring_rows kept (a long row's count, set by long_rows, exceeds kRowCap).
// A workgroup's 256 rows are one contiguous stretch of col: each lane puts its
// row into that stretch in LDS (long rows' entries marked -1), then the
// stretch goes out with consecutive lanes writing consecutive entries.  A
// stretch longer than kCopySeg entries (long rows in the workgroup) is
// written row by row instead.
constexpr int kCopySeg = 256 * 24;

__global__ void __launch_bounds__(256) copy_rows(const int32_t* __restrict__ store, int64_t n,
                                                 const uint32_t* __restrict__ deg,
                                                 const int64_t* __restrict__ row_ptr, int32_t* __restrict__ col)
{
    __shared__ int32_t seg[kCopySeg];
    const int t = (int)threadIdx.x;
    const int64_t r0 = (int64_t)xcd_tile((int)blockIdx.x, (int)gridDim.x) * 256, r = r0 + t;
    const int64_t r1 = min(r0 + 256, n);
    const int64_t base = row_ptr[r0], total = row_ptr[r1] - base;
    const bool live = r < n;
    const uint32_t d = live ? deg[r] : 0u;
    const bool kept = d <= (uint32_t)kRowCap;
    if (total > kCopySeg) {   // workgroup-uniform
        if (live && kept) {
            int32_t* out = col + row_ptr[r];
            for (uint32_t k = 0; k < d; ++k) out[k] = store[(int64_t)k * n + r];
        }
        return;
    }
    if (live) {
        int32_t* dst = seg + (row_ptr[r] - base);
        if (kept)
            for (uint32_t k = 0; k < d; ++k) dst[k] = store[(int64_t)k * n + r];
        else
            for (uint32_t k = 0; k < d; ++k) dst[k] = -1;
    }
    __syncthreads();
    for (int64_t e = t; e < total; e += 256) {
        const int32_t v = seg[e];
        if (v >= 0) col[base + e] = v;
    }
}

// A long row by a workgroup of 256 lanes: its candidates (the points of its
// incident cells, the point itself as a filler) sorted by a bitonic network
// in LDS, then one flag per first occurrence and their exclusive sum.  More
// than kLongCap candidates: *err |= 2 (the stencil is not built).  The
// workgroups loop over the long rows (their number is only known on the
// device).
template <int K, bool WRITE>
__global__ void __launch_bounds__(256) long_rows(const int32_t* __restrict__ cells, const int32_t* __restrict__ inc,
                                                 const uint32_t* __restrict__ off, const uint32_t* __restrict__ capp,
                                                 const uint32_t* __restrict__ longs,
                                                 const uint32_t* __restrict__ n_long, uint32_t* __restrict__ deg,
                                                 const int64_t* __restrict__ row_ptr, int32_t* __restrict__ col,
                                                 int* __restrict__ err)
{
    constexpr int kT = 256, kPer = kLongCap / kT;
    constexpr int32_t kFill = INT32_MAX;
    __shared__ int32_t s[kLongCap];
    __shared__ uint32_t part[kT];
    const int t = (int)threadIdx.x;
    const uint32_t nl = *n_long;
    for (uint32_t li = blockIdx.x; li < nl; li += gridDim.x) {
        const int64_t r = longs[li];
        const IncRange ir = inc_range(off, *capp, r);
        const uint32_t p0 = ir.p0, m = (ir.p1 - p0) * K;
        if (m > (uint32_t)kLongCap) {
            if (t == 0) atomicOr(err, 2);
            continue;
        }
        int p2 = 1;
        while (p2 < (int)m) p2 <<= 1;
        for (int i = t; i < p2; i += kT) {
            int32_t u = kFill;
            if (i < (int)m) {
                u = cells[(int64_t)inc[p0 + i / K] * K + i % K];
                if (u == (int32_t)r) u = kFill;
            }
            s[i] = u;
        }
        __syncthreads();
        for (int size = 2; size <= p2; size <<= 1)
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int i = t; i < p2; i += kT) {
                    const int j = i ^ stride;
                    if (j > i) {
                        const bool up = (i & size) == 0;
                        const int32_t a = s[i], b = s[j];
                        if ((a > b) == up) {
                            s[i] = b;
                            s[j] = a;
                        }
                    }
                }
                __syncthreads();
            }
        // lane t owns entries [t kPer, (t + 1) kPer): first occurrences, then their exclusive sum
        uint32_t c = 0;
        for (int k = 0; k < kPer; ++k) {
            const int i = t * kPer + k;
            c += (i < p2 && s[i] != kFill && (i == 0 || s[i] != s[i - 1])) ? 1u : 0u;
        }
        const uint32_t incl = block_inclusive_scan<uint32_t>(c, part, t, kT);
        if constexpr (!WRITE) {
            if (t == kT - 1) deg[r] = incl;
        } else {
            int32_t* out = col + row_ptr[r] + (incl - c);
            for (int k = 0; k < kPer; ++k) {
                const int i = t * kPer + k;
                if (i < p2 && s[i] != kFill && (i == 0 || s[i] != s[i - 1])) *out++ = s[i];
            }
        }
        __syncthreads();
    }
}

constexpr int kLongGrid = 256;

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Length of the fixed incidence lists, 0 where n of them would not be
// addressable with 32-bit positions (then only packed lists are built).
uint32_t inc_cap(int dim, int64_t n)
{
    const uint32_t cap = dim == 2 ? kIncCap2 : kIncCap3;
    return (uint64_t)n * cap <= 0xffffffffull ? cap : 0u;
}

// Workspace of ring1_build, carved in this order (carve_ring1): incidence
// counts and offsets (n + 1), cursors (n), incidence lists (the larger of
// K n_cells packed and n fixed lists), distinct counts (n + 1), long rows
// (n), stored lists (kRowCap n), scan partial sums, then the error flags,
// the long-row count and the fixed list length in use (0: packed lists).
struct Ring1Work {
    uint32_t *cnt, *cur, *deg, *longs, *n_long, *cap;
    int32_t *inc, *store;
    void* partial;
    int* err;
};

Ring1Work carve_ring1(void* workspace, int dim, int64_t n, int64_t n_cells, size_t* bytes)
{
    const int K = dim + 1;
    const int64_t tiles = (n + 1 + kScanTile - 1) / kScanTile + 1;
    unsigned char* base = static_cast<unsigned char*>(workspace);
    size_t at = 0;
    auto carve = [&](size_t b) {
        void* p = base ? base + at : nullptr;
        at += align256(b);
        return p;
    };
    Ring1Work w;
    w.cnt = static_cast<uint32_t*>(carve(4 * (size_t)(n + 1)));
    w.cur = static_cast<uint32_t*>(carve(4 * (size_t)n));
    w.inc = static_cast<int32_t*>(carve(4 * std::max((size_t)K * n_cells, (size_t)n * inc_cap(dim, n))));
    w.deg = static_cast<uint32_t*>(carve(4 * (size_t)(n + 1)));
    w.longs = static_cast<uint32_t*>(carve(4 * (size_t)n));
    w.store = static_cast<int32_t*>(carve(4 * (size_t)kRowCap * n));
    w.partial = carve(8 * (size_t)tiles);
    w.err = static_cast<int*>(carve(256));
    w.n_long = w.err ? reinterpret_cast<uint32_t*>(w.err + 1) : nullptr;
    w.cap = w.err ? reinterpret_cast<uint32_t*>(w.err + 2) : nullptr;
    if (bytes) *bytes = at;
    return w;
}

}  // namespace

size_t ring1_workspace_bytes(int dim, int64_t n, int64_t n_cells)
{
    size_t bytes = 0;
    (void)carve_ring1(nullptr, dim, n, n_cells, &bytes);
    return bytes;
}


hipError_t ring1_build(int dim, const int32_t* cells, int64_t n_cells, int64_t n, void* workspace, int64_t* row_ptr,
                       int32_t* col, int64_t col_capacity, int64_t* nnz, int* bad_mesh, int* too_long,
                       hipStream_t stream)
{
    const Ring1Work w = carve_ring1(workspace, dim, n, n_cells, nullptr);
    uint32_t* cnt = w.cnt;
    uint32_t* cur = w.cur;
    int32_t* inc = w.inc;
    uint32_t* deg = w.deg;
    uint32_t* longs = w.longs;
    void* partial = w.partial;
    int* err = w.err;
    uint32_t* n_long = w.n_long;
    hipError_t e;
#define FTLE_CHECK(x)                          \
    if ((e = (x)) != hipSuccess) return e;
    FTLE_CHECK(hipMemsetAsync(cnt, 0, 4 * (size_t)(n + 1), stream));
    FTLE_CHECK(hipMemsetAsync(err, 0, 12, stream));   // flags, long rows, fixed list length
    const dim3 ag(blocks_for(n_cells, kAggThreads * kAggCells)), ab(kAggThreads);
    // 1. fixed lists (with the counts), or the counts alone
    const uint32_t cap = n_cells > 0 ? inc_cap(dim, n) : 0u;
    if (n_cells > 0) {
        if (cap) {
            if (dim == 2)
                hipLaunchKernelGGL((incidence_pass<3, kFixed>), ag, ab, 0, stream, cells, n_cells, n, cnt, inc, err, cap);
            else
                hipLaunchKernelGGL((incidence_pass<4, kFixed>), ag, ab, 0, stream, cells, n_cells, n, cnt, inc, err, cap);
        } else {
            if (dim == 2)
                hipLaunchKernelGGL((incidence_pass<3, kCount>), ag, ab, 0, stream, cells, n_cells, n, cnt, nullptr, err, 0u);
            else
                hipLaunchKernelGGL((incidence_pass<4, kCount>), ag, ab, 0, stream, cells, n_cells, n, cnt, nullptr, err, 0u);
        }
        FTLE_CHECK(hipGetLastError());
    }
    int flags = 0;
    FTLE_CHECK(hipMemcpyAsync(&flags, err, sizeof(int), hipMemcpyDeviceToHost, stream));
    FTLE_CHECK(hipStreamSynchronize(stream));
    if (flags & 1) {
        *bad_mesh = 1;
        return hipSuccess;
    }
    if (cap && !(flags & 4)) {
        // every list fits: the rows read them in place
        FTLE_CHECK(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(w.cap), (int)cap, 1, stream));
    } else if (n_cells > 0) {
        // packed lists: 2. offsets from the counts (cnt becomes off, in place:
        // the tile scan reads a value before writing it), 3. the second pass
        FTLE_CHECK(hipMemsetAsync(err, 0, sizeof(int), stream));
        FTLE_CHECK(exclusive_scan<uint32_t>(cnt, n, cnt, static_cast<uint32_t*>(partial), stream));
        FTLE_CHECK(hipMemcpyAsync(cur, cnt, 4 * (size_t)n, hipMemcpyDeviceToDevice, stream));
        if (dim == 2)
            hipLaunchKernelGGL((incidence_pass<3, kPacked>), ag, ab, 0, stream, cells, n_cells, n, cur, inc, nullptr, 0u);
        else
            hipLaunchKernelGGL((incidence_pass<4, kPacked>), ag, ab, 0, stream, cells, n_cells, n, cur, inc, nullptr, 0u);
        FTLE_CHECK(hipGetLastError());
    }
    // 4. distinct counts, their offsets, then the lists
    const dim3 rg(blocks_for(n, kRowThreads)), rb(kRowThreads);
    if (dim == 2) {
        hipLaunchKernelGGL((ring_rows<3>), rg, rb, 0, stream, cells, inc, cnt, w.cap, n, deg, w.store, longs, n_long);
        hipLaunchKernelGGL((long_rows<3, false>), dim3(kLongGrid), dim3(256), 0, stream, cells, inc, cnt, w.cap, longs,
                           n_long, deg, nullptr, nullptr, err);
    } else {
        hipLaunchKernelGGL((ring_rows<4>), rg, rb, 0, stream, cells, inc, cnt, w.cap, n, deg, w.store, longs, n_long);
        hipLaunchKernelGGL((long_rows<4, false>), dim3(kLongGrid), dim3(256), 0, stream, cells, inc, cnt, w.cap, longs,
                           n_long, deg, nullptr, nullptr, err);
    }
    FTLE_CHECK(hipGetLastError());
    FTLE_CHECK(exclusive_scan<int64_t>(deg, n, row_ptr, static_cast<int64_t*>(partial), stream));
    int64_t total = 0;
    FTLE_CHECK(hipMemcpyAsync(&total, row_ptr + n, sizeof(int64_t), hipMemcpyDeviceToHost, stream));
    FTLE_CHECK(hipMemcpyAsync(&flags, err, sizeof(int), hipMemcpyDeviceToHost, stream));
    FTLE_CHECK(hipStreamSynchronize(stream));
    *nnz = total;
    if (flags & 2) {
        *too_long = 1;
        return hipSuccess;
    }
    if (!col || total > col_capacity || total == 0) return hipSuccess;
    return ring1_write(dim, cells, n_cells, n, workspace, row_ptr, col, stream);
#undef FTLE_CHECK
}

hipError_t ring1_write(int dim, const int32_t* cells, int64_t n_cells, int64_t n, void* workspace,
                       const int64_t* row_ptr, int32_t* col, hipStream_t stream)
{
    const Ring1Work w = carve_ring1(workspace, dim, n, n_cells, nullptr);
    hipLaunchKernelGGL(copy_rows, dim3(blocks_for(n)), dim3(256), 0, stream, w.store, n, w.deg, row_ptr, col);
    if (dim == 2)
        hipLaunchKernelGGL((long_rows<3, true>), dim3(kLongGrid), dim3(256), 0, stream, cells, w.inc, w.cnt, w.cap, w.longs,
                           w.n_long, w.deg, row_ptr, col, w.err);
    else
        hipLaunchKernelGGL((long_rows<4, true>), dim3(kLongGrid), dim3(256), 0, stream, cells, w.inc, w.cnt, w.cap, w.longs,
                           w.n_long, w.deg, row_ptr, col, w.err);
    return hipGetLastError();
}

hipError_t scan_exclusive_u32(const uint32_t* in, int64_t m, uint32_t* out, uint32_t* partial, hipStream_t stream)
{
    return exclusive_scan<uint32_t>(in, m, out, partial, stream);
}

hipError_t scan_exclusive_to_i64(const uint32_t* in, int64_t m, int64_t* out, int64_t* partial, hipStream_t stream)
{
    return exclusive_scan<int64_t>(in, m, out, partial, stream);
}

size_t scan_partial_bytes(int64_t m) { return 8 * (size_t)((m + kScanTile - 1) / kScanTile + 1); }

}  // namespace ftle
