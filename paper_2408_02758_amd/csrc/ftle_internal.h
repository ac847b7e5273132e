// Internal declarations shared by the host side (ftle_host.cpp) and the HIP
// kernels (ftle_*.hip) of the FTLE library.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ftle {

// ---------------------------------------------------------------------------
// Tile records (device layout).
//
// The mesh's points are cut, in Morton order, into tiles of at most
// tile_points points; one workgroup processes one tile.  The tile stages
// S = P + H points: its own P points (a Morton range), then its H halo points
// (neighbours owned by other tiles), each part in increasing caller (user)
// index; slot l is the position of a staged point in that order, and the
// stencil refers to staged points by slot ("local index").  A tile's record
// is a contiguous, 16-byte aligned block, copied whole into LDS:
//
//   uint32 words[nw]   stencil rows of the explicit rows (below): three
//                      10-bit local indices per word, in bits 0-9, 10-19 and
//                      20-29; a row's entries ascend and are padded to a
//                      multiple of 3 with the row's own slot; bits 30-31 of
//                      a row's last word hold its padding count (0-2)
//   uint32 runs[nr]    run r (a maximal stretch of slots with consecutive
//                      caller indices): caller index of its first slot minus
//                      that slot, so that slot l of run r is point runs[r] + l
//   uint32 smask[G]    bit i of smask[g]: slot 32 g + i starts a run
//   uint32 xmask[Q]    bit i of xmask[q]: row 32 q + i is explicit
//   uint16 spre[G]     runs that start before slot 32 g
//   uint16 xpre[Q]     explicit rows before row 32 q
//   uint16 xlast[Q]    the last explicit row before row 32 q
//   uint16 xend[nx]    end of explicit row k in words (cumulative)
//   (zero padding to a multiple of 16 bytes)
//
// with G = ceil(S / 32) and Q = ceil(P / 32).  Row l (the stencil of own slot
// l) is explicit unless l > 0 and it equals row l - 1 with every entry plus
// one; a row that is not explicit therefore equals its anchor, the last
// explicit row a <= l, with every entry plus l - a.  On a mesh whose points
// are numbered along grid lines most rows are such shifts, and the runs are
// the grid lines crossing the tile; on any other mesh the record degrades to
// one explicit row per point and one run per slot.
//
// 10-bit indices and 16-bit row ends are enough because P + H <= kMaxStaged
// and the explicit words stay <= kMaxTileWords, both enforced when the mesh
// is built.
// ---------------------------------------------------------------------------
struct TileMeta {
    uint32_t rec_off;  // record offset in 16-byte units
    uint16_t P;        // own points
    uint16_t H;        // halo points
    uint16_t nw;       // stencil words of the explicit rows
    uint16_t nr;       // runs
    uint16_t nx;       // explicit rows
    uint16_t nwf;      // stencil words of all rows (the tile's work; host only)
};
static_assert(sizeof(TileMeta) == 16, "TileMeta is one 16-byte load");

constexpr int kMaxStaged = 1024;       // staged points per tile: 10-bit local indices
constexpr int kMaxTileWords = 65535;   // stencil words per tile: 16-bit row ends
constexpr size_t kLdsBudget = 65536;   // LDS bytes one tile may stage (forward or adjoint)

__host__ __device__ inline int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Byte offsets of the record's arrays (words at 0) and its padded size.
struct RecLayout {
    uint32_t runs, smask, xmask, spre, xpre, xlast, xend, bytes;
};
__host__ __device__ inline RecLayout rec_layout(uint32_t P, uint32_t H, uint32_t nw, uint32_t nr, uint32_t nx)
{
    const uint32_t G = (P + H + 31u) / 32u, Q = (P + 31u) / 32u;
    RecLayout r;
    r.runs = 4u * nw;
    r.smask = r.runs + 4u * nr;
    r.xmask = r.smask + 4u * G;
    r.spre = r.xmask + 4u * Q;
    r.xpre = r.spre + 2u * G;
    r.xlast = r.xpre + 2u * Q;
    r.xend = r.xlast + 2u * Q;
    r.bytes = (r.xend + 2u * nx + 15u) & ~15u;
    return r;
}
__host__ __device__ inline RecLayout rec_layout(const TileMeta& m)
{
    return rec_layout(m.P, m.H, m.nw, m.nr, m.nx);
}

// LDS of a tile's staged points, with e the value size (4 or 8 bytes) and S
// the staged points:
//   forward  2D: one array of round_up(S, 4) slots (x0, x1, phi0, phi1), 4e
//            3D: three arrays of kMaxStaged slots of 2e: (x0, x1), (x2, phi0),
//                (phi1, phi2); the fixed array stride lets one per-neighbour
//                address reach all three through the instruction's offset
//   adjoint  2D: one array of round_up(S, 4) slots (x0, x1, w0, w1)
//                (h0, h1, -, -), 8e
//            3D: three arrays of bwd3_capacity slots: (x0, x1, x2, h0) and
//                (h1, h2, w0, w1) (4e each, the second at a fixed offset
//                from the first), then w2 (e)
// so that every array and the record copy after them start 16-byte aligned.
__host__ __device__ inline size_t elem_bytes(bool f64) { return f64 ? 8 : 4; }
__host__ __device__ inline size_t fwd_points_bytes(int dim, bool f64, int staged)
{
    return dim == 2 ? (size_t)round_up(staged, 4) * 4 * elem_bytes(f64) : (size_t)kMaxStaged * 6 * elem_bytes(f64);
}
// Staged points a 3D adjoint tile holds (its arrays have that many slots;
// float64 tiles are cut smaller to stay in the LDS budget).
__host__ __device__ constexpr int bwd3_capacity(bool f64) { return f64 ? 512 : kMaxStaged; }
__host__ __device__ inline size_t bwd_points_bytes(int dim, bool f64, int staged)
{
    return dim == 2 ? (size_t)round_up(staged, 4) * 8 * elem_bytes(f64)
                    : (size_t)bwd3_capacity(f64) * 9 * elem_bytes(f64);
}

// One tile set: the tiles of one stencil (the forward stencil, or its
// transpose for the adjoint when the stencil is not symmetric).
struct DevTiles {
    const TileMeta* meta;
    const uint4* rec;
    const void* minv;   // 3D forward tiles: per point (caller order) the six values of M^-1, else null
    int n_tiles;
    int max_staged;   // max over tiles of P + H
    int max_rec;      // max over tiles of the record bytes
};

// One work item of a batched launch: a tile of one mesh, with everything the
// workgroup needs to start on it (one 48-byte scalar load).
struct BatchItem {
    TileMeta meta;                  // rec_off relative to rec
    const uint4* rec;               // the mesh's tile records
    const void* x;                  // the mesh's coordinates
    unsigned long long* fp64_hits;  // the mesh's FP64-branch counter
    uint32_t mesh;                  // index into the call's flow/out/time arrays
    uint32_t pad;
};
static_assert(sizeof(BatchItem) == 48, "BatchItem is 48 bytes");

// Per-call parameters of a batched launch (kernel argument by value).
constexpr int kMaxBatch = 64;
struct BatchCall {
    const void* flow[kMaxBatch];
    void* out[kMaxBatch];
    double inv2T[kMaxBatch];
};

// The batched kernel keeps its queue word in the first bytes of its dynamic
// LDS and the tile's staged data after them.
constexpr uint32_t kBatchedLdsHead = 16;

// Launch helpers implemented in ftle_kernels.hip.  All return hipSuccess or
// the launch error.  lds_bytes() gives the dynamic LDS a launch needs.
size_t fwd_lds_bytes(int dim, bool f64, const DevTiles& t);
size_t bwd_lds_bytes(int dim, bool f64, const DevTiles& t);

// tape_sigma: the tape carries sigma (needed when the stencil is not
// symmetric; with a symmetric stencil the adjoint forms it itself).
hipError_t launch_forward(int dim, bool f64, const DevTiles& tiles, const void* x, const void* flow,
                          double inv2T, void* out, void* tape, bool tape_sigma, int64_t n, double eig_tau,
                          unsigned long long* hits, int block, hipStream_t stream);

// Half-precision flow-map storage (2D, float32 meshes): the forward from
// binary16 displacements d = phi - x, and the encoding of a float32 flow map.
hipError_t launch_forward_f16(const DevTiles& tiles, const void* x, const void* delta, double inv2T, void* out,
                              int64_t n, double eig_tau, unsigned long long* hits, int block, hipStream_t stream);
hipError_t launch_encode_f16(const void* x, const void* flow, void* delta, int64_t n, hipStream_t stream);

hipError_t launch_backward_gather(int dim, bool f64, const DevTiles& tiles, const void* x,
                                  const void* tape, bool tape_sigma, int64_t n, const void* g, void* grad,
                                  int block, hipStream_t stream);

// Block sizes (threads per workgroup) the kernels are compiled for.
inline bool supported_block(int b) { return b == 128 || b == 256 || b == 512; }

// Flow maps by RK4 advection (ftle_advect.hip): kind 0 double gyre, 1 ABC;
// per-point t0s / Ts when not null, else t0 / T for every particle.  At most
// kMaxAdvectSteps steps per particle.
constexpr int64_t kMaxAdvectSteps = 10000000;
// A velocity field sampled on a regular grid: shape[d] nodes at origin[d] +
// i spacing[d] per axis (x fastest), nt slices at t_first + k t_step.
struct GridField {
    int64_t shape[3];
    double origin[3];
    double spacing[3];
    int64_t nt;
    double t_first, t_step;
};
hipError_t launch_advect_grid(int dim, const GridField& g, const void* vel, bool vel_f64, bool f64, int64_t n,
                              const void* x0, const double* t0s, const double* Ts, double t0, double T, double dt,
                              void* phi, hipStream_t stream);
hipError_t launch_advect(int kind, const double* params, bool f64, int64_t n, const void* x0, const double* t0s,
                         const double* Ts, double t0, double T, double dt, void* phi, hipStream_t stream);

// One-ring stencil on the device (ftle_neighbours.hip): incidence lists (in
// one pass at fixed places, or packed after a count and its scan), then each
// point's distinct neighbours counted, scanned into row_ptr and written to
// col.  The workspace
// (ring1_workspace_bytes) is device memory the call may overwrite.  On return
// *bad_mesh (a cell index outside [0, n): nothing written) or *too_long (a
// point whose incident cells list more than 4096 points) may be set;
// otherwise *nnz holds the entry count, and row_ptr / col are written when it
// is at most col_capacity.  Synchronises the stream.
// col = NULL: count only (row_ptr written, nothing else); ring1_write then
// writes col from the same workspace.
size_t ring1_workspace_bytes(int dim, int64_t n, int64_t n_cells);
hipError_t ring1_build(int dim, const int32_t* cells, int64_t n_cells, int64_t n, void* workspace, int64_t* row_ptr,
                       int32_t* col, int64_t col_capacity, int64_t* nnz, int* bad_mesh, int* too_long,
                       hipStream_t stream);
hipError_t ring1_write(int dim, const int32_t* cells, int64_t n_cells, int64_t n, void* workspace,
                       const int64_t* row_ptr, int32_t* col, hipStream_t stream);
// Exclusive scan of m uint32 values into out[0..m), out[m] = their sum
// (in and out may coincide); partial: scan_partial_bytes(m) of device scratch.
hipError_t scan_exclusive_u32(const uint32_t* in, int64_t m, uint32_t* out, uint32_t* partial, hipStream_t stream);
size_t scan_partial_bytes(int64_t m);

// Morton quantisation of the points (both mesh builders): axis d of a point
// maps to q = clamp(floor(((x_d - lo_d) / unit_d + 0.2) * scale), 0, qmax),
// shifted up shift_bits when d is not the caller-order axis `fast` (>= 0),
// and the axes' bits are interleaved (axis d at bit positions d, d + dim, ...).
struct MortonParams {
    double lo[3];
    double unit[3];
    double scale;   // 2^sub, sub fractional bits per unit
    double qmax;
    int fast;       // caller-order axis, or -1
    int shift_bits;
};

// The mesh build on the device (ftle_meshbuild.hip).  Each launcher returns
// hipSuccess or the launch error; none synchronises.
//   mb_bbox: per-workgroup minima and maxima (part[b * 2 dim + d], then the
//     maxima at + dim) over nblocks workgroups; *first_bad (set to ~0 before)
//     gets the lowest point with a coordinate that is not finite
//   mb_gather_pairs: sample k = points k stride and k stride + 1, as float64
//   mb_morton: codes key[i] and values val[i] = i
//   mb_sort: stable sort of (key, val) by the low key_bits bits of key;
//     *sorted_val is val or a buffer inside scratch (mb_sort_scratch_bytes)
//   mb_invert: inv[perm[r]] = r
//   mb_relabel: cells renumbered to Morton positions; a cell with an index
//     outside [0, n) or a repeated point sets *flag and lowers *first
//   mb_tile_extent: for ranges [b, e) (int64 pairs) of the Morton order, the
//     halo size (kMaxStaged + 1 when larger) and the padded stencil words
//   mb_tile_record: write = false sizes each tile's record (counts[4 t] =
//     explicit words, runs, explicit rows, all words) and fills the row
//     buffer; write = true writes the records at 16 meta[t].rec_off bytes
//   mb_normal_inverse: the 3D inverse normal matrices (caller order)
hipError_t mb_bbox(int dim, bool f64, const void* x, int64_t n, double* part, int nblocks,
                   unsigned long long* first_bad, hipStream_t s);
hipError_t mb_gather_pairs(int dim, bool f64, const void* x, int64_t m, int64_t stride, double* out, hipStream_t s);
hipError_t mb_morton(int dim, bool f64, const void* x, int64_t n, const MortonParams& mp, uint64_t* key,
                     uint32_t* val, hipStream_t s);
size_t mb_sort_scratch_bytes(int64_t n);
hipError_t mb_sort(uint64_t* key, uint32_t* val, int64_t n, int key_bits, void* scratch, uint32_t** sorted_val,
                   hipStream_t s);
hipError_t mb_iota(uint32_t* v, int64_t n, hipStream_t s);
hipError_t mb_invert(const uint32_t* perm, int64_t n, int32_t* inv, hipStream_t s);
hipError_t mb_relabel(int dim, const int32_t* cells, int64_t n_cells, int64_t n, const int32_t* inv, int32_t* mc,
                      int* flag, unsigned long long* first, hipStream_t s);
hipError_t mb_tile_extent(const int64_t* row_ptr, const int32_t* col, const int64_t* ranges, int64_t n_ranges,
                          uint32_t* halo_words, hipStream_t s);
hipError_t mb_tile_record(bool write, const int64_t* row_ptr, const int32_t* col, const uint32_t* perm,
                          const int64_t* ranges, int64_t n_tiles, const int64_t* row_base, uint16_t* rowbuf,
                          uint32_t* counts, const TileMeta* meta, unsigned char* rec, hipStream_t s);
hipError_t mb_normal_inverse(bool f64, const int64_t* row_ptr, const int32_t* col, const uint32_t* perm,
                             const void* x, int64_t n, void* out, hipStream_t s);
//   mb_axis_stencil: the axis stencil's slots (n x 2 dim, -1 absent) and
//     counts per Morton row from the one-ring CSR; mb_axis_fill: its CSR
//   mb_transpose_count / mb_transpose_fill: column counts (tcnt zeroed
//     before), then, with trp their exclusive scan and cur zeroed, the
//     transposed rows, each sorted ascending
//   mb_csr_compare: *differ = 1 (set to 0 before) where two CSRs differ
hipError_t mb_axis_stencil(int dim, bool f64, const void* x, const uint32_t* perm, const int64_t* ring_rp,
                           const int32_t* ring_col, int64_t n, int32_t* slots, uint32_t* cnt, hipStream_t s);
hipError_t mb_axis_fill(int dim, const int32_t* slots, const int64_t* row_ptr, int64_t n, int32_t* col,
                        hipStream_t s);
hipError_t mb_transpose_count(const int32_t* col, int64_t nnz, uint32_t* tcnt, hipStream_t s);
hipError_t mb_transpose_fill(const int64_t* row_ptr, const int32_t* col, int64_t n, const int64_t* trp,
                             uint32_t* cur, int32_t* tcol, hipStream_t s);
hipError_t mb_csr_compare(const int64_t* rp_a, const int32_t* col_a, const int64_t* rp_b, const int32_t* col_b,
                          int64_t n, int64_t nnz, int* differ, hipStream_t s);
//   mb_csr_in_count / mb_csr_in_fill: a caller's CSR over caller indices
//     (nnz_in = row_ptr[n] entries) moved to Morton positions: per Morton row
//     the count of entries that are neither -1 nor the point itself (err[0]
//     and err[1], set to ~0 before, lower to a faulty row + 1, 0 for
//     row_ptr[0] != 0, and to a faulty entry), then the rows, renumbered by
//     inv and sorted ascending
hipError_t mb_csr_in_count(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz_in, const uint32_t* perm,
                           uint32_t* cnt, unsigned long long* err, hipStream_t s);
hipError_t mb_csr_in_fill(const int64_t* row_ptr, const int32_t* col, int64_t n, const uint32_t* perm,
                          const int32_t* inv, const int64_t* out_rp, int32_t* out, hipStream_t s);
// Exclusive scan of m uint32 values into int64 out[0..m), out[m] = their sum;
// partial: scan_partial_bytes(m) of device scratch.
hipError_t scan_exclusive_to_i64(const uint32_t* in, int64_t m, int64_t* out, int64_t* partial, hipStream_t stream);

// The paper's fixed-width axis list (ftle_ell.hip): the forward from it (one
// lane per caller point; staged: each workgroup's block of points in LDS),
// and its construction from a one-ring CSR.
hipError_t launch_forward_ell(int dim, bool f64, bool staged, const void* x, const void* flow, const int32_t* ell,
                              int64_t n, double inv2T, void* out, double eig_tau, unsigned long long* hits,
                              hipStream_t stream);
hipError_t launch_axis_ell(int dim, bool f64, const void* x, const int64_t* row_ptr, const int32_t* col, int64_t n,
                           int32_t* ell, hipStream_t stream);

// The allocation-free adjoint (ftle_noalloc.hip): its tape lives in a fixed
// device array of kNoAllocScratchBytes per GPU; noalloc_scratch gives that
// array's address on `device`, which must be current.
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
hipError_t noalloc_scratch(int device, void** ptr);

hipError_t launch_batched(int dim, bool f64, bool wide, const BatchItem* items, int n_items, int tiles_per_pop,
                          unsigned* queue, const BatchCall& call, size_t lds, double eig_tau, int block, int grid,
                          hipStream_t stream);

// The kernel a batched launch runs (for occupancy queries and graph nodes);
// nullptr for an unsupported block size.  wide: 64-bit element offsets, needed
// when some mesh of the batch has batched_needs_wide(dim, f64, n).
const void* batched_kernel_symbol(int dim, bool f64, int block, bool wide);
bool batched_needs_wide(int dim, bool f64, int64_t max_points);
// Testing aid: make every launch take the 64-bit offset path.
void set_force_wide(bool on);
void batched_kernel_args(const BatchItem* items, int n_items, int tiles_per_pop, unsigned* queue,
                         const BatchCall& call, double eig_tau, void* storage, void** args);
size_t batched_kernel_arg_storage();

}  // namespace ftle
