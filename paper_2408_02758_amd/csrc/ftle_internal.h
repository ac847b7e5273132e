// Internal declarations shared by the host side (ftle_host.cpp) and the HIP
// kernels (ftle_kernels.hip) of the FTLE library.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ftle {

// ---------------------------------------------------------------------------
// Tile records (device layout).
//
// The mesh's points are cut, in Morton order, into tiles of at most
// tile_points points; one workgroup processes one tile.  A tile's record is
// a contiguous, 16-byte aligned block:
//
//   uint32 idx[P + H]         caller (user) index of every staged point: the
//                             tile's own P points (a Morton range), then its H
//                             halo points (neighbours owned by other tiles),
//                             each part in increasing caller index, padded to
//                             a multiple of 4 entries
//   uint32 words[nw]          the stencil rows of the own points, three
//                             10-bit local indices (positions in idx) per
//                             word, in bits 0-9, 10-19 and 20-29; every row
//                             is padded to a multiple of 3 entries with the
//                             point's own index
//   uint16 rowend[P]          end of each row (cumulative, in words)
//                             (words and rowend: the "segment", padded to a
//                             multiple of 16 bytes)
//
// 10-bit indices and 16-bit row ends are enough because P + H <= kMaxStaged
// and nw <= kMaxTileWords, both enforced when the mesh is built.
// ---------------------------------------------------------------------------
struct TileMeta {
    uint32_t rec_off;  // record offset in 16-byte units
    uint32_t P;        // own points
    uint32_t H;        // halo points
    uint32_t nw;       // stencil words of the own points (3 entries each, rows padded)
};
static_assert(sizeof(TileMeta) == 16, "TileMeta is one 16-byte load");

constexpr int kMaxStaged = 1024;       // staged points per tile: 10-bit local indices
constexpr int kMaxTileWords = 65535;   // stencil words per tile: 16-bit row ends
constexpr size_t kLdsBudget = 65536;   // LDS bytes one tile may stage (forward or adjoint)

__host__ __device__ inline int round_up(int v, int m) { return (v + m - 1) / m * m; }
__host__ __device__ inline uint32_t idx_words(uint32_t P, uint32_t H) { return (P + H + 3u) & ~3u; }
// segment size in 16-bit units (a multiple of 8, i.e. of 16 bytes)
__host__ __device__ inline uint32_t seg_halfs(uint32_t P, uint32_t nw) { return (2u * nw + P + 7u) & ~7u; }

// LDS bytes per staged point, in units of the value size e (4 or 8 bytes):
//   forward  2D: 4e, one slot (x0, x1, phi0, phi1)
//            3D: 6e, two arrays: (phi1, phi2) slots of 2e at the start of
//                LDS, then (x0, x1, x2, phi0) slots of 4e
//   adjoint  2D: 8e, one slot (x0, x1, w0, w1) (h0, h1, -, -)
//            3D: 9e, three arrays: w2 slots of e, then (x0, x1, x2, h0)
//                slots of 4e, then (h1, h2, w0, w1) slots of 4e
// Each array holds round_up(P + H, 4) slots, so every array and the segment
// after them start 16-byte aligned.
__host__ __device__ inline size_t elem_bytes(bool f64) { return f64 ? 8 : 4; }
__host__ __device__ inline size_t fwd_slot_bytes(int dim, bool f64) { return elem_bytes(f64) * (dim == 2 ? 4 : 6); }
__host__ __device__ inline size_t bwd_slot_bytes(int dim, bool f64) { return elem_bytes(f64) * (dim == 2 ? 8 : 9); }
__host__ __device__ inline size_t tile_lds_bytes(size_t slot_bytes, int staged, int seg)
{
    return (size_t)round_up(staged, 4) * slot_bytes + (size_t)seg * 2;
}

// One tile set: the tiles of one stencil (the forward stencil, or its
// transpose for the adjoint when the stencil is not symmetric).
struct DevTiles {
    const TileMeta* meta;
    const uint4* rec;
    int n_tiles;
    int max_staged;   // max over tiles of P + H
    int max_seg;      // max over tiles of seg_halfs(P, nw)
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

hipError_t launch_backward_gather(int dim, bool f64, const DevTiles& tiles, const void* x,
                                  const void* tape, bool tape_sigma, int64_t n, const void* g, void* grad,
                                  int block, hipStream_t stream);

// Block sizes (threads per workgroup) the kernels are compiled for.
inline bool supported_block(int b) { return b == 128 || b == 256 || b == 512; }

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
