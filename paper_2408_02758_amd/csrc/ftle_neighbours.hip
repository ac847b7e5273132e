// The one-ring stencil of a cell mesh built on the GPU: the neighbour
// determination that precedes the FTLE path (Section 2.2 keeps it on the host,
// off the accelerator; the Conclusions list accelerating it as future work).
// Every point's neighbours are the other points sharing a cell with it,
// ascending, each once.
//
//   1. edge extraction: each cell of K = dim + 1 points emits its K (K - 1)
//      directed pairs (i, j) as 64-bit keys i * 2^b + j, with b the bit
//      length of n; a pair with i = j (a point repeated inside a cell)
//      becomes a sentinel key n * 2^b that sorts after every real key, and an
//      index outside [0, n) raises the error flag and becomes the sentinel too;
//   2. a radix sort of the keys over their 2 b bits (hipCUB);
//   3. deduplication: a flag per sorted key that is the first of its run of
//      equal keys and not the sentinel, and the exclusive sum of the flags
//      (hipCUB), which is each kept key's CSR position;
//   4. the CSR arrays: a kept key's column is its low b bits, and row r
//      starts at the first kept key whose row is >= r.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cstdint>

#include "ftle_internal.h"

namespace ftle {
namespace {

template <int K>
__global__ void __launch_bounds__(256) emit_edges(const int32_t* __restrict__ cells, int64_t n_cells, int64_t n,
                                                  int b, uint64_t* __restrict__ keys, int* __restrict__ err)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    int32_t v[K];
#pragma unroll
    for (int a = 0; a < K; ++a) v[a] = cells[c * K + a];
    bool bad = false;
#pragma unroll
    for (int a = 0; a < K; ++a) bad |= (v[a] < 0) || ((int64_t)v[a] >= n);
    if (bad) *err = 1;   // every writer stores the same value
    const uint64_t sentinel = (uint64_t)n << b;
    // pair o of every cell in one contiguous stretch: each store instruction
    // writes consecutive keys for consecutive cells (the sort ignores order)
    uint64_t* out = keys + c;
    int o = 0;
#pragma unroll
    for (int a = 0; a < K; ++a)
#pragma unroll
        for (int c2 = 0; c2 < K; ++c2) {
            if (a == c2) continue;
            const bool real = !bad && v[a] != v[c2];
            out[(int64_t)(o++) * n_cells] = real ? ((uint64_t)(uint32_t)v[a] << b) | (uint32_t)v[c2] : sentinel;
        }
}

// flag[p] = 1 where sorted key p is the first of its run and below the sentinel.
__global__ void __launch_bounds__(256) mark_first(const uint64_t* __restrict__ keys, int64_t m, uint64_t sentinel,
                                                  uint32_t* __restrict__ flag)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m) return;
    const uint64_t k = keys[p];
    flag[p] = (k < sentinel && (p == 0 || keys[p - 1] != k)) ? 1u : 0u;
}

// Kept key p (flag set) goes to CSR position pos[p]: its column, and the
// starts of the rows from the previous key's row + 1 up to its own (the
// previous key, kept or not, has the previous kept key's row); the last kept
// key also closes the rows after its own up to n.
__global__ void __launch_bounds__(256) csr_from_keys(const uint64_t* __restrict__ keys, const uint32_t* __restrict__ flag,
                                                     const uint32_t* __restrict__ pos, int64_t m, int64_t nnz,
                                                     int64_t n, int b, int64_t* __restrict__ row_ptr,
                                                     int32_t* __restrict__ col)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= m || !flag[p]) return;
    const uint64_t k = keys[p];
    const int64_t q = pos[p];
    const int64_t r = (int64_t)(k >> b);
    const int64_t rp = p == 0 ? -1 : (int64_t)(keys[p - 1] >> b);
    col[q] = (int32_t)(k & ((1ull << b) - 1));
    for (int64_t t = rp + 1; t <= r; ++t) row_ptr[t] = q;
    if (q == nnz - 1)
        for (int64_t t = r + 1; t <= n; ++t) row_ptr[t] = nnz;
}

__global__ void __launch_bounds__(256) fill_zero(int64_t* __restrict__ a, int64_t m)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) a[i] = 0;
}

inline unsigned blocks_for(int64_t m) { return (unsigned)((m + 255) / 256); }

}  // namespace

int ring1_key_bits(int64_t n)
{
    int b = 0;
    for (uint64_t v = (uint64_t)n; v; v >>= 1) ++b;
    return b;
}

hipError_t ring1_device_scratch_bytes(int64_t n_edges, size_t* bytes)
{
    size_t sort_bytes = 0, scan_bytes = 0;
    hipError_t e = hipcub::DeviceRadixSort::SortKeys(nullptr, sort_bytes, (const uint64_t*)nullptr,
                                                     (uint64_t*)nullptr, (int64_t)n_edges, 0, 64, (hipStream_t)0);
    if (e != hipSuccess) return e;
    e = hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                         (int64_t)n_edges, (hipStream_t)0);
    *bytes = sort_bytes > scan_bytes ? sort_bytes : scan_bytes;
    return e;
}

hipError_t launch_emit_edges(int dim, const int32_t* cells, int64_t n_cells, int64_t n, uint64_t* keys, int* err,
                             hipStream_t stream)
{
    if (n_cells == 0) return hipSuccess;
    if (dim == 2)
        hipLaunchKernelGGL(emit_edges<3>, dim3(blocks_for(n_cells)), dim3(256), 0, stream, cells, n_cells, n,
                           ring1_key_bits(n), keys, err);
    else
        hipLaunchKernelGGL(emit_edges<4>, dim3(blocks_for(n_cells)), dim3(256), 0, stream, cells, n_cells, n,
                           ring1_key_bits(n), keys, err);
    return hipGetLastError();
}

hipError_t sort_and_mark_keys(uint64_t* keys, uint64_t* sorted, int64_t n_edges, int64_t n, void* scratch,
                              size_t scratch_bytes, uint32_t* flag, uint32_t* pos, hipStream_t stream)
{
    // keys i * 2^b + j with i <= n (the sentinel's row) and j < n use 2 b bits
    const int b = ring1_key_bits(n);
    size_t bytes = scratch_bytes;
    hipError_t e = hipcub::DeviceRadixSort::SortKeys(scratch, bytes, keys, sorted, n_edges, 0, 2 * b, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mark_first, dim3(blocks_for(n_edges)), dim3(256), 0, stream, sorted, n_edges,
                       (uint64_t)n << b, flag);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    bytes = scratch_bytes;
    return hipcub::DeviceScan::ExclusiveSum(scratch, bytes, flag, pos, n_edges, stream);
}

hipError_t launch_csr_from_keys(const uint64_t* sorted, const uint32_t* flag, const uint32_t* pos, int64_t n_edges,
                                int64_t nnz, int64_t n, int64_t* row_ptr, int32_t* col, hipStream_t stream)
{
    if (nnz == 0) {
        hipLaunchKernelGGL(fill_zero, dim3(blocks_for(n + 1)), dim3(256), 0, stream, row_ptr, n + 1);
    } else {
        hipLaunchKernelGGL(csr_from_keys, dim3(blocks_for(n_edges)), dim3(256), 0, stream, sorted, flag, pos, n_edges,
                           nnz, n, ring1_key_bits(n), row_ptr, col);
    }
    return hipGetLastError();
}

}  // namespace ftle
