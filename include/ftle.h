/*
 * ftle.h -- C ABI of the MI355X (gfx950) Finite-Time Lyapunov Exponent library.
 *
 * The library computes, for every point of a 2D triangle mesh or a 3D
 * tetrahedral mesh, the finite-time Lyapunov exponent of a precomputed flow
 * map (the per-point FTLE kernels of UVaFTLE studied in de Castro et al.,
 * "Finite-Time Lyapunov Exponent Calculation on FPGA using High-Level
 * Synthesis Tools", Section 2):
 *
 *   J_i   = flow-map gradient at point i, least squares over i's mesh
 *           neighbours S(i):  J_i = B_i M_i^{-1},
 *           M_i = sum_j (x_j - x_i)(x_j - x_i)^T,
 *           B_i = sum_j (phi_j - phi_i)(x_j - x_i)^T;
 *   C_i   = J_i^T J_i  (Cauchy-Green tensor, 2x2 or 3x3);
 *   FTLE_i = ln( sqrt( lambda_max(C_i) ) ) / |T|.
 *
 * Problem statement as in Section 2.2 of the paper: point coordinates, mesh
 * connectivity, the advected flow map and the integration time go in; one
 * FTLE value per point comes out.  The neighbour list is computed once, when
 * the mesh is created: on the host as Section 2.2 does (neighbours precomputed
 * on the CPU into a list of integer indices; ftle_create_mesh), or on the
 * device as the Conclusions propose (ftle_create_mesh_device); the FTLE
 * kernels only stream it.
 *
 * Conventions for every entry point:
 *  - All functions return an ftle_status; none throws or aborts.  On failure
 *    ftle_last_error() returns a message for the calling thread.
 *  - Argument validation happens on the host before any device work, so
 *    invalid calls fail without touching the GPU.
 *  - "device pointer" arguments are HIP device memory of the current device
 *    (e.g. torch CUDA tensors' data_ptr()); "host pointer" arguments are
 *    ordinary CPU memory.  Point arrays are row-major n x dim in the CALLER's
 *    point order ("user order").
 *  - Device work is enqueued on the given stream (a hipStream_t, NULL means
 *    the null stream) and returns without waiting.  A fault inside a kernel
 *    surfaces as FTLE_ERR_DEVICE from a later call.
 *  - A point whose stencil is rank deficient (fewer than dim neighbours, or
 *    neighbours that do not span the space; this includes points that belong
 *    to no cell) gets NaN.  lambda_max = 0 gives -inf.  NaN or inf in the flow
 *    map propagate to NaN outputs.
 */
#ifndef FTLE_H
#define FTLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ftle_mesh_s* ftle_mesh_t;  /* opaque; immutable after creation */
typedef void* ftle_stream_t;              /* hipStream_t; NULL = null stream  */

typedef enum { FTLE_F32 = 0, FTLE_F64 = 1 } ftle_dtype;

typedef enum {
    FTLE_OK = 0,
    FTLE_ERR_INVALID_ARG = 1,   /* null pointer, bad dim/size, T = 0 or not finite, ... */
    FTLE_ERR_BAD_MESH = 2,      /* cell index outside [0, n) or repeated inside a cell   */
    FTLE_ERR_DTYPE = 3,         /* dtype differs from the mesh's dtype                    */
    FTLE_ERR_UNSUPPORTED = 4,   /* n > 2^31-1, degree too large for one tile, no device   */
    FTLE_ERR_OOM = 5,           /* host or device allocation failed                       */
    FTLE_ERR_DEVICE = 6         /* a HIP runtime call failed                               */
} ftle_status;

/* Flags of ftle_create_mesh (OR them together). */
enum {
    /* Stencil S(i): every vertex sharing a cell with i (default). */
    FTLE_STENCIL_RING1 = 0,
    /* Stencil S(i): the paper's fixed-width list (Section 2.2, exactly 4 slots
     * in 2D and 6 in 3D, -1 for an absent neighbour): for each signed axis
     * direction the RING1 neighbour with the largest cosine to that
     * direction among those on its side; absent slots are skipped. */
    FTLE_STENCIL_AXIS = 1,
    /* Keep the caller's point order instead of the Morton (Z-order) order. */
    FTLE_NO_REORDER = 1 << 4,
    /* Build the host-side structures only (no device upload).  Such a mesh
     * serves ftle_mesh_info / ftle_mesh_get_csr / ftle_mesh_tile_stats;
     * compute calls on it return FTLE_ERR_UNSUPPORTED. */
    FTLE_HOST_ONLY = 1 << 5
};
/* Points per tile (one workgroup's share): FTLE_TILE(k) asks for 2^k points,
 * 5 <= k <= 11; 0 selects the default, 512.  A tile is halved until its own
 * and halo points fit 1024 staged slots and 64 KiB of LDS. */
#define FTLE_TILE(k) ((unsigned)(k) << 8)

/*
 * Build a mesh: validate, build the neighbour stencil from the cells on the
 * host, order the points along a Morton curve, cut the order into tiles and
 * upload everything to the current device.
 *   dim      2 (triangles) or 3 (tetrahedra)
 *   n_points number of points, 1 <= n_points <= 2^31-1
 *   coords   host pointer, n_points x dim, float (FTLE_F32) or double (FTLE_F64);
 *            copied, must be finite
 *   dtype    storage and arithmetic precision of every later call on the mesh
 *   n_cells  number of cells (>= 0)
 *   cells    host pointer, n_cells x (dim+1) int32 point indices; copied
 *   flags    FTLE_STENCIL_*, FTLE_NO_REORDER, FTLE_HOST_ONLY, FTLE_TILE(k)
 *   out      receives the handle; the caller owns it until ftle_destroy_mesh
 * Errors: INVALID_ARG (null pointer, dim, n_points < 1, non-finite coordinate,
 * unknown flag), BAD_MESH (cell index out of range or repeated within a cell),
 * UNSUPPORTED (n_points > 2^31-1, a point whose stencil does not fit one
 * tile), OOM, DEVICE.
 */
ftle_status ftle_create_mesh(int dim, int64_t n_points, const void* coords, ftle_dtype dtype,
                             int64_t n_cells, const int32_t* cells, unsigned flags,
                             ftle_mesh_t* out);

/*
 * Build a mesh from a caller-supplied stencil instead of cells: the
 * neighbour list of Section 2.2 computed elsewhere (the paper's alternative
 * input mode).  Row i of (row_ptr, col) lists the neighbours of point i by
 * caller index, in any order; a repeated entry counts twice in the least
 * squares, -1 entries (the fixed-width list's absent sides) and i itself are
 * dropped.  The rest is as ftle_create_mesh: the stencil need not be
 * symmetric (the adjoint then gathers over its transpose).
 *   row_ptr  host, n_points+1 int64, row_ptr[0] = 0, non-decreasing; copied
 *   col      host, row_ptr[n_points] int32 in [-1, n_points); copied
 *   flags    FTLE_NO_REORDER, FTLE_HOST_ONLY, FTLE_TILE(k)
 * Errors: as ftle_create_mesh; BAD_MESH for a decreasing row_ptr, a
 * row_ptr[0] other than 0 or an entry out of range.
 */
ftle_status ftle_create_mesh_from_csr(int dim, int64_t n_points, const void* coords, ftle_dtype dtype,
                                      const int64_t* row_ptr, const int32_t* col, unsigned flags,
                                      ftle_mesh_t* out);

/*
 * Build a mesh from device coordinates and cells, every step on the device:
 * the one-ring neighbour determination of Section 2.2 (which the paper runs
 * on the host and its Conclusions name as future work for the accelerator),
 * the Morton order, the tile cut and the tile records, and in 3D the
 * inverse normal matrices; with FTLE_STENCIL_AXIS also the axis stencil and
 * its transpose (the adjoint's tiles).  The mesh is the one ftle_create_mesh
 * builds from the same arguments: the same permutation, stencil, tiles and
 * record bytes, hence bit-identical results from every call on it.  The host steers the steps from small downloads (bounds,
 * a 2^16-pair sample of the caller's order, tile sizes); the stencil and the
 * records stay on the device, and ftle_mesh_get_csr / ftle_mesh_get_tiles
 * copy them out when asked.
 *   coords   device pointer (current device), n_points x dim, float or
 *            double; copied into the mesh, must be finite
 *   cells    device pointer, n_cells x (dim+1) int32; read during the call
 *   n_cells  >= 0, at most (2^32-1) / (dim+1)
 *   flags    FTLE_STENCIL_*, FTLE_NO_REORDER, FTLE_TILE(k)
 *   stream   every kernel and copy of the build runs on it; the call
 *            returns when the mesh is complete (it synchronises the stream)
 * Errors: as ftle_create_mesh (the lowest faulty cell is reported);
 * UNSUPPORTED for FTLE_HOST_ONLY, a point whose incident
 * cells list more than 4096 points, or more than 2^31-1 stencil entries.
 */
ftle_status ftle_create_mesh_device(int dim, int64_t n_points, const void* coords, ftle_dtype dtype,
                                    int64_t n_cells, const int32_t* cells, unsigned flags, ftle_stream_t stream,
                                    ftle_mesh_t* out);

/*
 * ftle_create_mesh_from_csr with the stencil on the device, and every step of
 * the build there (the Morton order, the rows moved to Morton positions and
 * sorted, the transpose for the adjoint when the stencil is not symmetric,
 * the tiles and records): the same mesh, byte for byte.  Takes the output of
 * ftle_ring1_csr, or the paper's fixed-width list as it stands (row_ptr[i] =
 * 2 dim i; its -1 entries are dropped).
 *   coords   device pointer, n_points x dim, float or double; copied
 *   row_ptr  device, n_points+1 int64, row_ptr[0] = 0, non-decreasing; read
 *            during the call (row_ptr[n_points] is copied to the host first)
 *   col      device, row_ptr[n_points] int32 in [-1, n_points); read during
 *            the call
 *   flags    FTLE_NO_REORDER, FTLE_TILE(k)
 *   stream   as ftle_create_mesh_device
 * Errors: as ftle_create_mesh_from_csr (the lowest faulty row or entry is
 * reported); UNSUPPORTED for FTLE_HOST_ONLY.
 */
ftle_status ftle_create_mesh_device_from_csr(int dim, int64_t n_points, const void* coords, ftle_dtype dtype,
                                             const int64_t* row_ptr, const int32_t* col, unsigned flags,
                                             ftle_stream_t stream, ftle_mesh_t* out);

/*
 * The one-ring stencil of a cell mesh, built on the device: row i lists, in
 * ascending order and once each, every other point that shares a cell with
 * point i (the neighbour determination that Section 2.2 keeps off the
 * accelerator and the Conclusions name as future work; the same stencil
 * ftle_create_mesh builds on the host).  Hand-written kernels: incidence
 * counts and their scan, each point's incident cells, then each point's
 * distinct neighbours sorted in LDS, counted, scanned into row_ptr and
 * written.  The result feeds ftle_create_mesh_from_csr.
 *   dim          2 (triangles) or 3 (tetrahedra)
 *   n_points     1 <= n_points <= 2^31-1
 *   n_cells      >= 0, at most (2^32-1) / (dim+1)
 *   cells        device, n_cells x (dim+1) int32 point indices; a point
 *                repeated inside a cell adds no pair with itself
 *   row_ptr      device, n_points+1 int64, caller-owned, overwritten
 *   col          device, col_capacity int32, caller-owned; receives *nnz entries
 *   col_capacity n_cells * dim * (dim+1) always suffices
 *   nnz          host, receives the entry count (also when it exceeds
 *                col_capacity)
 * ftle_ring1_csr takes its workspace (ftle_ring1_csr_workspace bytes: the
 * larger of 4 bytes per cell corner and 64 (2D) or 128 (3D) bytes per point,
 * plus about 144 bytes per point) from the device memory the mesh builds keep
 * between calls (ftle_release_cached_memory), growing it if needed;
 * ftle_ring1_csr_ws takes it from the caller (device memory of at least that
 * size, overwritten).  Both return after the stream has finished
 * the work.
 * Errors: INVALID_ARG (dim, n_points < 1, n_cells < 0, null pointer, too
 * small a workspace), BAD_MESH (a cell index outside [0, n_points), found on
 * the device; row_ptr and col are then not written), UNSUPPORTED
 * (n_points > 2^31-1, too many cells, a point whose incident cells list more
 * than 4096 points, *nnz > col_capacity: col not written), OOM, DEVICE.
 */
ftle_status ftle_ring1_csr(int dim, int64_t n_points, int64_t n_cells, const int32_t* cells, int64_t* row_ptr,
                           int32_t* col, int64_t col_capacity, int64_t* nnz, ftle_stream_t stream);
ftle_status ftle_ring1_csr_workspace(int dim, int64_t n_points, int64_t n_cells, int64_t* bytes);
ftle_status ftle_ring1_csr_ws(int dim, int64_t n_points, int64_t n_cells, const int32_t* cells, int64_t* row_ptr,
                              int32_t* col, int64_t col_capacity, int64_t* nnz, void* workspace,
                              int64_t workspace_bytes, ftle_stream_t stream);

/* Analytic flows of ftle_advect_rk4. */
typedef enum {
    /* double gyre (Shadden, Lekien and Marsden 2005), 2D; params A, eps, omega
     * (default 0.1, 0.25, 2 pi / 10) */
    FTLE_FLOW_DOUBLE_GYRE = 0,
    /* steady ABC flow, 3D; params A, B, C (default sqrt 3, sqrt 2, 1) */
    FTLE_FLOW_ABC = 1
} ftle_flow;

/*
 * Flow map phi = x(t0 + T) of particles starting at x0 at time t0, by the
 * classical fourth-order Runge-Kutta method in float64 (the step before the
 * FTLE path: the paper's inputs are precomputed flow maps).  Each particle
 * takes max(1, ceil(|T|/dt - 1e-9)) steps of T/steps, at most 10^7: a
 * particle whose per-particle duration Ts[i] is not finite or needs more
 * steps gets NaN.
 *   flow     FTLE_FLOW_* (2D double gyre, 3D ABC)
 *   params   host, 3 doubles, or NULL for the defaults above
 *   n        particles (>= 0)
 *   x0       device, n x dim of dtype (dim 2 or 3 by the flow)
 *   t0s, Ts  device, n doubles each: per-particle start time and duration
 *            (many meshes' windows in one call), or NULL to use t0 / T
 *   dt       largest step (> 0)
 *   phi      device, n x dim of dtype, caller-owned, overwritten; not x0
 * Errors: INVALID_ARG (flow, dtype, n < 0, null pointer with n > 0, dt <= 0,
 * non-finite t0, T or parameter, a common T needing more than 10^7 steps),
 * DEVICE.
 */
ftle_status ftle_advect_rk4(int flow, const double* params, int64_t n, const void* x0, ftle_dtype dtype,
                            const double* t0s, const double* Ts, double t0, double T, double dt, void* phi,
                            ftle_stream_t stream);

/*
 * ftle_advect_rk4 in a velocity field sampled on a regular grid, the form
 * simulation output comes in (UVaFTLE's inputs are flow maps advected from
 * such data, Section 2.2).  The velocity is multilinear in space (bilinear in
 * 2D, trilinear in 3D) and linear in time; a point outside the grid's box
 * takes the value at the nearest point of the box, a time before the first
 * slice or after the last that slice's value.  Same steps, step limit and
 * per-particle windows as ftle_advect_rk4; float64 arithmetic.
 *   dim           2 or 3
 *   shape         host, dim node counts (x first), each in [2, 2^31)
 *   origin        host, dim: coordinates of node 0
 *   spacing       host, dim: node spacing per axis (> 0)
 *   n_times       slices (in [1, 2^31); one slice is a steady field), at times
 *                 t_first + k t_step (t_step > 0 when n_times > 1)
 *   velocity      device, n_times x [nz x] ny x nx x dim of velocity_dtype
 *                 (x fastest: slice k, node (i, j[, l]) at
 *                 ((k nz + l) ny + j) nx + i), read during the call
 *   x0, dtype, t0s, Ts, t0, T, dt, phi, stream   as ftle_advect_rk4
 * Errors: INVALID_ARG (dim, a null pointer, a shape or n_times out of range,
 * non-finite origin, spacing <= 0, t_step <= 0, and as ftle_advect_rk4),
 * DEVICE.
 */
ftle_status ftle_advect_rk4_grid(int dim, const int64_t* shape, const double* origin, const double* spacing,
                                 int64_t n_times, double t_first, double t_step, const void* velocity,
                                 ftle_dtype velocity_dtype, int64_t n, const void* x0, ftle_dtype dtype,
                                 const double* t0s, const double* Ts, double t0, double T, double dt, void* phi,
                                 ftle_stream_t stream);

/* Release a mesh and its device memory (waits for the device).  NULL is a no-op. */
void ftle_destroy_mesh(ftle_mesh_t mesh);

/*
 * The device mesh builds (ftle_create_mesh_device*) and ftle_ring1_csr keep
 * their temporary device memory per device between calls, grown when a call
 * needs more, so that repeated calls do not allocate and free it each time (a
 * few hundred bytes per point: 1.5 GB for a 4.1 M-point tetrahedral mesh).
 * ftle_cached_memory_bytes reports how much is held (all devices);
 * ftle_release_cached_memory frees what no build is using.
 * Errors: INVALID_ARG (bytes NULL), DEVICE.
 */
ftle_status ftle_cached_memory_bytes(int64_t* bytes);
ftle_status ftle_release_cached_memory(void);

/* Dimensions of a mesh: dim, number of points, number of stencil entries, and
 * (one output beyond the plain dimensions) the mesh dtype as an ftle_dtype
 * value.  Any output pointer may be NULL. */
ftle_status ftle_mesh_info(ftle_mesh_t mesh, int* dim, int64_t* n_points, int64_t* nnz,
                           int* dtype);

/*
 * Host copies of the stencil in Morton order (debug/test accessor).
 *   row_ptr  host, n_points+1 int32: row r (Morton position r) spans
 *            col[row_ptr[r] .. row_ptr[r+1])
 *   col      host, nnz int32: Morton positions of the neighbours, ascending
 *   perm     host, n_points int32: perm[r] = caller's index of Morton position r
 * Any output pointer may be NULL.
 */
ftle_status ftle_mesh_get_csr(ftle_mesh_t mesh, int32_t* row_ptr, int32_t* col, int32_t* perm);

/*
 * Tile statistics (host): number of tiles, the largest tile, the total halo
 * entries, and the bytes of the device-resident index records.  Any output
 * pointer may be NULL.
 */
ftle_status ftle_mesh_tile_stats(ftle_mesh_t mesh, int64_t* n_tiles, int64_t* max_tile_points,
                                 int64_t* halo_entries, int64_t* record_bytes);

/*
 * Host copies of the tile records the kernels read (debug/test accessor).
 *   adjoint   0: tiles of the stencil S; 1: tiles of its transpose S^T used by
 *             the adjoint (the same tiles when S is symmetric, as RING1 is)
 *   n_tiles, record_bytes: sizes (either may be NULL)
 *   meta      host, n_tiles x 16 bytes: per tile a uint32 record offset in
 *             16-byte units, then uint16 {P own points, H halo points, nw
 *             stored stencil words, nr index runs, nx explicit rows, nwf
 *             stencil words of all rows}
 *   records   host, record_bytes bytes; per tile, 16-byte aligned, in this
 *             order (S = P + H staged slots: the P own points, a range of the
 *             Morton order, then the H halo points, each part ascending in
 *             caller index; G = ceil(S/32), Q = ceil(P/32)):
 *               uint32 words[nw]  stencil rows of the explicit rows, three
 *                                 10-bit slots per word (bits 0-9, 10-19,
 *                                 20-29), ascending, each row padded to a
 *                                 multiple of 3 with the row's own slot;
 *                                 bits 30-31 of a row's last word: its
 *                                 padding count
 *               uint32 runs[nr]   per run of consecutive caller indices:
 *                                 caller index of its first slot minus that
 *                                 slot
 *               uint32 smask[G]   bit l%32 of word l/32: slot l starts a run
 *               uint32 xmask[Q]   bit l%32 of word l/32: row l is explicit
 *               uint16 spre[G], xpre[Q]  set bits before each word
 *               uint16 xlast[Q]   last explicit row before row 32 q
 *               uint16 xend[nx]   cumulative word ends of the explicit rows
 *             Row l is explicit unless it equals row l-1 with every slot
 *             plus one; then it is its last explicit row a plus l - a.
 *             P + H <= 1024: larger nominal tiles are split when built.
 * meta and records may be NULL (sizes only).
 */
ftle_status ftle_mesh_get_tiles(ftle_mesh_t mesh, int adjoint, int64_t* n_tiles, int64_t* record_bytes,
                                void* meta, void* records);

/*
 * Threads per workgroup of this mesh's forward (and forward+tape) kernel and
 * of its adjoint gather kernel: each 128, 256 or 512 (0 keeps the current
 * value; the default is 256 in 2D and 512 in 3D).  A workgroup always
 * processes one whole tile.
 * Errors: INVALID_ARG for a NULL mesh or another block size.
 */
ftle_status ftle_mesh_set_blocks(ftle_mesh_t mesh, int fwd_block, int adjoint_block);

/* The current threads per workgroup of the forward and adjoint kernels of a
 * mesh (either output pointer may be NULL). */
ftle_status ftle_mesh_get_blocks(ftle_mesh_t mesh, int* fwd_block, int* adjoint_block);

/*
 * Forward FTLE (the per-point kernel of Section 2).
 *   flow     device pointer, n_points x dim of dtype, the flow map phi(x_i) in user order
 *   dtype    must equal the mesh's dtype
 *   T        integration time; T != 0 and finite; the sign is ignored (|T|)
 *   out      device pointer, n_points of dtype; overwritten with FTLE in user order
 * flow and out must not overlap.
 */
ftle_status ftle_forward(ftle_mesh_t mesh, const void* flow, ftle_dtype dtype, double T,
                         void* out, ftle_stream_t stream);

/*
 * The paper's own neighbour list (Section 2.2; Table 1's 128 / 192 index bits
 * per point) as the kernel's input, with no mesh object: per point exactly
 * 2*dim int32 indices, one per signed axis direction in the order -x, +x,
 * -y, +y (2D), then -z, +z (3D), -1 where a side has no neighbour, row-major
 * n_points x 2*dim in the caller's point order, no row pointers.
 * ftle_axis_ell builds the list on the device from a one-ring stencil: for
 * each side, among the stencil's neighbours j with s (x_j - x_i)_d > 0, the
 * one with the largest cosine s (x_j - x_i)_d / |x_j - x_i|, ties to the
 * smaller index (the FTLE_STENCIL_AXIS stencil as a fixed-width list), in
 * float64.
 *   coords    device, n_points x dim of dtype
 *   row_ptr   device, n_points+1 int64; col device int32 (as ftle_ring1_csr
 *             writes them; rows in any order; entries outside [0, n_points)
 *             and i itself are skipped)
 *   ell       device, n_points x 2*dim int32, caller-owned, overwritten;
 *             16-byte aligned in 2D, 8-byte aligned in 3D
 * ftle_forward_ell computes FTLE from such a list, one lane per point, in the
 * caller's point order (no reordering, no tiles): least squares over the
 * present slots, C = J^T J, its largest eigenvalue, ln sqrt(lambda) / |T|.
 *   coords, ell  as above (entries outside [0, n_points) and i itself are
 *             treated as absent)
 *   flow      device, n_points x dim of dtype; out device, n_points of dtype
 *   flags     FTLE_ELL_DIRECT: every neighbour gathered from global memory
 *             (the paper's layout without reuse); FTLE_ELL_STAGED: each
 *             workgroup's block of 256 consecutive points staged in LDS first,
 *             neighbours inside the block read there
 * Points with fewer than dim usable neighbours, or neighbours that do not
 * span the space, get NaN; the 3D float32 eigenvalue takes the float64
 * recompute as ftle_forward does (not counted).
 * Errors: INVALID_ARG (dim, dtype, n_points < 0, NULL pointer, T, flag,
 * alignment), UNSUPPORTED (n_points > 2^31-1), DEVICE.
 */
enum { FTLE_ELL_DIRECT = 0, FTLE_ELL_STAGED = 1 };
ftle_status ftle_axis_ell(int dim, int64_t n_points, const void* coords, ftle_dtype dtype, const int64_t* row_ptr,
                          const int32_t* col, int32_t* ell, ftle_stream_t stream);
ftle_status ftle_forward_ell(int dim, int64_t n_points, const void* coords, ftle_dtype dtype, const int32_t* ell,
                             const void* flow, double T, void* out, unsigned flags, ftle_stream_t stream);

/*
 * Half-precision flow-map storage, 2D float32 meshes (the precision-for-
 * bandwidth trade Section 1.1 allows: 4 bytes of flow map per point, not 8).
 * The flow map is held as the displacement d = phi - x of each point,
 * rounded to binary16; the forward decodes phi' = x + d in float32 and
 * computes the float32 FTLE of phi' (as ftle_forward would of phi').
 * ftle_encode_flow_f16:
 *   flow     device, n_points x 2 float32, phi in user order
 *   delta    device, n_points x 2 binary16, caller-owned, overwritten with
 *            binary16(phi - x) (the float32 difference rounded to nearest
 *            even; beyond +-65504 it is +-inf, and the FTLE there not finite)
 * ftle_forward_f16:
 *   delta    device, n_points x 2 binary16, as ftle_encode_flow_f16 writes it
 *   T, out   as ftle_forward (out float32)
 * The FTLE of phi' differs from that of phi by the displacement's rounding
 * (2^-11 relative to |d|) over the neighbour spacing: a trade of accuracy
 * for bytes, not a float32 result.
 * Errors: INVALID_ARG (NULL pointer, T), UNSUPPORTED (3D or float64 mesh,
 * n_points >= 2^29, host-only mesh), DEVICE.
 */
ftle_status ftle_encode_flow_f16(ftle_mesh_t mesh, const void* flow, void* delta, ftle_stream_t stream);
ftle_status ftle_forward_f16(ftle_mesh_t mesh, const void* delta, double T, void* out, ftle_stream_t stream);

/*
 * Bytes of the adjoint tape written by ftle_forward_tape (2*dim+1 values of
 * dtype per point).
 */
ftle_status ftle_tape_bytes(ftle_mesh_t mesh, int64_t* bytes);

/*
 * Forward FTLE that also records, per point, what the adjoint needs
 * (p = J v / (|T| lambda), h = M^{-1} v, with v the unit top eigenvector of
 * C, and for a non-symmetric stencil sigma = h . sum_j (x_j - x_i), which
 * the adjoint otherwise forms itself).  The tape's layout is internal.  In
 * 3D the M^{-1} of every point is the mesh's, formed once in float64 when
 * the mesh is created, so that out agrees with ftle_forward's to rounding
 * (not bit for bit).  Points without a usable FTLE put zeros on the tape.
 * Same arguments as ftle_forward plus
 *   tape     device pointer of ftle_tape_bytes() bytes, caller-owned, overwritten
 */
ftle_status ftle_forward_tape(ftle_mesh_t mesh, const void* flow, ftle_dtype dtype, double T,
                              void* out, void* tape, ftle_stream_t stream);

/*
 * Adjoint from a tape: dL/dphi for L = sum_i g_i FTLE_i, with the tape of an
 * ftle_forward_tape call on the same mesh and flow map.
 *   grad_ftle  device pointer, n_points of dtype (g, user order)
 *   grad_flow  device pointer, n_points x dim of dtype; overwritten (not accumulated)
 * Points whose FTLE is not finite contribute nothing.
 */
ftle_status ftle_backward_tape(ftle_mesh_t mesh, const void* tape, ftle_dtype dtype,
                               const void* grad_ftle, void* grad_flow, ftle_stream_t stream);

/*
 * Adjoint without a tape: recomputes the forward quantities from the flow
 * map into a workspace owned by the mesh, then gathers dL/dphi.
 *   flow, dtype, T as in ftle_forward; grad_ftle, grad_flow as in ftle_backward_tape.
 * The workspace (ftle_tape_bytes) is allocated on the mesh's first call and
 * kept until ftle_destroy_mesh; ftle_backward_noalloc is the variant that
 * allocates nothing.  Calls on one mesh share the workspace: they are ordered
 * on the device (a later call on another stream waits for the previous one).
 */
ftle_status ftle_backward(ftle_mesh_t mesh, const void* flow, ftle_dtype dtype, double T,
                          const void* grad_ftle, void* grad_flow, ftle_stream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): ftle_backward
 * with its tape in a fixed 128 MiB device array that the library holds on
 * each GPU it runs on (until the process ends) instead of a workspace it
 * allocates.  The call allocates nothing, on the device or the host; its
 * results equal ftle_backward's bit for bit (same kernels).
 *   arguments as ftle_backward
 * Limit: the tape, n_points * (2 dim + 1) values of dtype, must fit 128 MiB
 * (3D float32: up to 4,793,490 points; 2D float32: 6,710,886; 3D float64:
 * 2,396,745; 2D float64: 3,355,443).
 * Every call on one GPU shares that GPU's array and leaves its tape there:
 * calls that overlap on one GPU (on different streams, or from several host
 * threads) race; order them on one stream.
 * Errors: as ftle_backward; UNSUPPORTED for a mesh whose tape exceeds the
 * limit (checked before any device work).
 */
ftle_status ftle_backward_noalloc(ftle_mesh_t mesh, const void* flow, ftle_dtype dtype, double T,
                                  const void* grad_ftle, void* grad_flow, ftle_stream_t stream);

/*
 * Batched forward FTLE over independent meshes (same dim and dtype), in one
 * launch over a work list of (mesh, tile) items, replayed from a cached HIP
 * graph.  The first call for a given list of meshes builds the work list,
 * times candidate launch shapes -- a persistent grid draining an atomic work
 * queue (threads per workgroup, tiles per queue pop, resident workgroups per
 * CU) or a flat grid of one workgroup per tile -- and keeps the fastest;
 * later calls only update the graph node's arguments.  Each output equals
 * ftle_forward's bit for bit (same tile body).  Calls with one list of meshes
 * share its queue counters: a call on another stream than the previous call
 * with that list waits (on the device) for the previous launch.
 *   n         1 <= n <= 64 meshes
 *   meshes    host array of n handles (all dim and dtype equal)
 *   flows     host array of n device pointers (flow maps, user order)
 *   T         host array of n integration times (each nonzero and finite)
 *   outs      host array of n device pointers (FTLE outputs)
 * Errors: INVALID_ARG (n, NULL arrays or pointers, T, mixed dim or device),
 * DTYPE, UNSUPPORTED (host-only mesh), DEVICE.
 */
ftle_status ftle_batched(int n, const ftle_mesh_t* meshes, const void* const* flows,
                         const double* T, void* const* outs, ftle_dtype dtype,
                         ftle_stream_t stream);

/*
 * The launch shape the batched autotuner chose for this list of meshes
 * (after at least one ftle_batched call with it): threads per workgroup,
 * tiles taken per queue pop (0 for the flat one-tile-per-workgroup grid),
 * workgroups in the grid.
 */
ftle_status ftle_batched_config(int n, const ftle_mesh_t* meshes, int* block, int* tiles_per_pop,
                                int* grid);

/*
 * Number of points whose 3D float32 eigenvalue was recomputed in float64
 * because the top two eigenvalues of C were nearly equal, accumulated over
 * forward calls on this mesh since the last reset.  Synchronises the device.
 */
ftle_status ftle_mesh_fp64_hits(ftle_mesh_t mesh, int64_t* hits, int reset);

/*
 * Testing aid: while on is nonzero, every launch uses the kernels' 64-bit
 * element offsets, the code path otherwise taken only when some per-point
 * array of a mesh reaches 4 GiB, so that path can be checked against the
 * default one on small meshes.  Process-wide; a batched plan keeps the choice
 * it was built with.  Always returns FTLE_OK.
 */
ftle_status ftle_force_wide_offsets(int on);

/*
 * Testing aid: the threshold of the 3D float32 eigenvalue recompute.  The
 * trigonometric eigenvalue formula (lambda = q + 2 p cos(acos(r)/3)) loses
 * accuracy where r -> -1, i.e. where the two largest eigenvalues of C nearly
 * coincide; points with r + 1 < tau redo C = J^T J and the formula in
 * float64 from the float32 Jacobian (ftle_mesh_fp64_hits counts them).
 *   tau  >= 0: the new threshold (0 disables the recompute; any tau > 2
 *        sends every point with a usable stencil through it, since
 *        r + 1 <= 2); < 0: back to the default (the FTLE_EIG_TAU environment
 *        variable, read once, else 2e-3).
 * Process-wide; it applies to forward, tape-forward, adjoint and batched
 * launches enqueued after the call.
 * Errors: INVALID_ARG for a NaN or infinite tau.
 */
ftle_status ftle_set_eig_threshold(double tau);

/* The threshold ftle_set_eig_threshold set, or the default.
 * Errors: INVALID_ARG for a NULL tau. */
ftle_status ftle_get_eig_threshold(double* tau);

/*
 * Testing aid: pin the launch shape of ftle_batched instead of autotuning it,
 * so that every form can be checked against ftle_forward.
 *   block          0: unpin (lists of meshes without a chosen shape are
 *                  autotuned again; the others keep theirs); else 128, 256
 *                  or 512 threads per workgroup
 *   tiles_per_pop  0: the flat grid (one workgroup per tile); 1..64: the
 *                  persistent grid draining the atomic queue, that many
 *                  tiles per pop
 *   per_cu_cap     persistent grid only: at most this many resident
 *                  workgroups per CU (1..32; ignored when tiles_per_pop is 0)
 * Process-wide: the next ftle_batched call of every list of meshes adopts the
 * pinned shape (rebuilding its cached graph) until it is unpinned.
 * ftle_batched_config reports the shape in use.
 * Errors: INVALID_ARG for a value outside these ranges.
 */
ftle_status ftle_batched_pin_config(int block, int tiles_per_pop, int per_cu_cap);

/* Message of the last failure on the calling thread ("" if none). */
const char* ftle_last_error(void);

/* Library version string. */
const char* ftle_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FTLE_H */
