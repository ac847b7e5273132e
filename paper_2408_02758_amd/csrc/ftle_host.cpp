// Host side of the FTLE library: the C ABI declared in include/ftle.h.
//
// Mesh creation does, on the CPU, what Section 2.2 of de Castro et al.
// assigns to the host processor: it determines every point's neighbours once
// (from the cells, or takes them from the caller) and stores them as a list
// of integer indices that the accelerator then reads in a fixed order.  On
// top of that it orders the points along a Morton curve and cuts the order
// into LDS-sized tiles with compressed records (see ftle_internal.h for the
// layout), so the GPU reads every index sequentially and every coordinate and
// flow-map value about once.  The flow-map advection entry point
// (ftle_advect_rk4) is validated here too.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/ftle.h"
#include "ftle_internal.h"

using namespace ftle;

// ===========================================================================
// Errors
// ===========================================================================
namespace {

thread_local std::string g_last_error;

struct Failure {
    ftle_status status;
    std::string msg;
};

[[noreturn]] void fail(ftle_status st, const std::string& msg) { throw Failure{st, msg}; }

void check_hip(hipError_t e, const char* what)
{
    if (e != hipSuccess) {
        const ftle_status st = (e == hipErrorOutOfMemory) ? FTLE_ERR_OOM : FTLE_ERR_DEVICE;
        fail(st, std::string(what) + ": " + hipGetErrorString(e));
    }
}

template <typename F>
ftle_status guarded(F&& body)
{
    try {
        body();
        g_last_error.clear();
        return FTLE_OK;
    } catch (const Failure& f) {
        g_last_error = f.msg;
        return f.status;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return FTLE_ERR_OOM;
    } catch (const std::exception& e) {
        g_last_error = std::string("internal error: ") + e.what();
        return FTLE_ERR_DEVICE;
    } catch (...) {
        g_last_error = "internal error";
        return FTLE_ERR_DEVICE;
    }
}

// ===========================================================================
// Small host utilities
// ===========================================================================
int host_threads()
{
    unsigned hc = std::thread::hardware_concurrency();
    if (const char* e = std::getenv("FTLE_HOST_THREADS")) hc = (unsigned)std::max(1, std::atoi(e));
    return (int)std::max(1u, std::min(hc, 32u));
}

// Run body(begin, end) over [0, n) split into contiguous chunks, one per thread.
template <typename F>
void parallel_for(int64_t n, F&& body, int64_t min_chunk = 16384)
{
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), (n + min_chunk - 1) / min_chunk));
    if (nt <= 1) {
        body((int64_t)0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    std::vector<std::exception_ptr> err(nt);
    for (int t = 0; t < nt; ++t) {
        const int64_t b = n * t / nt, e = n * (t + 1) / nt;
        th.emplace_back([&, b, e, t] {
            try {
                body(b, e, t);
            } catch (...) {
                err[t] = std::current_exception();
            }
        });
    }
    for (auto& x : th) x.join();
    for (auto& e : err)
        if (e) std::rethrow_exception(e);
}

// Spread the low 32 bits of v to the even bit positions of a 64-bit word.
uint64_t spread2(uint64_t v)
{
    v &= 0xffffffffULL;
    v = (v | (v << 16)) & 0x0000ffff0000ffffULL;
    v = (v | (v << 8)) & 0x00ff00ff00ff00ffULL;
    v = (v | (v << 4)) & 0x0f0f0f0f0f0f0f0fULL;
    v = (v | (v << 2)) & 0x3333333333333333ULL;
    v = (v | (v << 1)) & 0x5555555555555555ULL;
    return v;
}

// Spread the low 21 bits of v to every third bit position.
uint64_t spread3(uint64_t v)
{
    v &= 0x1fffffULL;
    v = (v | (v << 32)) & 0x001f00000000ffffULL;
    v = (v | (v << 16)) & 0x001f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

// Stable LSD radix sort of (key, value) pairs by key, 16 bits per pass.
void radix_sort_pairs(std::vector<uint64_t>& key, std::vector<int32_t>& val)
{
    const size_t n = key.size();
    std::vector<uint64_t> k2(n);
    std::vector<int32_t> v2(n);
    std::vector<size_t> cnt(65536 + 1);
    for (int pass = 0; pass < 4; ++pass) {
        const int sh = 16 * pass;
        std::fill(cnt.begin(), cnt.end(), 0);
        for (size_t i = 0; i < n; ++i) ++cnt[((key[i] >> sh) & 0xffff) + 1];
        bool trivial = false;
        for (size_t d = 1; d <= 65536; ++d)
            if (cnt[d] == n) trivial = true;
        if (trivial) continue;
        for (size_t d = 0; d < 65536; ++d) cnt[d + 1] += cnt[d];
        for (size_t i = 0; i < n; ++i) {
            const size_t p = cnt[(key[i] >> sh) & 0xffff]++;
            k2[p] = key[i];
            v2[p] = val[i];
        }
        key.swap(k2);
        val.swap(v2);
    }
}

// ===========================================================================
// CSR helpers (rows and columns are Morton positions)
// ===========================================================================
struct Csr {
    std::vector<int32_t> row_ptr;  // n+1 (int32: nnz < 2^31 is checked)
    std::vector<int32_t> col;
};

Csr transpose(const Csr& a, int64_t n)
{
    Csr t;
    t.row_ptr.assign(n + 1, 0);
    for (int32_t c : a.col) ++t.row_ptr[c + 1];
    for (int64_t i = 0; i < n; ++i) t.row_ptr[i + 1] += t.row_ptr[i];
    t.col.resize(a.col.size());
    std::vector<int32_t> fill(t.row_ptr.begin(), t.row_ptr.end() - 1);
    for (int64_t r = 0; r < n; ++r)
        for (int32_t p = a.row_ptr[r]; p < a.row_ptr[r + 1]; ++p) t.col[fill[a.col[p]]++] = (int32_t)r;
    return t;  // rows ascending by construction
}

bool csr_equal(const Csr& a, const Csr& b) { return a.row_ptr == b.row_ptr && a.col == b.col; }

}  // namespace

// ===========================================================================
// Mesh object
// ===========================================================================
struct TileSet {
    std::vector<TileMeta> meta;
    std::vector<uint32_t> rec;     // record words (16-byte aligned blocks)
    int max_staged = 0;
    int max_rec = 0;
    int max_P = 0;
    int64_t halo_total = 0;
    int64_t rec_bytes = 0;    // records on the device (rec holds a host copy unless built there)
    void* d_meta = nullptr;
    void* d_rec = nullptr;
    void* d_minv = nullptr;   // 3D forward tile set: inverse normal matrices (caller order)

    DevTiles dev() const
    {
        DevTiles d;
        d.meta = static_cast<const TileMeta*>(d_meta);
        d.rec = static_cast<const uint4*>(d_rec);
        d.minv = d_minv;
        d.n_tiles = (int)meta.size();
        d.max_staged = max_staged;
        d.max_rec = max_rec;
        return d;
    }
};

struct ftle_mesh_s {
    int dim = 0;
    int64_t n = 0;
    ftle_dtype dtype = FTLE_F32;
    unsigned flags = 0;
    int tile_points = 0;
    int fwd_block = 256;
    int bwd_block = 256;
    bool symmetric = true;
    bool host_only = false;
    bool device_built = false;     // perm, csr and tile records live on the device only
    int64_t nnz = 0;               // stencil entries
    std::vector<int32_t> perm;     // Morton position -> user index
    Csr csr;                       // forward stencil, Morton positions
    int32_t* d_perm = nullptr;     // device-built: perm, stencil row offsets (int64) and columns
    int64_t* d_row_ptr = nullptr;
    int32_t* d_col = nullptr;
    TileSet fwd, bwd;              // bwd empty when symmetric (fwd serves both)
    std::vector<unsigned char> x_user;   // coordinates, user order, dtype
    int device = -1;
    void* d_x = nullptr;
    unsigned long long* d_hits = nullptr;
    void* d_work = nullptr;        // adjoint workspace (tape) of ftle_backward
    hipEvent_t work_done = nullptr;
    hipStream_t work_stream = nullptr;
    std::mutex mu;

    bool f64() const { return dtype == FTLE_F64; }
    size_t elem() const { return f64() ? 8 : 4; }
    const TileSet& adj_tiles() const { return symmetric ? fwd : bwd; }
};

namespace {

// ---------------------------------------------------------------------------
// Neighbour stencils (Section 2.2: computed once, on the host)
// ---------------------------------------------------------------------------

// RING1: every point sharing a cell with r, excluding r, ascending.
// cells are already renumbered to Morton positions.
Csr build_ring1(int dim, int64_t n, int64_t ncells, const std::vector<int32_t>& cells)
{
    const int k = dim + 1;
    // point -> incident cells
    std::vector<int64_t> inc_ptr(n + 1, 0);
    for (int64_t c = 0; c < ncells * k; ++c) ++inc_ptr[cells[c] + 1];
    for (int64_t i = 0; i < n; ++i) inc_ptr[i + 1] += inc_ptr[i];
    std::vector<int32_t> inc(inc_ptr[n]);
    {
        std::vector<int64_t> fill(inc_ptr.begin(), inc_ptr.end() - 1);
        for (int64_t c = 0; c < ncells; ++c)
            for (int a = 0; a < k; ++a) inc[fill[cells[c * k + a]]++] = (int32_t)c;
    }
    Csr out;
    out.row_ptr.assign(n + 1, 0);
    std::vector<int64_t> deg(n, 0);
    auto row = [&](int64_t r, std::vector<int32_t>& buf) {
        buf.clear();
        for (int64_t p = inc_ptr[r]; p < inc_ptr[r + 1]; ++p) {
            const int64_t c = inc[p];
            for (int a = 0; a < k; ++a) {
                const int32_t v = cells[c * k + a];
                if (v != r) buf.push_back(v);
            }
        }
        std::sort(buf.begin(), buf.end());
        buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
    };
    parallel_for(n, [&](int64_t b, int64_t e, int) {
        std::vector<int32_t> buf;
        for (int64_t r = b; r < e; ++r) {
            row(r, buf);
            deg[r] = (int64_t)buf.size();
        }
    });
    int64_t total = 0;
    for (int64_t r = 0; r < n; ++r) {
        total += deg[r];
        if (total > INT32_MAX) fail(FTLE_ERR_UNSUPPORTED, "stencil has more than 2^31-1 entries");
        out.row_ptr[r + 1] = (int32_t)total;
    }
    out.col.resize(total);
    parallel_for(n, [&](int64_t b, int64_t e, int) {
        std::vector<int32_t> buf;
        for (int64_t r = b; r < e; ++r) {
            row(r, buf);
            std::copy(buf.begin(), buf.end(), out.col.begin() + out.row_ptr[r]);
        }
    });
    return out;
}

// AXIS: the paper's fixed-width list (4 slots in 2D, 6 in 3D).  Slot (d, s)
// takes, among the RING1 neighbours on side s of axis d, the one with the
// largest cosine to that direction; ties go to the smaller caller index.
// Absent slots are dropped from the row (the -1 entries of the paper's list).
template <typename T>
Csr build_axis(int dim, int64_t n, const Csr& ring, const T* xm /* Morton order */,
               const std::vector<int32_t>& perm)
{
    Csr out;
    out.row_ptr.assign(n + 1, 0);
    std::vector<int32_t> slots((size_t)n * 2 * dim, -1);
    parallel_for(n, [&](int64_t b, int64_t e, int) {
        for (int64_t r = b; r < e; ++r) {
            for (int d = 0; d < dim; ++d)
                for (int sg = 0; sg < 2; ++sg) {
                    const double sigma = sg ? 1.0 : -1.0;
                    double best = 0.0;
                    int32_t arg = -1;
                    for (int32_t p = ring.row_ptr[r]; p < ring.row_ptr[r + 1]; ++p) {
                        const int32_t c = ring.col[p];
                        double nrm2 = 0.0;
                        for (int q = 0; q < dim; ++q) {
                            const double t = (double)xm[(size_t)c * dim + q] - (double)xm[(size_t)r * dim + q];
                            nrm2 += t * t;
                        }
                        const double along = sigma * ((double)xm[(size_t)c * dim + d] - (double)xm[(size_t)r * dim + d]);
                        if (!(along > 0.0)) continue;
                        const double cs = along / std::sqrt(nrm2);
                        if (arg < 0 || cs > best || (cs == best && perm[c] < perm[arg])) {
                            best = cs;
                            arg = c;
                        }
                    }
                    slots[(size_t)r * 2 * dim + 2 * d + sg] = arg;
                }
        }
    });
    for (int64_t r = 0; r < n; ++r) {
        int cnt = 0;
        for (int s = 0; s < 2 * dim; ++s) cnt += slots[(size_t)r * 2 * dim + s] >= 0;
        out.row_ptr[r + 1] = out.row_ptr[r] + cnt;
    }
    out.col.reserve(out.row_ptr[n]);
    for (int64_t r = 0; r < n; ++r)
        for (int s = 0; s < 2 * dim; ++s) {
            const int32_t c = slots[(size_t)r * 2 * dim + s];
            if (c >= 0) out.col.push_back(c);
        }
    return out;
}

// ---------------------------------------------------------------------------
// Tiles
// ---------------------------------------------------------------------------
struct TileExtent {
    int64_t begin, end;
    uint32_t H, nw;
};

// Halo of [b, e): neighbours outside the range, as Morton positions sorted by
// caller index (so the staging gathers of a tile walk memory in order).
void tile_halo(const Csr& a, const std::vector<int32_t>& perm, int64_t b, int64_t e,
               std::vector<uint32_t>& stamp, uint32_t tag, std::vector<int32_t>& halo)
{
    halo.clear();
    for (int64_t r = b; r < e; ++r)
        for (int32_t p = a.row_ptr[r]; p < a.row_ptr[r + 1]; ++p) {
            const int32_t c = a.col[p];
            if (c >= b && c < e) continue;
            if (stamp[c] == tag) continue;
            stamp[c] = tag;
            halo.push_back(c);
        }
    std::sort(halo.begin(), halo.end(), [&](int32_t u, int32_t v) { return perm[u] < perm[v]; });
}

// Stencil words of rows [b, e): each row padded to a multiple of 3 entries.
int64_t padded_words(const Csr& a, int64_t b, int64_t e)
{
    int64_t t = 0;
    for (int64_t r = b; r < e; ++r) t += (a.row_ptr[r + 1] - a.row_ptr[r] + 2) / 3;
    return t;
}

// The least-squares normal matrix of a 3D point i depends on the mesh alone:
// M_i = sum over its stencil row of (x_j - x_i)(x_j - x_i)^T (with repeated
// entries repeated).  Its inverse is formed once, in float64, for the tape
// forward: six values (00, 01, 02, 11, 12, 22) per point in caller order, in
// the mesh dtype, all NaN where M fails the rank test det M > tau (tr M / 3)^3
// (tau = 1e-5 for float32 meshes, 1e-12 for float64, as in the kernels).
std::vector<unsigned char> normal_inverse3(const Csr& a, const std::vector<int32_t>& perm,
                                           const std::vector<double>& xd, bool f64)
{
    const int64_t n = (int64_t)perm.size();
    std::vector<unsigned char> out((size_t)n * 6 * (f64 ? 8 : 4));
    const double tau = f64 ? 1e-12 : 1e-5;
    parallel_for(n, [&](int64_t b, int64_t e, int) {
        for (int64_t r = b; r < e; ++r) {
            const int64_t i = perm[r];
            const double* xi = &xd[(size_t)i * 3];
            double m00 = 0, m01 = 0, m02 = 0, m11 = 0, m12 = 0, m22 = 0;
            for (int32_t p = a.row_ptr[r]; p < a.row_ptr[r + 1]; ++p) {
                const double* xj = &xd[(size_t)perm[a.col[p]] * 3];
                const double d0 = xj[0] - xi[0], d1 = xj[1] - xi[1], d2 = xj[2] - xi[2];
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
                for (double& t : v) t = std::nan("");
            for (int k = 0; k < 6; ++k) {
                if (f64)
                    reinterpret_cast<double*>(out.data())[i * 6 + k] = v[k];
                else
                    reinterpret_cast<float*>(out.data())[i * 6 + k] = (float)v[k];
            }
        }
    });
    return out;
}

// nw: the padded stencil words of all P rows.  The record is checked at its
// largest (every row explicit, one run per slot).
bool tile_fits(int dim, bool f64, int64_t P, int64_t H, int64_t nw)
{
    if (P + H > kMaxStaged || nw > kMaxTileWords) return false;
    const RecLayout r = rec_layout((uint32_t)P, (uint32_t)H, (uint32_t)nw, (uint32_t)(P + H), (uint32_t)P);
    const int S = (int)(P + H);
    if (dim == 3 && S > bwd3_capacity(f64)) return false;
    return std::max(fwd_points_bytes(dim, f64, S), bwd_points_bytes(dim, f64, S)) + r.bytes <= kLdsBudget;
}

// The record of one tile (layout in ftle_internal.h): own points [b, e) of
// the Morton order, halo `halo` (ascending in caller index).
void tile_record(const Csr& a, const std::vector<int32_t>& perm, int64_t b, int64_t e,
                 const std::vector<int32_t>& halo, TileMeta& m, std::vector<uint32_t>& out)
{
    const uint32_t P = (uint32_t)(e - b), H = (uint32_t)halo.size(), S = P + H;
    // own points take slots in caller order, as the halo does: adjacent lanes
    // then load and store adjacent caller-order entries
    std::vector<int32_t> order((size_t)P), slot((size_t)P);
    for (int64_t r = b; r < e; ++r) order[r - b] = (int32_t)r;
    std::sort(order.begin(), order.end(), [&](int32_t u, int32_t v) { return perm[u] < perm[v]; });
    std::vector<uint32_t> caller(S);
    for (uint32_t l = 0; l < P; ++l) {
        caller[l] = (uint32_t)perm[order[l]];
        slot[order[l] - b] = (int32_t)l;
    }
    std::vector<std::pair<int32_t, int32_t>> hs(H);   // (Morton position, slot) of the halo
    for (uint32_t h = 0; h < H; ++h) {
        caller[P + h] = (uint32_t)perm[halo[h]];
        hs[h] = {halo[h], (int32_t)(P + h)};
    }
    std::sort(hs.begin(), hs.end());

    // runs of consecutive caller indices
    std::vector<uint32_t> runs;
    std::vector<uint8_t> starts(S, 0);
    for (uint32_t l = 0; l < S; ++l)
        if (l == 0 || caller[l] != caller[l - 1] + 1u) {
            starts[l] = 1;
            runs.push_back(caller[l] - l);
        }

    // rows: local indices ascending, padded with the row's own slot; a row
    // equal to the previous one plus one is not stored
    std::vector<uint32_t> words, prev, row;
    std::vector<uint16_t> xend;
    std::vector<uint8_t> expl(P, 0);
    uint32_t nwf = 0;
    for (uint32_t l = 0; l < P; ++l) {
        const int64_t r = order[l];
        row.clear();
        for (int32_t p = a.row_ptr[r]; p < a.row_ptr[r + 1]; ++p) {
            const int32_t c = a.col[p];
            if (c >= b && c < e) {
                row.push_back((uint32_t)slot[c - b]);
            } else {
                auto it = std::lower_bound(hs.begin(), hs.end(), std::make_pair(c, INT32_MIN));
                row.push_back((uint32_t)it->second);
            }
        }
        std::sort(row.begin(), row.end());
        const uint32_t pad = (3 - row.size() % 3) % 3;
        for (uint32_t k = 0; k < pad; ++k) row.push_back(l);
        nwf += (uint32_t)row.size() / 3;
        bool shift = l > 0 && row.size() == prev.size();
        for (size_t k = 0; shift && k < row.size(); ++k) shift = row[k] == prev[k] + 1u;
        if (!shift) {
            expl[l] = 1;
            for (size_t k = 0; k < row.size(); k += 3) words.push_back(row[k] | row[k + 1] << 10 | row[k + 2] << 20);
            if (!row.empty()) words.back() |= pad << 30;   // the last word's padding entries
            xend.push_back((uint16_t)words.size());
        }
        prev.swap(row);
    }

    m.P = (uint16_t)P;
    m.H = (uint16_t)H;
    m.nw = (uint16_t)words.size();
    m.nr = (uint16_t)runs.size();
    m.nx = (uint16_t)xend.size();
    m.nwf = (uint16_t)nwf;
    const RecLayout L = rec_layout(m);
    out.assign(L.bytes / 4, 0u);
    unsigned char* base = reinterpret_cast<unsigned char*>(out.data());
    std::memcpy(base, words.data(), words.size() * 4);
    std::memcpy(base + L.runs, runs.data(), runs.size() * 4);
    uint32_t* smask = reinterpret_cast<uint32_t*>(base + L.smask);
    uint32_t* xmask = reinterpret_cast<uint32_t*>(base + L.xmask);
    uint16_t* spre = reinterpret_cast<uint16_t*>(base + L.spre);
    uint16_t* xpre = reinterpret_cast<uint16_t*>(base + L.xpre);
    uint16_t* xlast = reinterpret_cast<uint16_t*>(base + L.xlast);
    uint32_t cnt = 0;
    for (uint32_t l = 0; l < S; ++l) {
        if (l % 32 == 0) spre[l / 32] = (uint16_t)cnt;
        if (starts[l]) {
            smask[l / 32] |= 1u << (l % 32);
            ++cnt;
        }
    }
    cnt = 0;
    uint32_t last = 0;
    for (uint32_t l = 0; l < P; ++l) {
        if (l % 32 == 0) {
            xpre[l / 32] = (uint16_t)cnt;
            xlast[l / 32] = (uint16_t)last;
        }
        if (expl[l]) {
            xmask[l / 32] |= 1u << (l % 32);
            ++cnt;
            last = l;
        }
    }
    std::memcpy(base + L.xend, xend.data(), xend.size() * 2);
}

TileSet build_tiles(int dim, bool f64, int64_t n, int tile_points, const Csr& a,
                    const std::vector<int32_t>& perm)
{
    // 1. extents: nominal chunks of tile_points, halved until they fit the caps
    //    (10-bit local indices, 16-bit row ends, the LDS budget)
    const int64_t nchunks = (n + tile_points - 1) / tile_points;
    std::vector<std::vector<TileExtent>> per_chunk(nchunks);
    parallel_for(nchunks, [&](int64_t cb, int64_t ce, int) {
        std::vector<uint32_t> stamp(n, 0);
        uint32_t tag = 0;
        std::vector<int32_t> halo;
        for (int64_t ch = cb; ch < ce; ++ch) {
            std::vector<std::pair<int64_t, int64_t>> todo{{ch * tile_points, std::min<int64_t>(n, (ch + 1) * tile_points)}};
            while (!todo.empty()) {
                auto [b, e] = todo.back();
                todo.pop_back();
                if (++tag == 0) {
                    std::fill(stamp.begin(), stamp.end(), 0);
                    tag = 1;
                }
                tile_halo(a, perm, b, e, stamp, tag, halo);
                const int64_t nw = padded_words(a, b, e);
                if (tile_fits(dim, f64, e - b, (int64_t)halo.size(), nw)) {
                    per_chunk[ch].push_back({b, e, (uint32_t)halo.size(), (uint32_t)nw});
                } else if (e - b == 1) {
                    fail(FTLE_ERR_UNSUPPORTED, "point " + std::to_string(perm[b]) + " has " +
                                                   std::to_string(a.row_ptr[b + 1] - a.row_ptr[b]) +
                                                   " neighbours, more than one tile holds");
                } else {
                    const int64_t m = b + (e - b) / 2;
                    todo.push_back({m, e});   // processed after [b, m): keeps ascending order
                    todo.push_back({b, m});
                }
            }
        }
    }, 1);
    std::vector<TileExtent> ext;
    for (auto& v : per_chunk) ext.insert(ext.end(), v.begin(), v.end());

    // 2. records, then their offsets
    TileSet ts;
    ts.meta.resize(ext.size());
    std::vector<std::vector<uint32_t>> recs(ext.size());
    parallel_for((int64_t)ext.size(), [&](int64_t tb, int64_t te, int) {
        std::vector<uint32_t> stamp(n, 0);
        std::vector<int32_t> halo;
        uint32_t tag = 0;
        for (int64_t t = tb; t < te; ++t) {
            if (++tag == 0) {
                std::fill(stamp.begin(), stamp.end(), 0);
                tag = 1;
            }
            tile_halo(a, perm, ext[t].begin, ext[t].end, stamp, tag, halo);
            tile_record(a, perm, ext[t].begin, ext[t].end, halo, ts.meta[t], recs[t]);
        }
    }, 1);
    uint64_t off = 0;  // in 16-byte units
    for (size_t t = 0; t < ext.size(); ++t) {
        if (off > UINT32_MAX) fail(FTLE_ERR_UNSUPPORTED, "tile records exceed 64 GiB");
        TileMeta& m = ts.meta[t];
        m.rec_off = (uint32_t)off;
        off += recs[t].size() / 4;
        ts.max_staged = std::max(ts.max_staged, (int)(m.P + m.H));
        ts.max_rec = std::max(ts.max_rec, (int)(recs[t].size() * 4));
        ts.max_P = std::max(ts.max_P, (int)m.P);
        ts.halo_total += m.H;
    }
    ts.rec.resize(off * 4);
    ts.rec_bytes = (int64_t)off * 16;
    parallel_for((int64_t)ext.size(), [&](int64_t tb, int64_t te, int) {
        for (int64_t t = tb; t < te; ++t)
            std::copy(recs[t].begin(), recs[t].end(), ts.rec.begin() + (size_t)ts.meta[t].rec_off * 4);
    }, 1);
    return ts;
}

// ---------------------------------------------------------------------------
// Device memory
// ---------------------------------------------------------------------------
void* dev_upload(const void* src, size_t bytes)
{
    void* p = nullptr;
    if (bytes == 0) bytes = 16;
    check_hip(hipMalloc(&p, bytes), "hipMalloc");
    if (src) {
        const hipError_t e = hipMemcpy(p, src, bytes, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(p);
            check_hip(e, "hipMemcpy");
        }
    }
    return p;
}

void free_tiles(TileSet& t)
{
    if (t.d_meta) (void)hipFree(t.d_meta);
    if (t.d_rec) (void)hipFree(t.d_rec);
    if (t.d_minv) (void)hipFree(t.d_minv);
    t.d_meta = t.d_rec = t.d_minv = nullptr;
}

void upload_tiles(TileSet& t)
{
    t.d_meta = dev_upload(t.meta.data(), t.meta.size() * sizeof(TileMeta));
    t.d_rec = dev_upload(t.rec.data(), t.rec.size() * sizeof(uint32_t));
}

void release_device(ftle_mesh_s* m)
{
    if (m->device < 0) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(m->device);
    (void)hipDeviceSynchronize();
    free_tiles(m->fwd);
    free_tiles(m->bwd);
    if (m->d_x) (void)hipFree(m->d_x);
    if (m->d_hits) (void)hipFree(m->d_hits);
    if (m->d_work) (void)hipFree(m->d_work);
    if (m->work_done) (void)hipEventDestroy(m->work_done);
    if (m->d_perm) (void)hipFree(m->d_perm);
    if (m->d_row_ptr) (void)hipFree(m->d_row_ptr);
    if (m->d_col) (void)hipFree(m->d_col);
    m->d_perm = nullptr;
    m->d_row_ptr = nullptr;
    m->d_col = nullptr;
    m->d_x = nullptr;
    m->d_hits = nullptr;
    m->d_work = nullptr;
    m->work_done = nullptr;
    (void)hipSetDevice(cur);
}

// ---------------------------------------------------------------------------
// Tunables (environment, read once)
// ---------------------------------------------------------------------------
double env_double(const char* name, double dflt)
{
    const char* v = std::getenv(name);
    return v ? std::atof(v) : dflt;
}

// r < -1 + tau selects the float64 eigenvalue recompute (3D, float32 meshes).
// The default comes from FTLE_EIG_TAU (read once) or is 2e-3;
// ftle_set_eig_threshold replaces it at run time.
double default_eig_tau()
{
    static const double t = env_double("FTLE_EIG_TAU", 2e-3);
    return t;
}
std::atomic<double> g_eig_tau{-1.0};   // < 0: the default
double eig_tau()
{
    const double t = g_eig_tau.load(std::memory_order_relaxed);
    return t < 0.0 ? default_eig_tau() : t;
}

void check_mesh(ftle_mesh_t m)
{
    if (!m) fail(FTLE_ERR_INVALID_ARG, "mesh is NULL");
}

// Called after every argument check, right before device work.
void need_device(ftle_mesh_t m)
{
    if (m->host_only) fail(FTLE_ERR_UNSUPPORTED, "mesh was created with FTLE_HOST_ONLY");
}

void check_T(double T)
{
    if (!(T != 0.0) || !std::isfinite(T)) fail(FTLE_ERR_INVALID_ARG, "T must be finite and nonzero");
}

void check_dtype(ftle_mesh_t m, ftle_dtype d)
{
    if (d != FTLE_F32 && d != FTLE_F64) fail(FTLE_ERR_INVALID_ARG, "unknown dtype");
    if (d != m->dtype) fail(FTLE_ERR_DTYPE, "dtype differs from the mesh's dtype");
}

struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev)
    {
        check_hip(hipGetDevice(&prev), "hipGetDevice");
        if (prev != dev) check_hip(hipSetDevice(dev), "hipSetDevice");
    }
    ~DeviceScope()
    {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* ftle_last_error(void) { return g_last_error.c_str(); }

const char* ftle_version(void) { return "ftle-mi355x 0.1 (gfx950)"; }

ftle_status ftle_force_wide_offsets(int on)
{
    set_force_wide(on != 0);
    return FTLE_OK;
}

ftle_status ftle_set_eig_threshold(double tau)
{
    return guarded([&] {
        if (std::isnan(tau) || std::isinf(tau)) fail(FTLE_ERR_INVALID_ARG, "tau must be finite");
        g_eig_tau.store(tau < 0.0 ? -1.0 : tau, std::memory_order_relaxed);
    });
}

ftle_status ftle_get_eig_threshold(double* tau)
{
    return guarded([&] {
        if (!tau) fail(FTLE_ERR_INVALID_ARG, "tau is NULL");
        *tau = eig_tau();
    });
}

// The axis along which the caller's point order advances, or -1: over a
// sample of consecutive caller indices the median step is about one spacing
// along that axis and under a quarter spacing along every other axis.  The
// sample: m pairs (points k stride and k stride + 1), none below 64 points.
void order_sample(int64_t n, int64_t* m, int64_t* stride)
{
    *m = n < 64 ? 0 : std::min<int64_t>(n - 1, 1 << 16);
    *stride = *m ? (n - 1) / *m : 0;
}

// pairs[k * 2 dim + d] and [k * 2 dim + dim + d]: axis d of the two points of sample k.
int order_axis_from_pairs(int dim, int64_t m, const double* pairs, const double* unit)
{
    if (m == 0) return -1;
    double med[3] = {0, 0, 0};
    std::vector<double> v((size_t)m);
    for (int d = 0; d < dim; ++d) {
        for (int64_t k = 0; k < m; ++k)
            v[(size_t)k] = std::fabs(pairs[k * 2 * dim + dim + d] - pairs[k * 2 * dim + d]) / unit[d];
        std::nth_element(v.begin(), v.begin() + m / 2, v.end());
        med[d] = v[(size_t)(m / 2)];
    }
    int f = 0;
    for (int d = 1; d < dim; ++d)
        if (med[d] > med[f]) f = d;
    if (med[f] < 0.5 || med[f] > 2.0) return -1;
    for (int d = 0; d < dim; ++d)
        if (d != f && med[d] > 0.25) return -1;
    return f;
}

// Quantise each axis in units of the mean point spacing, with `sub`
// fractional bits.  The unit is the span over n^(1/dim) - 1/2 points and the
// offset 0.2 unit, so that floor() sends point i of an m-point lattice to i
// (i (1 + 1/(2m-2)) + 0.2 < i + 1) and also keeps cell-centred points
// jittered by up to +-0.3 spacing inside their own cell.  On such grids the
// integer parts are the grid indices, runs of 2^(k*dim) consecutive codes are
// aligned blocks and tiles have minimal halos; the fractional bits keep
// irregular meshes finely ordered.  `range`: the largest span in units, plus
// one.
void morton_units(int dim, int64_t n, const double* lo, const double* hi, double* unit, double* range)
{
    const double per_axis = std::max(2.0, std::pow((double)n, 1.0 / dim));
    *range = 1.0;
    for (int d = 0; d < dim; ++d) {
        const double span = hi[d] - lo[d];
        unit[d] = span > 0 ? span / (per_axis - 0.5) : 1.0;
        *range = std::max(*range, span / unit[d] + 1.0);
    }
}

// With a caller order that walks one axis (consecutive caller indices one
// spacing apart along it and fixed along the others, as in a structured grid
// stored row by row) the other axes' codes move up one bit, so a run of 512
// codes is a block long along that axis (32 x 16 in 2D, 16 x 8 x 4 instead of
// 8^3 in 3D) and a tile's points form longer caller-order runs.  (Longer
// blocks, 64 x 8 in 2D, grow the halo more than they gain.)  The fractional
// bits shrink until the codes fit 31 bits per axis in 2D, 21 in 3D.
MortonParams morton_params(int dim, const double* lo, const double* unit, double range, int fast)
{
    const int bits = (dim == 2) ? 31 : 21;
    MortonParams mp{};
    for (int d = 0; d < dim; ++d) {
        mp.lo[d] = lo[d];
        mp.unit[d] = unit[d];
    }
    mp.fast = fast;
    mp.shift_bits = fast >= 0 ? 1 : 0;
    int sub = 8;
    while (sub > 0 && std::ldexp(range, sub + mp.shift_bits) >= std::ldexp(1.0, bits)) --sub;
    mp.scale = std::ldexp(1.0, sub);
    mp.qmax = std::ldexp(1.0, bits - mp.shift_bits) - 1.0;
    return mp;
}

// The low bits that hold every code of these parameters: per axis the
// quantised value stays below (range + 0.2) scale, shifted by shift_bits.
int morton_key_bits(int dim, const MortonParams& mp, double range)
{
    const double top = std::min(mp.qmax + 1.0, std::ceil((range + 0.2) * mp.scale) + 1.0) * std::ldexp(1.0, mp.shift_bits);
    int b = 1;
    while (b < 64 && std::ldexp(1.0, b) < top) ++b;
    return std::min(64, dim * b);
}

uint64_t morton_code(int dim, const MortonParams& mp, const double* xi)
{
    uint64_t code = 0;
    for (int d = 0; d < dim; ++d) {
        const double t = std::floor(((xi[d] - mp.lo[d]) / mp.unit[d] + 0.2) * mp.scale);
        uint64_t q = (uint64_t)std::min(mp.qmax, std::max(0.0, t));
        if (mp.fast >= 0 && d != mp.fast) q <<= mp.shift_bits;
        code |= (dim == 2 ? spread2(q) : spread3(q)) << d;
    }
    return code;
}

}  // namespace

namespace {

// Common part of the two mesh constructors: the Morton order of the points,
// the stencil (from `stencil`, given the Morton permutation and its inverse,
// returning the CSR over Morton positions), the tiles and the upload.
template <typename StencilFn>
ftle_mesh_t build_mesh(int dim, int64_t n, const void* coords, ftle_dtype dtype, unsigned flags, int tile_log2,
                       const std::vector<double>& xd, StencilFn&& stencil)
{
    const bool f64 = dtype == FTLE_F64;
    std::unique_ptr<ftle_mesh_s> m(new ftle_mesh_s);
    m->dim = dim;
    m->n = n;
    m->dtype = dtype;
    m->flags = flags;
    m->host_only = (flags & FTLE_HOST_ONLY) != 0;
    m->tile_points = tile_log2 ? (1 << tile_log2) : 512;
    // launch shapes measured best on MI355X for 512-point tiles: two points
    // per lane in 2D, one in 3D (whose per-lane registers cap occupancy)
    m->fwd_block = (dim == 2) ? 256 : 512;
    m->bwd_block = (dim == 2) ? 256 : 512;
    // Morton order: quantise to the bounding box, interleave, stable sort
    m->perm.resize(n);
    for (int64_t i = 0; i < n; ++i) m->perm[i] = (int32_t)i;
    if (!(flags & FTLE_NO_REORDER) && n > 1) {
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t i = 0; i < n; ++i)
            for (int d = 0; d < dim; ++d) {
                lo[d] = std::min(lo[d], xd[i * dim + d]);
                hi[d] = std::max(hi[d], xd[i * dim + d]);
            }
        double unit[3] = {1, 1, 1}, range = 1.0;
        morton_units(dim, n, lo, hi, unit, &range);
        int64_t ms = 0, stride = 0;
        order_sample(n, &ms, &stride);
        std::vector<double> pairs((size_t)ms * 2 * dim);
        for (int64_t k = 0; k < ms; ++k)
            for (int d = 0; d < 2 * dim; ++d) pairs[(size_t)k * 2 * dim + d] = xd[(size_t)k * stride * dim + d];
        const MortonParams mp = morton_params(dim, lo, unit, range, order_axis_from_pairs(dim, ms, pairs.data(), unit));
        std::vector<uint64_t> key(n);
        parallel_for(n, [&](int64_t b, int64_t e, int) {
            for (int64_t i = b; i < e; ++i) key[i] = morton_code(dim, mp, &xd[(size_t)i * dim]);
        });
        radix_sort_pairs(key, m->perm);
    }
    std::vector<int32_t> inv(n);
    for (int64_t r = 0; r < n; ++r) inv[m->perm[r]] = (int32_t)r;

    m->csr = stencil(m->perm, inv);
    m->nnz = (int64_t)m->csr.col.size();
    Csr tr = transpose(m->csr, n);
    m->symmetric = csr_equal(tr, m->csr);
    m->fwd = build_tiles(dim, f64, n, m->tile_points, m->csr, m->perm);
    if (!m->symmetric) m->bwd = build_tiles(dim, f64, n, m->tile_points, tr, m->perm);
    // coordinates in user order, stored in the mesh dtype
    m->x_user.resize((size_t)n * dim * m->elem());
    std::memcpy(m->x_user.data(), coords, m->x_user.size());
    std::vector<unsigned char> minv;
    if (dim == 3 && !m->host_only) minv = normal_inverse3(m->csr, m->perm, xd, f64);

    if (!m->host_only) {
        int dev = 0;
        check_hip(hipGetDevice(&dev), "hipGetDevice (no usable GPU?)");
        m->device = dev;
        try {
            upload_tiles(m->fwd);
            if (!minv.empty()) m->fwd.d_minv = dev_upload(minv.data(), minv.size());
            if (!m->symmetric) upload_tiles(m->bwd);
            m->d_x = dev_upload(m->x_user.data(), m->x_user.size());
            m->d_hits = static_cast<unsigned long long*>(dev_upload(nullptr, sizeof(unsigned long long)));
            check_hip(hipMemset(m->d_hits, 0, sizeof(unsigned long long)), "hipMemset");
            check_hip(hipEventCreateWithFlags(&m->work_done, hipEventDisableTiming), "hipEventCreate");
        } catch (...) {
            release_device(m.get());
            throw;
        }
    }
    return m.release();
}

// Shared validation of (dim, n_points, coords, dtype, flags); returns the
// coordinates as float64 and the tile exponent.
std::vector<double> checked_coords(int dim, int64_t n_points, const void* coords, ftle_dtype dtype, unsigned flags,
                                   unsigned allowed, int* tile_log2)
{
    if (dim != 2 && dim != 3) fail(FTLE_ERR_INVALID_ARG, "dim must be 2 or 3");
    if (dtype != FTLE_F32 && dtype != FTLE_F64) fail(FTLE_ERR_INVALID_ARG, "unknown dtype");
    if (n_points < 1) fail(FTLE_ERR_INVALID_ARG, "n_points must be >= 1");
    if (n_points > INT32_MAX) fail(FTLE_ERR_UNSUPPORTED, "n_points > 2^31-1");
    if (!coords) fail(FTLE_ERR_INVALID_ARG, "coords is NULL");
    if (flags & ~allowed) fail(FTLE_ERR_INVALID_ARG, "unknown flag bits");
    *tile_log2 = (int)((flags >> 8) & 0xff);
    if (*tile_log2 != 0 && (*tile_log2 < 5 || *tile_log2 > 11))
        fail(FTLE_ERR_INVALID_ARG, "FTLE_TILE(k) needs 5 <= k <= 11");
    const bool f64 = dtype == FTLE_F64;
    std::vector<double> xd((size_t)n_points * dim);
    for (int64_t i = 0; i < n_points * dim; ++i) {
        const double v = f64 ? static_cast<const double*>(coords)[i] : (double)static_cast<const float*>(coords)[i];
        if (!std::isfinite(v)) fail(FTLE_ERR_INVALID_ARG, "coordinate " + std::to_string(i / dim) + " is not finite");
        xd[i] = v;
    }
    return xd;
}

// ---------------------------------------------------------------------------
// The mesh build on the device (ftle_create_mesh_device): the same steps and
// the same result as build_mesh with the one-ring stencil, with every pass
// over points, cells or stencil entries in the kernels of ftle_meshbuild.hip
// and ftle_neighbours.hip.  The host keeps the control: the bounding box
// reduction over workgroups, the caller-order test on a 2^16-pair sample, the
// tile-size halving and the record offsets, each from a small download.
// ---------------------------------------------------------------------------

// A device allocation freed on scope exit unless released.
struct DevBuf {
    void* p = nullptr;
    DevBuf() = default;
    explicit DevBuf(size_t bytes) { check_hip(hipMalloc(&p, bytes ? bytes : 16), "hipMalloc"); }
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf& operator=(DevBuf&& o) noexcept
    {
        std::swap(p, o.p);
        return *this;
    }
    template <typename T>
    T* as() const
    {
        return static_cast<T*>(p);
    }
    void reset()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
    }
    void* release()
    {
        void* q = p;
        p = nullptr;
        return q;
    }
};

// The build's temporaries, carved from one allocation: a hipMalloc / hipFree
// pair per temporary array cost more than the kernels that use them.
// Scratch device memory of the device mesh builds, kept per device between
// builds and grown when a build needs more, so that a build does not pay for
// allocating and releasing its temporaries each time.  One build at a time
// holds it (a concurrent build on the same device takes memory of its own);
// ftle_release_cached_memory frees it.  Never freed by a static destructor:
// the runtime may be gone by then, and the process's end returns it anyway.
struct BuildScratch {
    std::mutex m;
    void* p = nullptr;
    size_t bytes = 0;
    bool busy = false;
};
constexpr int kMaxCachedDevices = 64;
BuildScratch g_build_scratch[kMaxCachedDevices];

class ScratchLease {
  public:
    ScratchLease(size_t need, hipStream_t s) : s_(s)
    {
        int dev = -1;
        check_hip(hipGetDevice(&dev), "hipGetDevice");
        if (dev >= 0 && dev < kMaxCachedDevices) {
            BuildScratch& c = g_build_scratch[dev];
            std::lock_guard<std::mutex> lk(c.m);
            if (!c.busy) {
                if (c.bytes < need) {
                    if (c.p) (void)hipFree(c.p);
                    c.p = nullptr;
                    c.bytes = 0;
                    check_hip(hipMalloc(&c.p, need ? need : 16), "hipMalloc (mesh build scratch)");
                    c.bytes = need;
                }
                c.busy = true;
                cache_ = &c;
                p_ = c.p;
                return;
            }
        }
        own_ = DevBuf(need);
        p_ = own_.p;
    }
    ~ScratchLease()
    {
        if (!cache_) return;
        (void)hipStreamSynchronize(s_);   // the build's kernels are done with it (also after a failure)
        std::lock_guard<std::mutex> lk(cache_->m);
        cache_->busy = false;
    }
    ScratchLease(const ScratchLease&) = delete;
    ScratchLease& operator=(const ScratchLease&) = delete;
    void* get() const { return p_; }

  private:
    hipStream_t s_;
    BuildScratch* cache_ = nullptr;
    DevBuf own_;
    void* p_ = nullptr;
};

struct Arena {
    unsigned char* base = nullptr;
    size_t size = 0, at = 0;
    static size_t round(size_t b) { return ((b ? b : 1) + 255) & ~(size_t)255; }   // every array takes >= 256 B
    template <typename T>
    T* take(size_t bytes)
    {
        const size_t b = round(bytes);
        if (at + b > size) fail(FTLE_ERR_DEVICE, "mesh build: temporary arena exhausted");
        void* p = base + at;
        at += b;
        return static_cast<T*>(p);
    }
};

void to_host(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    if (!bytes) return;
    check_hip(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
}

void to_device(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    if (!bytes) return;
    check_hip(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
}

struct Extent {
    int64_t b, e;
    uint32_t H, nw;
};

// Tile extents as build_tiles cuts them: nominal chunks of tile_points,
// halved until they fit; the halo and word counts of all candidates of one
// generation come from one launch.
std::vector<Extent> device_extents(int dim, bool f64, int64_t n, int tile_points, const int64_t* row_ptr,
                                   const int32_t* col, const int32_t* perm, Arena& arena, hipStream_t s)
{
    std::vector<std::pair<int64_t, int64_t>> todo, next;
    for (int64_t b = 0; b < n; b += tile_points) todo.push_back({b, std::min<int64_t>(n, b + tile_points)});
    std::vector<Extent> out;
    std::vector<int64_t> ranges;
    std::vector<uint32_t> hw;
    while (!todo.empty()) {
        ranges.resize(2 * todo.size());
        for (size_t i = 0; i < todo.size(); ++i) {
            ranges[2 * i] = todo[i].first;
            ranges[2 * i + 1] = todo[i].second;
        }
        const size_t mark = arena.at;
        int64_t* d_ranges = arena.take<int64_t>(ranges.size() * 8);
        uint32_t* d_hw = arena.take<uint32_t>(todo.size() * 8);
        to_device(d_ranges, ranges.data(), ranges.size() * 8, s);
        check_hip(mb_tile_extent(row_ptr, col, d_ranges, (int64_t)todo.size(), d_hw, s), "tile extent kernel");
        hw.resize(2 * todo.size());
        to_host(hw.data(), d_hw, hw.size() * 4, s);
        arena.at = mark;
        next.clear();
        for (size_t i = 0; i < todo.size(); ++i) {
            const auto [b, e] = todo[i];
            if (tile_fits(dim, f64, e - b, hw[2 * i], hw[2 * i + 1])) {
                out.push_back({b, e, hw[2 * i], hw[2 * i + 1]});
            } else if (e - b == 1) {
                int64_t rp[2];
                int32_t user = 0;
                to_host(rp, row_ptr + b, sizeof rp, s);
                to_host(&user, perm + b, sizeof user, s);
                fail(FTLE_ERR_UNSUPPORTED, "point " + std::to_string(user) + " has " + std::to_string(rp[1] - rp[0]) +
                                               " neighbours, more than one tile holds");
            } else {
                const int64_t m = b + (e - b) / 2;
                next.push_back({b, m});
                next.push_back({m, e});
            }
        }
        todo.swap(next);
    }
    std::sort(out.begin(), out.end(), [](const Extent& u, const Extent& v) { return u.b < v.b; });
    return out;
}

// The records of the tiles `ext` (two passes: sizes and rows, then the
// records at their offsets), into ts (meta on host and device, records on
// the device).
void device_tiles(const std::vector<Extent>& ext, const int64_t* row_ptr, const int32_t* col, const int32_t* perm,
                  TileSet& ts, Arena& arena, hipStream_t s)
{
    const size_t T = ext.size();
    std::vector<int64_t> ranges(2 * T), row_base(T);
    int64_t entries = 0;
    for (size_t t = 0; t < T; ++t) {
        ranges[2 * t] = ext[t].b;
        ranges[2 * t + 1] = ext[t].e;
        row_base[t] = entries;
        entries += 3 * (int64_t)ext[t].nw;
    }
    // the row buffer from the arena when it fits there, else its own allocation
    const size_t need = Arena::round(T * 16) * 2 + Arena::round(T * 8) + Arena::round((size_t)entries * 2);
    DevBuf own;
    Arena local;
    if (arena.at + need > arena.size) {
        own = DevBuf(need);
        local.base = static_cast<unsigned char*>(own.p);
        local.size = need;
    }
    Arena& a = own.p ? local : arena;
    int64_t* d_ranges = a.take<int64_t>(T * 16);
    int64_t* d_base = a.take<int64_t>(T * 8);
    uint32_t* d_counts = a.take<uint32_t>(T * 16);
    uint16_t* d_rows = a.take<uint16_t>((size_t)entries * 2);
    to_device(d_ranges, ranges.data(), T * 16, s);
    to_device(d_base, row_base.data(), T * 8, s);
    const uint32_t* uperm = reinterpret_cast<const uint32_t*>(perm);
    check_hip(mb_tile_record(false, row_ptr, col, uperm, d_ranges, (int64_t)T, d_base, d_rows, d_counts, nullptr,
                             nullptr, s),
              "tile record kernel (sizes)");
    std::vector<uint32_t> counts(4 * T);
    to_host(counts.data(), d_counts, T * 16, s);
    ts.meta.resize(T);
    uint64_t off = 0;   // in 16-byte units
    for (size_t t = 0; t < T; ++t) {
        const uint32_t* c = &counts[4 * t];
        if (c[0] > (uint32_t)kMaxTileWords || c[3] != ext[t].nw)
            fail(FTLE_ERR_DEVICE, "tile " + std::to_string(t) + ": record sizes disagree with its extent");
        if (off > UINT32_MAX) fail(FTLE_ERR_UNSUPPORTED, "tile records exceed 64 GiB");
        TileMeta& m = ts.meta[t];
        m.rec_off = (uint32_t)off;
        m.P = (uint16_t)(ext[t].e - ext[t].b);
        m.H = (uint16_t)ext[t].H;
        m.nw = (uint16_t)c[0];
        m.nr = (uint16_t)c[1];
        m.nx = (uint16_t)c[2];
        m.nwf = (uint16_t)c[3];
        const uint32_t bytes = rec_layout(m).bytes;
        off += bytes / 16;
        ts.max_staged = std::max(ts.max_staged, (int)(m.P + m.H));
        ts.max_rec = std::max(ts.max_rec, (int)bytes);
        ts.max_P = std::max(ts.max_P, (int)m.P);
        ts.halo_total += m.H;
    }
    ts.rec_bytes = (int64_t)off * 16;
    ts.d_meta = dev_upload(ts.meta.data(), T * sizeof(TileMeta));
    ts.d_rec = dev_upload(nullptr, (size_t)ts.rec_bytes);
    check_hip(hipMemsetAsync(ts.d_rec, 0, (size_t)ts.rec_bytes, s), "hipMemsetAsync");
    check_hip(mb_tile_record(true, row_ptr, col, uperm, d_ranges, (int64_t)T, d_base, d_rows, nullptr,
                             static_cast<const TileMeta*>(ts.d_meta), static_cast<unsigned char*>(ts.d_rec), s),
              "tile record kernel (records)");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
}

// The skeleton shared by both device builds: the mesh's coordinates, the
// bounds, the Morton order; then `stencil(m, perm, arena)` sets the forward
// stencil over Morton positions (m->d_row_ptr, m->d_col, m->nnz); then, unless
// the stencil is known to be symmetric, its transpose is formed and compared
// (the host build's test); then the tiles (and the transpose's tiles when it
// differs), the 3D inverse normal matrices and the mesh's counters.
// stencil_bytes: the arena the stencil step needs.
template <typename Stencil>
ftle_mesh_t build_device(int dim, int64_t n, const void* coords, ftle_dtype dtype, unsigned flags, int tile_log2,
                         size_t stencil_bytes, bool known_symmetric, hipStream_t s, Stencil&& stencil)
{
    const bool f64 = dtype == FTLE_F64;
    const size_t eb = f64 ? 8 : 4;
    std::unique_ptr<ftle_mesh_s> m(new ftle_mesh_s);
    m->dim = dim;
    m->n = n;
    m->dtype = dtype;
    m->flags = flags;
    m->device_built = true;
    m->tile_points = tile_log2 ? (1 << tile_log2) : 512;
    m->fwd_block = (dim == 2) ? 256 : 512;
    m->bwd_block = (dim == 2) ? 256 : 512;
    check_hip(hipGetDevice(&m->device), "hipGetDevice (no usable GPU?)");
    struct Release {
        ftle_mesh_s* m;
        ~Release()
        {
            if (m) release_device(m);
        }
    } guard{m.get()};

    // One arena for every temporary: the bounds and the sort first, then the
    // stencil step's arrays, later the tile passes.
    const int nb = (int)std::min<int64_t>(1024, (n + 255) / 256);
    int64_t ms = 0, stride = 0;
    order_sample(n, &ms, &stride);
    const size_t phase_sort = Arena::round((size_t)nb * 2 * dim * 8 + 8) + Arena::round((size_t)ms * 2 * dim * 8) +
                              Arena::round((size_t)n * 8) + Arena::round(mb_sort_scratch_bytes(n));
    ScratchLease arena_buf(std::max(phase_sort, stencil_bytes), s);
    Arena arena;
    arena.base = static_cast<unsigned char*>(arena_buf.get());
    arena.size = std::max(phase_sort, stencil_bytes);

    // the mesh's own copy of the coordinates; bounds and finiteness
    m->d_x = dev_upload(nullptr, (size_t)n * dim * eb);
    check_hip(hipMemcpyAsync(m->d_x, coords, (size_t)n * dim * eb, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
    double* part = arena.take<double>((size_t)nb * 2 * dim * 8 + 8);
    unsigned long long* first_bad = reinterpret_cast<unsigned long long*>(part + (size_t)nb * 2 * dim);
    check_hip(hipMemsetAsync(first_bad, 0xff, 8, s), "hipMemsetAsync");
    check_hip(mb_bbox(dim, f64, m->d_x, n, part, nb, first_bad, s), "bounds kernel");
    std::vector<double> hp((size_t)nb * 2 * dim + 1);
    to_host(hp.data(), part, hp.size() * 8, s);
    unsigned long long bad = 0;
    std::memcpy(&bad, &hp.back(), 8);
    if (bad != ~0ull) fail(FTLE_ERR_INVALID_ARG, "coordinate " + std::to_string(bad) + " is not finite");

    // Morton order
    m->d_perm = static_cast<int32_t*>(dev_upload(nullptr, (size_t)n * 4));
    uint32_t* perm = reinterpret_cast<uint32_t*>(m->d_perm);
    if (!(flags & FTLE_NO_REORDER) && n > 1) {
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int b = 0; b < nb; ++b)
            for (int d = 0; d < dim; ++d) {
                lo[d] = std::min(lo[d], hp[(size_t)b * 2 * dim + d]);
                hi[d] = std::max(hi[d], hp[(size_t)b * 2 * dim + dim + d]);
            }
        double unit[3] = {1, 1, 1}, range = 1.0;
        morton_units(dim, n, lo, hi, unit, &range);
        std::vector<double> pairs((size_t)ms * 2 * dim);
        if (ms) {
            double* d_pairs = arena.take<double>(pairs.size() * 8);
            check_hip(mb_gather_pairs(dim, f64, m->d_x, ms, stride, d_pairs, s), "sample kernel");
            to_host(pairs.data(), d_pairs, pairs.size() * 8, s);
        }
        const MortonParams mp = morton_params(dim, lo, unit, range, order_axis_from_pairs(dim, ms, pairs.data(), unit));
        uint64_t* key = arena.take<uint64_t>((size_t)n * 8);
        void* scratch = arena.take<void>(mb_sort_scratch_bytes(n));
        check_hip(mb_morton(dim, f64, m->d_x, n, mp, key, perm, s), "Morton kernel");
        uint32_t* sorted = nullptr;
        check_hip(mb_sort(key, perm, n, morton_key_bits(dim, mp, range), scratch, &sorted, s), "radix sort");
        if (sorted != perm)
            check_hip(hipMemcpyAsync(perm, sorted, (size_t)n * 4, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
    } else {
        check_hip(mb_iota(perm, n, s), "iota kernel");
    }

    // the stencil over Morton positions
    arena.at = 0;
    stencil(m.get(), perm, arena);
    arena.at = 0;
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    const int64_t nnz = m->nnz;

    // its transpose, when the stencil is not known to be symmetric
    DevBuf t_rp, t_col;
    m->symmetric = true;
    if (!known_symmetric) {
        DevBuf cnt(((size_t)n + 1) * 4), partial(scan_partial_bytes(n + 1) + 16), flag(16);
        t_rp = DevBuf(((size_t)n + 1) * 8);
        t_col = DevBuf((size_t)nnz * 4);
        check_hip(hipMemsetAsync(cnt.p, 0, ((size_t)n + 1) * 4, s), "hipMemsetAsync");
        check_hip(mb_transpose_count(m->d_col, nnz, cnt.as<uint32_t>(), s), "transpose kernel");
        check_hip(scan_exclusive_to_i64(cnt.as<uint32_t>(), n, t_rp.as<int64_t>(), partial.as<int64_t>(), s), "scan");
        check_hip(hipMemsetAsync(cnt.p, 0, ((size_t)n + 1) * 4, s), "hipMemsetAsync");
        check_hip(mb_transpose_fill(m->d_row_ptr, m->d_col, n, t_rp.as<int64_t>(), cnt.as<uint32_t>(),
                                    t_col.as<int32_t>(), s),
                  "transpose kernel");
        check_hip(hipMemsetAsync(flag.p, 0, 4, s), "hipMemsetAsync");
        check_hip(mb_csr_compare(m->d_row_ptr, m->d_col, t_rp.as<int64_t>(), t_col.as<int32_t>(), n, nnz,
                                 flag.as<int>(), s),
                  "compare kernel");
        int differ = 0;
        to_host(&differ, flag.p, 4, s);
        m->symmetric = differ == 0;
    }

    const std::vector<Extent> ext =
        device_extents(dim, f64, n, m->tile_points, m->d_row_ptr, m->d_col, m->d_perm, arena, s);
    device_tiles(ext, m->d_row_ptr, m->d_col, m->d_perm, m->fwd, arena, s);
    if (!m->symmetric) {
        const std::vector<Extent> text =
            device_extents(dim, f64, n, m->tile_points, t_rp.as<int64_t>(), t_col.as<int32_t>(), m->d_perm, arena, s);
        device_tiles(text, t_rp.as<int64_t>(), t_col.as<int32_t>(), m->d_perm, m->bwd, arena, s);
    }
    if (dim == 3) {
        m->fwd.d_minv = dev_upload(nullptr, (size_t)n * 6 * eb);
        check_hip(mb_normal_inverse(f64, m->d_row_ptr, m->d_col, perm, m->d_x, n, m->fwd.d_minv, s),
                  "normal matrix kernel");
    }
    m->d_hits = static_cast<unsigned long long*>(dev_upload(nullptr, sizeof(unsigned long long)));
    check_hip(hipMemsetAsync(m->d_hits, 0, sizeof(unsigned long long), s), "hipMemsetAsync");
    check_hip(hipEventCreateWithFlags(&m->work_done, hipEventDisableTiming), "hipEventCreate");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
    guard.m = nullptr;
    return m.release();
}

// From device cells: the cells relabelled and checked, the one-ring stencil,
// and with FTLE_STENCIL_AXIS the axis stencil from it.
ftle_mesh_t build_mesh_device(int dim, int64_t n, const void* coords, ftle_dtype dtype, int64_t n_cells,
                              const int32_t* cells, unsigned flags, int tile_log2, hipStream_t s)
{
    const int k = dim + 1;
    const bool axis = (flags & FTLE_STENCIL_AXIS) != 0;
    const size_t mc_bytes = Arena::round((size_t)n_cells * k * 4);
    const size_t need = mc_bytes + std::max(Arena::round((size_t)n * 4) + Arena::round(16),
                                            Arena::round(ring1_workspace_bytes(dim, n, n_cells)));
    return build_device(dim, n, coords, dtype, flags, tile_log2, need, !axis, s,
                        [&](ftle_mesh_s* m, const uint32_t* perm, Arena& arena) {
        const bool f64 = dtype == FTLE_F64;
        int32_t* mc = arena.take<int32_t>((size_t)n_cells * k * 4);
        const size_t phase_base = arena.at;
        {
            int32_t* inv = arena.take<int32_t>((size_t)n * 4);
            unsigned char* flag = arena.take<unsigned char>(16);
            check_hip(hipMemsetAsync(flag, 0xff, 8, s), "hipMemsetAsync");
            check_hip(hipMemsetAsync(flag + 8, 0, 4, s), "hipMemsetAsync");
            check_hip(mb_invert(perm, n, inv, s), "inverse permutation kernel");
            check_hip(mb_relabel(dim, cells, n_cells, n, inv, mc, reinterpret_cast<int*>(flag + 8),
                                 reinterpret_cast<unsigned long long*>(flag), s),
                      "cell relabel kernel");
            unsigned long long hf[2] = {0, 0};
            to_host(hf, flag, 12, s);
            if (hf[1] & 0xffffffffu) {
                const int64_t c = (int64_t)hf[0];
                int32_t v[4] = {0, 0, 0, 0};
                to_host(v, cells + c * k, (size_t)k * 4, s);
                int kind = 0;   // the first fault in vertex order, as the host build reports it
                for (int a = 0; a < k && !kind; ++a) {
                    if (v[a] < 0 || v[a] >= n) kind = 1;
                    for (int q = 0; q < a && !kind; ++q)
                        if (v[q] == v[a]) kind = 2;
                }
                fail(FTLE_ERR_BAD_MESH, std::string(kind == 1 ? "cell index out of range" : "repeated vertex") +
                                            " in cell " + std::to_string(c));
            }
        }
        arena.at = phase_base;
        // the one-ring stencil: the mesh's own (RING1), or the input of the axis stencil
        DevBuf ring_rp, ring_col;
        int64_t* rp = nullptr;
        if (axis) {
            ring_rp = DevBuf(((size_t)n + 1) * 8);
            rp = ring_rp.as<int64_t>();
        } else {
            m->d_row_ptr = static_cast<int64_t*>(dev_upload(nullptr, ((size_t)n + 1) * 8));
            rp = m->d_row_ptr;
        }
        int64_t nnz = 0;
        int32_t* colp = nullptr;
        {
            void* ws = arena.take<void>(ring1_workspace_bytes(dim, n, n_cells));
            int bad_mesh = 0, too_long = 0;
            check_hip(ring1_build(dim, mc, n_cells, n, ws, rp, nullptr, 0, &nnz, &bad_mesh, &too_long, s),
                      "one-ring stencil kernels");
            if (bad_mesh) fail(FTLE_ERR_DEVICE, "relabelled cells failed the stencil's range check");
            if (too_long) fail(FTLE_ERR_UNSUPPORTED, "a point's incident cells list more than 4096 points");
            if (nnz > INT32_MAX) fail(FTLE_ERR_UNSUPPORTED, "stencil has more than 2^31-1 entries");
            if (axis) {
                ring_col = DevBuf((size_t)nnz * 4);
                colp = ring_col.as<int32_t>();
            } else {
                m->d_col = static_cast<int32_t*>(dev_upload(nullptr, (size_t)nnz * 4));
                colp = m->d_col;
            }
            if (nnz) check_hip(ring1_write(dim, mc, n_cells, n, ws, rp, colp, s), "one-ring stencil kernels");
            check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
        }
        if (axis) {
            // the axis stencil from the one-ring rows
            DevBuf slots((size_t)n * 2 * dim * 4), cnt(((size_t)n + 1) * 4), partial(scan_partial_bytes(n + 1) + 16);
            check_hip(mb_axis_stencil(dim, f64, m->d_x, perm, rp, colp, n, slots.as<int32_t>(), cnt.as<uint32_t>(),
                                      s),
                      "axis stencil kernel");
            m->d_row_ptr = static_cast<int64_t*>(dev_upload(nullptr, ((size_t)n + 1) * 8));
            check_hip(scan_exclusive_to_i64(cnt.as<uint32_t>(), n, m->d_row_ptr, partial.as<int64_t>(), s), "scan");
            to_host(&nnz, m->d_row_ptr + n, 8, s);
            m->d_col = static_cast<int32_t*>(dev_upload(nullptr, (size_t)nnz * 4));
            check_hip(mb_axis_fill(dim, slots.as<int32_t>(), m->d_row_ptr, n, m->d_col, s), "axis stencil kernel");
            check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
        }
        m->nnz = nnz;
    });
}

// From a caller's device CSR over caller indices (rows in any order, -1 and
// self entries dropped, repeats kept): rows moved to Morton positions and
// sorted, as ftle_create_mesh_from_csr does on the host.
ftle_mesh_t build_mesh_device_csr(int dim, int64_t n, const void* coords, ftle_dtype dtype, const int64_t* row_ptr,
                                  const int32_t* col, int64_t nnz_in, unsigned flags, int tile_log2, hipStream_t s)
{
    const size_t need = Arena::round((size_t)n * 4) * 2 + Arena::round(scan_partial_bytes(n + 1)) + Arena::round(32);
    return build_device(dim, n, coords, dtype, flags, tile_log2, need, false, s,
                        [&](ftle_mesh_s* m, const uint32_t* perm, Arena& arena) {
        int32_t* inv = arena.take<int32_t>((size_t)n * 4);
        uint32_t* cnt = arena.take<uint32_t>((size_t)n * 4);
        int64_t* partial = arena.take<int64_t>(scan_partial_bytes(n + 1));
        unsigned long long* err = arena.take<unsigned long long>(32);   // [0]: lowest bad row, [1]: lowest bad entry
        check_hip(hipMemsetAsync(err, 0xff, 16, s), "hipMemsetAsync");
        check_hip(mb_invert(perm, n, inv, s), "inverse permutation kernel");
        check_hip(mb_csr_in_count(row_ptr, col, n, nnz_in, perm, cnt, err, s), "stencil count kernel");
        unsigned long long he[2] = {0, 0};
        to_host(he, err, 16, s);
        if (he[0] != ~0ull) {
            if (he[0] == 0) fail(FTLE_ERR_BAD_MESH, "row_ptr[0] must be 0");
            fail(FTLE_ERR_BAD_MESH, "row_ptr decreases at row " + std::to_string(he[0] - 1));
        }
        if (he[1] != ~0ull) fail(FTLE_ERR_BAD_MESH, "col[" + std::to_string(he[1]) + "] out of range");
        m->d_row_ptr = static_cast<int64_t*>(dev_upload(nullptr, ((size_t)n + 1) * 8));
        check_hip(scan_exclusive_to_i64(cnt, n, m->d_row_ptr, partial, s), "scan");
        int64_t nnz = 0;
        to_host(&nnz, m->d_row_ptr + n, 8, s);
        if (nnz > INT32_MAX) fail(FTLE_ERR_UNSUPPORTED, "stencil has more than 2^31-1 entries");
        m->d_col = static_cast<int32_t*>(dev_upload(nullptr, (size_t)nnz * 4));
        check_hip(mb_csr_in_fill(row_ptr, col, n, perm, inv, m->d_row_ptr, m->d_col, s), "stencil fill kernel");
        check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
        m->nnz = nnz;
    });
}

}  // namespace

extern "C" {

ftle_status ftle_create_mesh(int dim, int64_t n_points, const void* coords, ftle_dtype dtype,
                             int64_t n_cells, const int32_t* cells, unsigned flags, ftle_mesh_t* out)
{
    return guarded([&] {
        if (!out) fail(FTLE_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        int tile_log2 = 0;
        const unsigned known = FTLE_STENCIL_AXIS | FTLE_NO_REORDER | FTLE_HOST_ONLY | FTLE_TILE(0xff);
        const std::vector<double> xd = checked_coords(dim, n_points, coords, dtype, flags, known, &tile_log2);
        if (n_cells < 0) fail(FTLE_ERR_INVALID_ARG, "n_cells < 0");
        if (n_cells > 0 && !cells) fail(FTLE_ERR_INVALID_ARG, "cells is NULL");
        const int64_t n = n_points;
        const int k = dim + 1;
        if (n_cells > INT64_MAX / k) fail(FTLE_ERR_INVALID_ARG, "n_cells too large");
        // validate cells
        std::atomic<int64_t> bad_cell{-1};
        std::atomic<int> bad_kind{0};
        parallel_for(n_cells, [&](int64_t b, int64_t e, int) {
            for (int64_t c = b; c < e && bad_cell.load(std::memory_order_relaxed) < 0; ++c) {
                for (int a = 0; a < k; ++a) {
                    const int32_t v = cells[c * k + a];
                    if (v < 0 || v >= n) {
                        bad_kind = 1;
                        bad_cell = c;
                        return;
                    }
                    for (int q = 0; q < a; ++q)
                        if (cells[c * k + q] == v) {
                            bad_kind = 2;
                            bad_cell = c;
                            return;
                        }
                }
            }
        });
        if (bad_cell >= 0)
            fail(FTLE_ERR_BAD_MESH, std::string(bad_kind == 1 ? "cell index out of range" : "repeated vertex") +
                                        " in cell " + std::to_string(bad_cell.load()));

        *out = build_mesh(dim, n, coords, dtype, flags, tile_log2, xd,
                          [&](const std::vector<int32_t>& perm, const std::vector<int32_t>& inv) {
                              // cells in Morton positions, then the stencil
                              std::vector<int32_t> mc((size_t)n_cells * k);
                              parallel_for(n_cells * k, [&](int64_t b, int64_t e, int) {
                                  for (int64_t i = b; i < e; ++i) mc[i] = inv[cells[i]];
                              });
                              Csr ring = build_ring1(dim, n, n_cells, mc);
                              mc.clear();
                              mc.shrink_to_fit();
                              if (!(flags & FTLE_STENCIL_AXIS)) return ring;
                              std::vector<double> xm((size_t)n * dim);
                              for (int64_t r = 0; r < n; ++r)
                                  for (int d = 0; d < dim; ++d) xm[r * dim + d] = xd[(size_t)perm[r] * dim + d];
                              return build_axis<double>(dim, n, ring, xm.data(), perm);
                          });
    });
}

ftle_status ftle_create_mesh_from_csr(int dim, int64_t n_points, const void* coords, ftle_dtype dtype,
                                      const int64_t* row_ptr, const int32_t* col, unsigned flags,
                                      ftle_mesh_t* out)
{
    return guarded([&] {
        if (!out) fail(FTLE_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        int tile_log2 = 0;
        const unsigned known = FTLE_NO_REORDER | FTLE_HOST_ONLY | FTLE_TILE(0xff);
        const std::vector<double> xd = checked_coords(dim, n_points, coords, dtype, flags, known, &tile_log2);
        if (!row_ptr) fail(FTLE_ERR_INVALID_ARG, "row_ptr is NULL");
        const int64_t n = n_points;
        if (row_ptr[0] != 0) fail(FTLE_ERR_BAD_MESH, "row_ptr[0] must be 0");
        for (int64_t i = 0; i < n; ++i)
            if (row_ptr[i + 1] < row_ptr[i]) fail(FTLE_ERR_BAD_MESH, "row_ptr decreases at row " + std::to_string(i));
        if (row_ptr[n] > 0 && !col) fail(FTLE_ERR_INVALID_ARG, "col is NULL");
        for (int64_t p = 0; p < row_ptr[n]; ++p)
            if (col[p] < -1 || col[p] >= n)
                fail(FTLE_ERR_BAD_MESH, "col[" + std::to_string(p) + "] out of range");
        *out = build_mesh(dim, n, coords, dtype, flags, tile_log2, xd,
                          [&](const std::vector<int32_t>& perm, const std::vector<int32_t>& inv) {
                              // rows in Morton positions, ascending; -1 and the point itself dropped
                              Csr c;
                              c.row_ptr.assign(n + 1, 0);
                              int64_t total = 0;
                              for (int64_t r = 0; r < n; ++r) {
                                  const int64_t i = perm[r];
                                  for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
                                      total += (col[p] >= 0 && col[p] != i) ? 1 : 0;
                                  if (total > INT32_MAX)
                                      fail(FTLE_ERR_UNSUPPORTED, "stencil has more than 2^31-1 entries");
                                  c.row_ptr[r + 1] = (int32_t)total;
                              }
                              c.col.resize(total);
                              parallel_for(n, [&](int64_t b, int64_t e, int) {
                                  for (int64_t r = b; r < e; ++r) {
                                      const int64_t i = perm[r];
                                      int32_t q = c.row_ptr[r];
                                      for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p)
                                          if (col[p] >= 0 && col[p] != i) c.col[q++] = inv[col[p]];
                                      std::sort(c.col.begin() + c.row_ptr[r], c.col.begin() + q);
                                  }
                              });
                              return c;
                          });
    });
}

ftle_status ftle_create_mesh_device_from_csr(int dim, int64_t n_points, const void* coords, ftle_dtype dtype,
                                             const int64_t* row_ptr, const int32_t* col, unsigned flags,
                                             ftle_stream_t stream, ftle_mesh_t* out)
{
    return guarded([&] {
        if (!out) fail(FTLE_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (dim != 2 && dim != 3) fail(FTLE_ERR_INVALID_ARG, "dim must be 2 or 3");
        if (dtype != FTLE_F32 && dtype != FTLE_F64) fail(FTLE_ERR_INVALID_ARG, "unknown dtype");
        if (n_points < 1) fail(FTLE_ERR_INVALID_ARG, "n_points must be >= 1");
        if (n_points > INT32_MAX) fail(FTLE_ERR_UNSUPPORTED, "n_points > 2^31-1");
        if (!coords) fail(FTLE_ERR_INVALID_ARG, "coords is NULL");
        if (!row_ptr) fail(FTLE_ERR_INVALID_ARG, "row_ptr is NULL");
        if (flags & FTLE_HOST_ONLY) fail(FTLE_ERR_UNSUPPORTED, "a device-built mesh lives on the device");
        if (flags & ~(unsigned)(FTLE_NO_REORDER | FTLE_HOST_ONLY | FTLE_TILE(0xff)))
            fail(FTLE_ERR_INVALID_ARG, "unknown flag bits");
        const int tile_log2 = (int)((flags >> 8) & 0xff);
        if (tile_log2 != 0 && (tile_log2 < 5 || tile_log2 > 11))
            fail(FTLE_ERR_INVALID_ARG, "FTLE_TILE(k) needs 5 <= k <= 11");
        const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        int64_t nnz_in = 0;
        to_host(&nnz_in, row_ptr + n_points, 8, s);
        if (nnz_in < 0) fail(FTLE_ERR_BAD_MESH, "row_ptr[n_points] < 0");
        if (nnz_in > 0 && !col) fail(FTLE_ERR_INVALID_ARG, "col is NULL");
        *out = build_mesh_device_csr(dim, n_points, coords, dtype, row_ptr, col, nnz_in, flags, tile_log2, s);
    });
}

ftle_status ftle_create_mesh_device(int dim, int64_t n_points, const void* coords, ftle_dtype dtype,
                                    int64_t n_cells, const int32_t* cells, unsigned flags, ftle_stream_t stream,
                                    ftle_mesh_t* out)
{
    return guarded([&] {
        if (!out) fail(FTLE_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (dim != 2 && dim != 3) fail(FTLE_ERR_INVALID_ARG, "dim must be 2 or 3");
        if (dtype != FTLE_F32 && dtype != FTLE_F64) fail(FTLE_ERR_INVALID_ARG, "unknown dtype");
        if (n_points < 1) fail(FTLE_ERR_INVALID_ARG, "n_points must be >= 1");
        if (n_points > INT32_MAX) fail(FTLE_ERR_UNSUPPORTED, "n_points > 2^31-1");
        if (!coords) fail(FTLE_ERR_INVALID_ARG, "coords is NULL");
        if (flags & FTLE_HOST_ONLY) fail(FTLE_ERR_UNSUPPORTED, "a device-built mesh lives on the device");
        if (flags & ~(unsigned)(FTLE_STENCIL_AXIS | FTLE_NO_REORDER | FTLE_HOST_ONLY | FTLE_TILE(0xff)))
            fail(FTLE_ERR_INVALID_ARG, "unknown flag bits");
        const int tile_log2 = (int)((flags >> 8) & 0xff);
        if (tile_log2 != 0 && (tile_log2 < 5 || tile_log2 > 11))
            fail(FTLE_ERR_INVALID_ARG, "FTLE_TILE(k) needs 5 <= k <= 11");
        if (n_cells < 0) fail(FTLE_ERR_INVALID_ARG, "n_cells < 0");
        if (n_cells > 0 && !cells) fail(FTLE_ERR_INVALID_ARG, "cells is NULL");
        if (n_cells > (int64_t)(UINT32_MAX / (unsigned)(dim + 1)))
            fail(FTLE_ERR_UNSUPPORTED, "n_cells (dim + 1) must stay below 2^32");
        const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        *out = build_mesh_device(dim, n_points, coords, dtype, n_cells, cells, flags, tile_log2, s);
    });
}

ftle_status ftle_mesh_info(ftle_mesh_t mesh, int* dim, int64_t* n_points, int64_t* nnz, int* dtype)
{
    return guarded([&] {
        check_mesh(mesh);
        if (dim) *dim = mesh->dim;
        if (n_points) *n_points = mesh->n;
        if (nnz) *nnz = mesh->nnz;
        if (dtype) *dtype = (int)mesh->dtype;
    });
}

ftle_status ftle_mesh_get_csr(ftle_mesh_t mesh, int32_t* row_ptr, int32_t* col, int32_t* perm)
{
    return guarded([&] {
        check_mesh(mesh);
        if (mesh->device_built) {
            // copied from the device (row offsets narrowed: nnz <= 2^31 - 1 is checked when built)
            DeviceScope scope(mesh->device);
            const int64_t n = mesh->n;
            if (row_ptr) {
                std::vector<int64_t> rp((size_t)n + 1);
                check_hip(hipMemcpy(rp.data(), mesh->d_row_ptr, rp.size() * 8, hipMemcpyDeviceToHost), "hipMemcpy");
                for (int64_t i = 0; i <= n; ++i) row_ptr[i] = (int32_t)rp[(size_t)i];
            }
            if (col && mesh->nnz)
                check_hip(hipMemcpy(col, mesh->d_col, (size_t)mesh->nnz * 4, hipMemcpyDeviceToHost), "hipMemcpy");
            if (perm) check_hip(hipMemcpy(perm, mesh->d_perm, (size_t)n * 4, hipMemcpyDeviceToHost), "hipMemcpy");
            return;
        }
        if (row_ptr) std::memcpy(row_ptr, mesh->csr.row_ptr.data(), mesh->csr.row_ptr.size() * 4);
        if (col) std::memcpy(col, mesh->csr.col.data(), mesh->csr.col.size() * 4);
        if (perm) std::memcpy(perm, mesh->perm.data(), mesh->perm.size() * 4);
    });
}

ftle_status ftle_mesh_tile_stats(ftle_mesh_t mesh, int64_t* n_tiles, int64_t* max_tile_points,
                                 int64_t* halo_entries, int64_t* record_bytes)
{
    return guarded([&] {
        check_mesh(mesh);
        if (n_tiles) *n_tiles = (int64_t)mesh->fwd.meta.size();
        if (max_tile_points) *max_tile_points = mesh->fwd.max_P;
        if (halo_entries) *halo_entries = mesh->fwd.halo_total;
        if (record_bytes) *record_bytes = mesh->fwd.rec_bytes + (int64_t)mesh->fwd.meta.size() * 16;
    });
}

ftle_status ftle_mesh_set_blocks(ftle_mesh_t mesh, int fwd_block, int adjoint_block)
{
    return guarded([&] {
        check_mesh(mesh);
        for (int b : {fwd_block, adjoint_block})
            if (b != 0 && !supported_block(b)) fail(FTLE_ERR_INVALID_ARG, "block sizes must be 128, 256 or 512");
        if (fwd_block) mesh->fwd_block = fwd_block;
        if (adjoint_block) mesh->bwd_block = adjoint_block;
    });
}

ftle_status ftle_mesh_get_blocks(ftle_mesh_t mesh, int* fwd_block, int* adjoint_block)
{
    return guarded([&] {
        check_mesh(mesh);
        if (fwd_block) *fwd_block = mesh->fwd_block;
        if (adjoint_block) *adjoint_block = mesh->bwd_block;
    });
}

ftle_status ftle_mesh_get_tiles(ftle_mesh_t mesh, int adjoint, int64_t* n_tiles, int64_t* record_bytes,
                                void* meta, void* records)
{
    return guarded([&] {
        check_mesh(mesh);
        const TileSet& ts = adjoint ? mesh->adj_tiles() : mesh->fwd;
        if (n_tiles) *n_tiles = (int64_t)ts.meta.size();
        if (record_bytes) *record_bytes = ts.rec_bytes;
        if (meta) std::memcpy(meta, ts.meta.data(), ts.meta.size() * sizeof(TileMeta));
        if (records && ts.rec_bytes) {
            if (mesh->device_built) {
                DeviceScope scope(mesh->device);
                check_hip(hipMemcpy(records, ts.d_rec, (size_t)ts.rec_bytes, hipMemcpyDeviceToHost), "hipMemcpy");
            } else {
                std::memcpy(records, ts.rec.data(), (size_t)ts.rec_bytes);
            }
        }
    });
}

ftle_status ftle_forward(ftle_mesh_t mesh, const void* flow, ftle_dtype dtype, double T, void* out,
                         ftle_stream_t stream)
{
    return guarded([&] {
        check_mesh(mesh);
        check_dtype(mesh, dtype);
        check_T(T);
        if (!flow || !out) fail(FTLE_ERR_INVALID_ARG, "flow or out is NULL");
        need_device(mesh);
        DeviceScope ds(mesh->device);
        check_hip(launch_forward(mesh->dim, mesh->f64(), mesh->fwd.dev(), mesh->d_x, flow, 0.5 / std::fabs(T),
                                 out, nullptr, false, mesh->n, eig_tau(), mesh->d_hits, mesh->fwd_block,
                                 static_cast<hipStream_t>(stream)),
                  "forward launch");
    });
}

namespace {
void check_f16_mesh(ftle_mesh_t mesh)
{
    check_mesh(mesh);
    if (mesh->dim != 2 || mesh->f64())
        fail(FTLE_ERR_UNSUPPORTED, "half-precision flow maps are for 2D float32 meshes");
    if (mesh->n >= ((int64_t)1 << 29)) fail(FTLE_ERR_UNSUPPORTED, "mesh too large for half-precision flow maps");
}
}  // namespace

ftle_status ftle_encode_flow_f16(ftle_mesh_t mesh, const void* flow, void* delta, ftle_stream_t stream)
{
    return guarded([&] {
        check_f16_mesh(mesh);
        if (!flow || !delta) fail(FTLE_ERR_INVALID_ARG, "flow or delta is NULL");
        need_device(mesh);
        DeviceScope ds(mesh->device);
        check_hip(launch_encode_f16(mesh->d_x, flow, delta, mesh->n, static_cast<hipStream_t>(stream)),
                  "encode launch");
    });
}

ftle_status ftle_forward_f16(ftle_mesh_t mesh, const void* delta, double T, void* out, ftle_stream_t stream)
{
    return guarded([&] {
        check_f16_mesh(mesh);
        check_T(T);
        if (!delta || !out) fail(FTLE_ERR_INVALID_ARG, "delta or out is NULL");
        need_device(mesh);
        DeviceScope ds(mesh->device);
        check_hip(launch_forward_f16(mesh->fwd.dev(), mesh->d_x, delta, 0.5 / std::fabs(T), out, mesh->n, eig_tau(),
                                     mesh->d_hits, mesh->fwd_block, static_cast<hipStream_t>(stream)),
                  "forward (half-precision flow) launch");
    });
}

ftle_status ftle_tape_bytes(ftle_mesh_t mesh, int64_t* bytes)
{
    return guarded([&] {
        check_mesh(mesh);
        if (!bytes) fail(FTLE_ERR_INVALID_ARG, "bytes is NULL");
        *bytes = mesh->n * (2 * mesh->dim + 1) * (int64_t)mesh->elem();
    });
}

ftle_status ftle_forward_tape(ftle_mesh_t mesh, const void* flow, ftle_dtype dtype, double T, void* out,
                              void* tape, ftle_stream_t stream)
{
    return guarded([&] {
        check_mesh(mesh);
        check_dtype(mesh, dtype);
        check_T(T);
        if (!flow || !out || !tape) fail(FTLE_ERR_INVALID_ARG, "flow, out or tape is NULL");
        need_device(mesh);
        DeviceScope ds(mesh->device);
        check_hip(launch_forward(mesh->dim, mesh->f64(), mesh->fwd.dev(), mesh->d_x, flow, 0.5 / std::fabs(T),
                                 out, tape, !mesh->symmetric, mesh->n, eig_tau(), mesh->d_hits, mesh->fwd_block,
                                 static_cast<hipStream_t>(stream)),
                  "forward+tape launch");
    });
}

ftle_status ftle_backward_tape(ftle_mesh_t mesh, const void* tape, ftle_dtype dtype, const void* grad_ftle,
                               void* grad_flow, ftle_stream_t stream)
{
    return guarded([&] {
        check_mesh(mesh);
        check_dtype(mesh, dtype);
        if (!tape || !grad_ftle || !grad_flow) fail(FTLE_ERR_INVALID_ARG, "tape, grad_ftle or grad_flow is NULL");
        need_device(mesh);
        DeviceScope ds(mesh->device);
        check_hip(launch_backward_gather(mesh->dim, mesh->f64(), mesh->adj_tiles().dev(), mesh->d_x, tape,
                                         !mesh->symmetric, mesh->n, grad_ftle, grad_flow, mesh->bwd_block,
                                         static_cast<hipStream_t>(stream)),
                  "adjoint launch");
    });
}

ftle_status ftle_backward(ftle_mesh_t mesh, const void* flow, ftle_dtype dtype, double T, const void* grad_ftle,
                          void* grad_flow, ftle_stream_t stream)
{
    return guarded([&] {
        check_mesh(mesh);
        check_dtype(mesh, dtype);
        check_T(T);
        if (!flow || !grad_ftle || !grad_flow) fail(FTLE_ERR_INVALID_ARG, "flow, grad_ftle or grad_flow is NULL");
        need_device(mesh);
        DeviceScope ds(mesh->device);
        std::lock_guard<std::mutex> lk(mesh->mu);
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (!mesh->d_work) {
            const size_t bytes = (size_t)mesh->n * (2 * mesh->dim + 1) * mesh->elem();
            check_hip(hipMalloc(&mesh->d_work, bytes), "hipMalloc (adjoint workspace)");
        } else if (mesh->work_stream != s) {
            // the previous call on another stream may still use the workspace
            check_hip(hipStreamWaitEvent(s, mesh->work_done, 0), "hipStreamWaitEvent");
        }
        check_hip(launch_forward(mesh->dim, mesh->f64(), mesh->fwd.dev(), mesh->d_x, flow, 0.5 / std::fabs(T),
                                 nullptr, mesh->d_work, !mesh->symmetric, mesh->n, eig_tau(), mesh->d_hits,
                                 mesh->fwd_block, s),
                  "adjoint tape launch");
        check_hip(launch_backward_gather(mesh->dim, mesh->f64(), mesh->adj_tiles().dev(), mesh->d_x, mesh->d_work,
                                         !mesh->symmetric, mesh->n, grad_ftle, grad_flow, mesh->bwd_block, s),
                  "adjoint launch");
        check_hip(hipEventRecord(mesh->work_done, s), "hipEventRecord");
        mesh->work_stream = s;
    });
}

ftle_status ftle_backward_noalloc(ftle_mesh_t mesh, const void* flow, ftle_dtype dtype, double T,
                                  const void* grad_ftle, void* grad_flow, ftle_stream_t stream)
{
    return guarded([&] {
        check_mesh(mesh);
        check_dtype(mesh, dtype);
        check_T(T);
        if (!flow || !grad_ftle || !grad_flow) fail(FTLE_ERR_INVALID_ARG, "flow, grad_ftle or grad_flow is NULL");
        const size_t bytes = (size_t)mesh->n * (2 * mesh->dim + 1) * mesh->elem();
        if (bytes > kNoAllocScratchBytes)
            fail(FTLE_ERR_UNSUPPORTED, "the adjoint tape (" + std::to_string(bytes) +
                                           " bytes) exceeds the fixed scratch of ftle_backward_noalloc (" +
                                           std::to_string(kNoAllocScratchBytes) + " bytes)");
        need_device(mesh);
        DeviceScope ds(mesh->device);
        void* tape = nullptr;
        check_hip(noalloc_scratch(mesh->device, &tape), "hipGetSymbolAddress (scratch)");
        const hipStream_t s = static_cast<hipStream_t>(stream);
        // the tape forward writes every point's tape entry, so nothing is cleared first
        check_hip(launch_forward(mesh->dim, mesh->f64(), mesh->fwd.dev(), mesh->d_x, flow, 0.5 / std::fabs(T),
                                 nullptr, tape, !mesh->symmetric, mesh->n, eig_tau(), mesh->d_hits,
                                 mesh->fwd_block, s),
                  "adjoint tape launch");
        check_hip(launch_backward_gather(mesh->dim, mesh->f64(), mesh->adj_tiles().dev(), mesh->d_x, tape,
                                         !mesh->symmetric, mesh->n, grad_ftle, grad_flow, mesh->bwd_block, s),
                  "adjoint launch");
    });
}

ftle_status ftle_mesh_fp64_hits(ftle_mesh_t mesh, int64_t* hits, int reset)
{
    return guarded([&] {
        check_mesh(mesh);
        if (!hits) fail(FTLE_ERR_INVALID_ARG, "hits is NULL");
        need_device(mesh);
        DeviceScope ds(mesh->device);
        check_hip(hipDeviceSynchronize(), "hipDeviceSynchronize");
        unsigned long long h = 0;
        check_hip(hipMemcpy(&h, mesh->d_hits, sizeof(h), hipMemcpyDeviceToHost), "hipMemcpy");
        *hits = (int64_t)h;
        if (reset) check_hip(hipMemset(mesh->d_hits, 0, sizeof(h)), "hipMemset");
    });
}

}  // extern "C"

// ===========================================================================
// Batched launches: work list, autotuner, graph cache
// ===========================================================================
namespace {

struct BatchPlan {
    int dim = 0;
    bool f64 = false;
    bool wide = false;   // 64-bit element offsets (some mesh is that large)
    int device = -1;
    std::vector<ftle_mesh_t> meshes;
    void* d_items = nullptr;      // BatchItem[n_items], costliest tiles first
    unsigned* d_queue = nullptr;  // 2 counters
    int n_items = 0;
    size_t lds = 0;
    // chosen launch shape (cap: resident workgroups per CU of a persistent grid)
    int block = 256, tiles_per_pop = 1, grid = 0, cap = 0;
    bool tuned = false;
    // graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t node = nullptr;
    std::vector<unsigned char> arg_storage;
    void* args[6] = {};
    BatchCall last{};          // arguments the graph node holds now
    double last_tau = -1.0;    // eigen threshold the graph node holds now
    // the queue counters are reused by every launch: a launch on another
    // stream than the previous one waits for it
    hipEvent_t done = nullptr;
    hipStream_t done_stream = nullptr;
    bool launched = false;
};

std::mutex g_batch_mu;
std::map<std::vector<ftle_mesh_t>, std::unique_ptr<BatchPlan>> g_plans;

// Launch shape pinned by ftle_batched_pin_config (block 0: not pinned).
struct PinnedShape {
    int block = 0, tiles_per_pop = 0, cap = 0;
};
PinnedShape g_pin;   // guarded by g_batch_mu

BatchPlan* get_plan(int n, const ftle_mesh_t* meshes)
{
    std::vector<ftle_mesh_t> key(meshes, meshes + n);
    auto it = g_plans.find(key);
    if (it != g_plans.end()) return it->second.get();
    std::unique_ptr<BatchPlan> p(new BatchPlan);
    p->meshes = key;
    p->dim = meshes[0]->dim;
    p->f64 = meshes[0]->f64();
    p->device = meshes[0]->device;
    DevTiles maxt{};
    struct Item {
        BatchItem it;
        uint32_t cost;
    };
    std::vector<Item> items;
    uint32_t max_cost = 1;
    for (int k = 0; k < n; ++k) {
        const ftle_mesh_t m = meshes[k];
        p->wide = p->wide || batched_needs_wide(p->dim, p->f64, m->n);
        maxt.max_staged = std::max(maxt.max_staged, m->fwd.max_staged);
        maxt.max_rec = std::max(maxt.max_rec, m->fwd.max_rec);
        const DevTiles dt = m->fwd.dev();
        for (size_t t = 0; t < m->fwd.meta.size(); ++t) {
            const TileMeta& tm = m->fwd.meta[t];
            Item e{};
            e.it.meta = tm;
            e.it.rec = dt.rec;
            e.it.x = m->d_x;
            e.it.fp64_hits = m->d_hits;
            e.it.mesh = (uint32_t)k;
            e.cost = 3 * tm.nwf + tm.P + tm.H;
            items.push_back(e);
            max_cost = std::max(max_cost, e.cost);
        }
    }
    if (items.size() > (size_t)INT32_MAX) fail(FTLE_ERR_UNSUPPORTED, "too many tiles for one batch");
    // costliest first (in eighths of the largest tile), natural order within a bucket
    std::stable_sort(items.begin(), items.end(), [&](const Item& a, const Item& b) {
        return (a.cost * 8ull / (max_cost + 1)) > (b.cost * 8ull / (max_cost + 1));
    });
    std::vector<BatchItem> flat(items.size());
    for (size_t i = 0; i < items.size(); ++i) flat[i] = items[i].it;
    p->n_items = (int)flat.size();
    p->lds = fwd_lds_bytes(p->dim, p->f64, maxt) + kBatchedLdsHead;
    p->d_items = dev_upload(flat.data(), flat.size() * sizeof(BatchItem));
    p->d_queue = static_cast<unsigned*>(dev_upload(nullptr, 2 * sizeof(unsigned)));
    check_hip(hipMemset(p->d_queue, 0, 2 * sizeof(unsigned)), "hipMemset");
    check_hip(hipEventCreateWithFlags(&p->done, hipEventDisableTiming), "hipEventCreateWithFlags");
    check_hip(hipDeviceSynchronize(), "hipDeviceSynchronize");
    BatchPlan* raw = p.get();
    g_plans[key] = std::move(p);
    return raw;
}

int resident_grid(BatchPlan* p, int block, int per_cu_cap)
{
    int per_cu = 0;
    check_hip(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batched_kernel_symbol(p->dim, p->f64, block, p->wide),
                                                           block, p->lds),
              "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    int cus = 0;
    check_hip(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device), "hipDeviceGetAttribute");
    per_cu = std::max(1, std::min(per_cu, per_cu_cap));
    return std::max(1, std::min(p->n_items, per_cu * cus));
}

void autotune(BatchPlan* p, const BatchCall& call, hipStream_t s)
{
    hipEvent_t e0, e1;
    check_hip(hipEventCreate(&e0), "hipEventCreate");
    check_hip(hipEventCreate(&e1), "hipEventCreate");
    static const bool verbose = std::getenv("FTLE_AUTOTUNE_LOG") != nullptr;
    float best = INFINITY;
    const int blocks[] = {128, 256, 512};
    const int pops[] = {0, 1, 2, 4, 8};   // 0: flat launch, one item per workgroup
    const int caps[] = {2, 4, 8};
    for (int b : blocks)
        for (int k : pops)
            for (int cap : caps) {
                if (k == 0 && cap != caps[0]) continue;   // the flat grid has no residency cap
                const int grid = (k == 0) ? p->n_items : resident_grid(p, b, cap);
                if (k > 1 && (int64_t)grid * k > p->n_items) continue;
                float tot = 0.f;
                for (int rep = 0; rep < 4; ++rep) {
                    check_hip(hipEventRecord(e0, s), "hipEventRecord");
                    check_hip(launch_batched(p->dim, p->f64, p->wide, static_cast<const BatchItem*>(p->d_items),
                                             p->n_items, k, p->d_queue, call, p->lds, eig_tau(), b, grid, s),
                              "batched launch");
                    check_hip(hipEventRecord(e1, s), "hipEventRecord");
                    check_hip(hipEventSynchronize(e1), "hipEventSynchronize");
                    float ms = 0.f;
                    check_hip(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime");
                    if (rep > 0) tot += ms;   // first launch warms up
                }
                if (verbose)
                    std::fprintf(stderr, "[ftle autotune] block %d tiles/pop %d grid %d: %.2f us\n", b, k, grid,
                                 1e3f * tot / 3.0f);
                if (tot < best) {
                    best = tot;
                    p->block = b;
                    p->tiles_per_pop = k;
                    p->grid = grid;
                    p->cap = k == 0 ? 0 : cap;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->tuned = true;
}

void build_graph(BatchPlan* p, const BatchCall& call)
{
    p->arg_storage.resize(batched_kernel_arg_storage());
    batched_kernel_args(static_cast<const BatchItem*>(p->d_items), p->n_items, p->tiles_per_pop, p->d_queue, call,
                        eig_tau(), p->arg_storage.data(), p->args);
    check_hip(hipGraphCreate(&p->graph, 0), "hipGraphCreate");
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(batched_kernel_symbol(p->dim, p->f64, p->block, p->wide));
    kp.gridDim = dim3(p->grid);
    kp.blockDim = dim3(p->block);
    kp.sharedMemBytes = (unsigned)p->lds;
    kp.kernelParams = p->args;
    kp.extra = nullptr;
    check_hip(hipGraphAddKernelNode(&p->node, p->graph, nullptr, 0, &kp), "hipGraphAddKernelNode");
    check_hip(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
}

void drop_graph(BatchPlan* p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    p->node = nullptr;
}

// Adopt the pinned launch shape (the graph is rebuilt on the next launch).
void apply_pin(BatchPlan* p, const PinnedShape& pin)
{
    const int cap = pin.tiles_per_pop == 0 ? 0 : pin.cap;
    if (p->tuned && p->block == pin.block && p->tiles_per_pop == pin.tiles_per_pop && p->cap == cap) return;
    p->block = pin.block;
    p->tiles_per_pop = pin.tiles_per_pop;
    p->cap = cap;
    p->grid = pin.tiles_per_pop == 0 ? p->n_items : resident_grid(p, pin.block, cap);
    p->tuned = true;
    drop_graph(p);
}

void free_plan(BatchPlan* p)
{
    drop_graph(p);
    if (p->done) (void)hipEventDestroy(p->done);
    if (p->d_items) (void)hipFree(p->d_items);
    if (p->d_queue) (void)hipFree(p->d_queue);
}

// Drop every cached batch plan that references mesh (its device pointers die with it).
void purge_plans(ftle_mesh_t mesh)
{
    std::lock_guard<std::mutex> lk(g_batch_mu);
    for (auto it = g_plans.begin(); it != g_plans.end();) {
        if (std::find(it->first.begin(), it->first.end(), mesh) != it->first.end()) {
            free_plan(it->second.get());
            it = g_plans.erase(it);
        } else {
            ++it;
        }
    }
}

}  // namespace

extern "C" {

void ftle_destroy_mesh(ftle_mesh_t mesh)
{
    if (!mesh) return;
    if (!mesh->host_only) {
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(mesh->device);
        (void)hipDeviceSynchronize();
        purge_plans(mesh);
        (void)hipSetDevice(cur);
    }
    release_device(mesh);
    delete mesh;
}

ftle_status ftle_release_cached_memory(void)
{
    return guarded([&] {
        int cur = -1;   // the current device, read once something is to be freed
        for (int dev = 0; dev < kMaxCachedDevices; ++dev) {
            BuildScratch& c = g_build_scratch[dev];
            std::lock_guard<std::mutex> lk(c.m);
            if (!c.p || c.busy) continue;
            if (cur < 0) check_hip(hipGetDevice(&cur), "hipGetDevice");
            check_hip(hipSetDevice(dev), "hipSetDevice");
            (void)hipFree(c.p);
            c.p = nullptr;
            c.bytes = 0;
        }
        if (cur >= 0) check_hip(hipSetDevice(cur), "hipSetDevice");
    });
}

ftle_status ftle_cached_memory_bytes(int64_t* bytes)
{
    return guarded([&] {
        if (!bytes) fail(FTLE_ERR_INVALID_ARG, "bytes is NULL");
        int64_t total = 0;
        for (int dev = 0; dev < kMaxCachedDevices; ++dev) {
            BuildScratch& c = g_build_scratch[dev];
            std::lock_guard<std::mutex> lk(c.m);
            total += (int64_t)c.bytes;
        }
        *bytes = total;
    });
}

ftle_status ftle_batched(int n, const ftle_mesh_t* meshes, const void* const* flows, const double* T,
                         void* const* outs, ftle_dtype dtype, ftle_stream_t stream)
{
    return guarded([&] {
        if (n < 1 || n > kMaxBatch) fail(FTLE_ERR_INVALID_ARG, "n must be in [1, 64]");
        if (!meshes || !flows || !T || !outs) fail(FTLE_ERR_INVALID_ARG, "NULL array argument");
        for (int k = 0; k < n; ++k) {
            check_mesh(meshes[k]);
            check_dtype(meshes[k], dtype);
            check_T(T[k]);
            if (!flows[k] || !outs[k]) fail(FTLE_ERR_INVALID_ARG, "NULL flow or out pointer");
            if (meshes[k]->dim != meshes[0]->dim) fail(FTLE_ERR_INVALID_ARG, "meshes of mixed dimension");
            if (meshes[k]->device != meshes[0]->device) fail(FTLE_ERR_INVALID_ARG, "meshes on different devices");
        }
        for (int k = 0; k < n; ++k) need_device(meshes[k]);
        DeviceScope ds(meshes[0]->device);
        std::lock_guard<std::mutex> lk(g_batch_mu);
        BatchPlan* p = get_plan(n, meshes);
        BatchCall call{};
        for (int k = 0; k < n; ++k) {
            call.flow[k] = flows[k];
            call.out[k] = outs[k];
            call.inv2T[k] = 0.5 / std::fabs(T[k]);
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        // the previous launch of this plan may still use the queue counters
        // (only a persistent launch records that it used them)
        if (p->launched && p->done_stream != s) check_hip(hipStreamWaitEvent(s, p->done, 0), "hipStreamWaitEvent");
        if (g_pin.block)
            apply_pin(p, g_pin);
        else if (!p->tuned)
            autotune(p, call, s);
        const double tau = eig_tau();
        if (!p->exec) {
            build_graph(p, call);
            p->last = call;
            p->last_tau = tau;
        }
        if (std::memcmp(&p->last, &call, sizeof(BatchCall)) != 0 || p->last_tau != tau) {
            // new pointers, times or threshold: update the graph's kernel node in place
            batched_kernel_args(static_cast<const BatchItem*>(p->d_items), p->n_items, p->tiles_per_pop, p->d_queue,
                                call, tau, p->arg_storage.data(), p->args);
            hipKernelNodeParams kp{};
            kp.func = const_cast<void*>(batched_kernel_symbol(p->dim, p->f64, p->block, p->wide));
            kp.gridDim = dim3(p->grid);
            kp.blockDim = dim3(p->block);
            kp.sharedMemBytes = (unsigned)p->lds;
            kp.kernelParams = p->args;
            kp.extra = nullptr;
            check_hip(hipGraphExecKernelNodeSetParams(p->exec, p->node, &kp), "hipGraphExecKernelNodeSetParams");
            p->last = call;
            p->last_tau = tau;
        }
        check_hip(hipGraphLaunch(p->exec, s), "hipGraphLaunch");
        if (p->tiles_per_pop > 0) {
            check_hip(hipEventRecord(p->done, s), "hipEventRecord");
            p->done_stream = s;
            p->launched = true;
        }
    });
}

ftle_status ftle_advect_rk4(int flow, const double* params, int64_t n, const void* x0, ftle_dtype dtype,
                            const double* t0s, const double* Ts, double t0, double T, double dt, void* phi,
                            ftle_stream_t stream)
{
    return guarded([&] {
        if (flow != FTLE_FLOW_DOUBLE_GYRE && flow != FTLE_FLOW_ABC) fail(FTLE_ERR_INVALID_ARG, "unknown flow");
        if (dtype != FTLE_F32 && dtype != FTLE_F64) fail(FTLE_ERR_INVALID_ARG, "unknown dtype");
        if (n < 0) fail(FTLE_ERR_INVALID_ARG, "n < 0");
        if (n > 0 && (!x0 || !phi)) fail(FTLE_ERR_INVALID_ARG, "x0 or phi is NULL");
        if (!(dt > 0.0) || !std::isfinite(dt)) fail(FTLE_ERR_INVALID_ARG, "dt must be positive and finite");
        if (!std::isfinite(t0) || !std::isfinite(T)) fail(FTLE_ERR_INVALID_ARG, "t0 and T must be finite");
        if (!Ts && !(std::ceil(std::fabs(T) / dt - 1e-9) <= (double)kMaxAdvectSteps))
            fail(FTLE_ERR_INVALID_ARG, "|T| / dt exceeds the step limit (10^7 steps per particle)");
        double prm[3];
        if (params) {
            for (int k = 0; k < 3; ++k) {
                if (!std::isfinite(params[k])) fail(FTLE_ERR_INVALID_ARG, "non-finite flow parameter");
                prm[k] = params[k];
            }
        } else if (flow == FTLE_FLOW_DOUBLE_GYRE) {
            prm[0] = 0.1, prm[1] = 0.25, prm[2] = 2.0 * 3.14159265358979323846 / 10.0;
        } else {
            prm[0] = std::sqrt(3.0), prm[1] = std::sqrt(2.0), prm[2] = 1.0;
        }
        if (n == 0) return;
        int dev = 0;
        check_hip(hipGetDevice(&dev), "hipGetDevice (no usable GPU?)");
        check_hip(launch_advect(flow, prm, dtype == FTLE_F64, n, x0, t0s, Ts, t0, T, dt, phi,
                                static_cast<hipStream_t>(stream)),
                  "advect launch");
    });
}

ftle_status ftle_advect_rk4_grid(int dim, const int64_t* shape, const double* origin, const double* spacing,
                                 int64_t n_times, double t_first, double t_step, const void* velocity,
                                 ftle_dtype velocity_dtype, int64_t n, const void* x0, ftle_dtype dtype,
                                 const double* t0s, const double* Ts, double t0, double T, double dt, void* phi,
                                 ftle_stream_t stream)
{
    return guarded([&] {
        if (dim != 2 && dim != 3) fail(FTLE_ERR_INVALID_ARG, "dim must be 2 or 3");
        if (!shape || !origin || !spacing) fail(FTLE_ERR_INVALID_ARG, "shape, origin or spacing is NULL");
        if (n_times < 1 || n_times > INT32_MAX) fail(FTLE_ERR_INVALID_ARG, "n_times must be in [1, 2^31)");
        if (!velocity) fail(FTLE_ERR_INVALID_ARG, "velocity is NULL");
        for (ftle_dtype d : {velocity_dtype, dtype})
            if (d != FTLE_F32 && d != FTLE_F64) fail(FTLE_ERR_INVALID_ARG, "unknown dtype");
        GridField g{};
        double values = (double)n_times * dim;
        for (int d = 0; d < dim; ++d) {
            if (shape[d] < 2 || shape[d] > INT32_MAX)
                fail(FTLE_ERR_INVALID_ARG, "every axis needs between 2 and 2^31 - 1 grid nodes");
            if (!std::isfinite(origin[d])) fail(FTLE_ERR_INVALID_ARG, "origin must be finite");
            if (!(spacing[d] > 0.0) || !std::isfinite(spacing[d]))
                fail(FTLE_ERR_INVALID_ARG, "spacing must be positive and finite");
            g.shape[d] = shape[d];
            g.origin[d] = origin[d];
            g.spacing[d] = spacing[d];
            values *= (double)shape[d];
        }
        if (values > 9.0e15) fail(FTLE_ERR_INVALID_ARG, "grid too large");
        if (!std::isfinite(t_first)) fail(FTLE_ERR_INVALID_ARG, "t_first must be finite");
        if (n_times > 1 && (!(t_step > 0.0) || !std::isfinite(t_step)))
            fail(FTLE_ERR_INVALID_ARG, "t_step must be positive and finite");
        g.nt = n_times;
        g.t_first = t_first;
        g.t_step = n_times > 1 ? t_step : 1.0;
        if (n < 0) fail(FTLE_ERR_INVALID_ARG, "n < 0");
        if (n > 0 && (!x0 || !phi)) fail(FTLE_ERR_INVALID_ARG, "x0 or phi is NULL");
        if (!(dt > 0.0) || !std::isfinite(dt)) fail(FTLE_ERR_INVALID_ARG, "dt must be positive and finite");
        if (!std::isfinite(t0) || !std::isfinite(T)) fail(FTLE_ERR_INVALID_ARG, "t0 and T must be finite");
        if (!Ts && !(std::ceil(std::fabs(T) / dt - 1e-9) <= (double)kMaxAdvectSteps))
            fail(FTLE_ERR_INVALID_ARG, "|T| / dt exceeds the step limit (10^7 steps per particle)");
        if (n == 0) return;
        int dev = 0;
        check_hip(hipGetDevice(&dev), "hipGetDevice (no usable GPU?)");
        check_hip(launch_advect_grid(dim, g, velocity, velocity_dtype == FTLE_F64, dtype == FTLE_F64, n, x0, t0s, Ts,
                                     t0, T, dt, phi, static_cast<hipStream_t>(stream)),
                  "advect launch");
    });
}

namespace {

void check_ring1_args(int dim, int64_t n_points, int64_t n_cells, const int32_t* cells, const int64_t* row_ptr,
                      const int32_t* col, int64_t col_capacity, const int64_t* nnz)
{
    if (dim != 2 && dim != 3) fail(FTLE_ERR_INVALID_ARG, "dim must be 2 or 3");
    if (n_points < 1) fail(FTLE_ERR_INVALID_ARG, "n_points < 1");
    if (n_points > INT32_MAX) fail(FTLE_ERR_UNSUPPORTED, "n_points > 2^31-1");
    if (n_cells < 0) fail(FTLE_ERR_INVALID_ARG, "n_cells < 0");
    if (!row_ptr || !nnz || (n_cells > 0 && (!cells || !col)) || col_capacity < 0)
        fail(FTLE_ERR_INVALID_ARG, "null pointer or negative capacity");
    if (n_cells > (int64_t)UINT32_MAX / (dim + 1)) fail(FTLE_ERR_UNSUPPORTED, "more than 2^32-1 cell corners");
}

void ring1_run(int dim, int64_t n_points, int64_t n_cells, const int32_t* cells, int64_t* row_ptr, int32_t* col,
               int64_t col_capacity, int64_t* nnz, void* workspace, hipStream_t s)
{
    int bad = 0, too_long = 0;
    int64_t count = 0;
    check_hip(ring1_build(dim, cells, n_cells, n_points, workspace, row_ptr, col, col_capacity, &count, &bad,
                          &too_long, s),
              "one-ring stencil");
    if (bad) fail(FTLE_ERR_BAD_MESH, "cell index outside [0, n_points)");
    if (too_long) fail(FTLE_ERR_UNSUPPORTED, "a point's incident cells list more than 4096 points");
    *nnz = count;
    if (count > col_capacity) fail(FTLE_ERR_UNSUPPORTED, "col_capacity below the stencil's entry count (in *nnz)");
    check_hip(hipStreamSynchronize(s), "hipStreamSynchronize");
}

}  // namespace

ftle_status ftle_ring1_csr_workspace(int dim, int64_t n_points, int64_t n_cells, int64_t* bytes)
{
    return guarded([&] {
        if (!bytes) fail(FTLE_ERR_INVALID_ARG, "bytes is NULL");
        int64_t dummy = 0;
        check_ring1_args(dim, n_points, n_cells, n_cells ? reinterpret_cast<const int32_t*>(16) : nullptr,
                         reinterpret_cast<const int64_t*>(16), n_cells ? reinterpret_cast<const int32_t*>(16) : nullptr,
                         0, &dummy);
        *bytes = (int64_t)ring1_workspace_bytes(dim, n_points, n_cells);
    });
}

ftle_status ftle_ring1_csr_ws(int dim, int64_t n_points, int64_t n_cells, const int32_t* cells, int64_t* row_ptr,
                              int32_t* col, int64_t col_capacity, int64_t* nnz, void* workspace,
                              int64_t workspace_bytes, ftle_stream_t stream)
{
    return guarded([&] {
        check_ring1_args(dim, n_points, n_cells, cells, row_ptr, col, col_capacity, nnz);
        if (!workspace) fail(FTLE_ERR_INVALID_ARG, "workspace is NULL");
        if (workspace_bytes < (int64_t)ring1_workspace_bytes(dim, n_points, n_cells))
            fail(FTLE_ERR_INVALID_ARG, "workspace smaller than ftle_ring1_csr_workspace's size");
        int dev = 0;
        check_hip(hipGetDevice(&dev), "hipGetDevice (no usable GPU?)");
        ring1_run(dim, n_points, n_cells, cells, row_ptr, col, col_capacity, nnz, workspace,
                  static_cast<hipStream_t>(stream));
    });
}

ftle_status ftle_ring1_csr(int dim, int64_t n_points, int64_t n_cells, const int32_t* cells, int64_t* row_ptr,
                           int32_t* col, int64_t col_capacity, int64_t* nnz, ftle_stream_t stream)
{
    return guarded([&] {
        check_ring1_args(dim, n_points, n_cells, cells, row_ptr, col, col_capacity, nnz);
        int dev = 0;
        check_hip(hipGetDevice(&dev), "hipGetDevice (no usable GPU?)");
        // the device builds' cached scratch (or memory of its own while a build holds it)
        const hipStream_t s = static_cast<hipStream_t>(stream);
        ScratchLease w(ring1_workspace_bytes(dim, n_points, n_cells), s);
        ring1_run(dim, n_points, n_cells, cells, row_ptr, col, col_capacity, nnz, w.get(), s);
    });
}

ftle_status ftle_forward_ell(int dim, int64_t n_points, const void* coords, ftle_dtype dtype, const int32_t* ell,
                             const void* flow, double T, void* out, unsigned flags, ftle_stream_t stream)
{
    return guarded([&] {
        if (dim != 2 && dim != 3) fail(FTLE_ERR_INVALID_ARG, "dim must be 2 or 3");
        if (dtype != FTLE_F32 && dtype != FTLE_F64) fail(FTLE_ERR_INVALID_ARG, "unknown dtype");
        if (n_points < 0) fail(FTLE_ERR_INVALID_ARG, "n_points < 0");
        if (n_points > INT32_MAX) fail(FTLE_ERR_UNSUPPORTED, "n_points > 2^31-1");
        check_T(T);
        if (flags & ~(unsigned)FTLE_ELL_STAGED) fail(FTLE_ERR_INVALID_ARG, "unknown flag");
        if (n_points > 0 && (!coords || !ell || !flow || !out)) fail(FTLE_ERR_INVALID_ARG, "NULL pointer");
        if (reinterpret_cast<uintptr_t>(ell) % (dim == 2 ? 16 : 8) != 0)
            fail(FTLE_ERR_INVALID_ARG, "ell must be 16-byte (2D) or 8-byte (3D) aligned");
        if (n_points == 0) return;
        int dev = 0;
        check_hip(hipGetDevice(&dev), "hipGetDevice (no usable GPU?)");
        check_hip(launch_forward_ell(dim, dtype == FTLE_F64, (flags & FTLE_ELL_STAGED) != 0, coords, flow, ell,
                                     n_points, 0.5 / std::fabs(T), out, eig_tau(), nullptr,
                                     static_cast<hipStream_t>(stream)),
                  "forward (axis list) launch");
    });
}

ftle_status ftle_axis_ell(int dim, int64_t n_points, const void* coords, ftle_dtype dtype, const int64_t* row_ptr,
                          const int32_t* col, int32_t* ell, ftle_stream_t stream)
{
    return guarded([&] {
        if (dim != 2 && dim != 3) fail(FTLE_ERR_INVALID_ARG, "dim must be 2 or 3");
        if (dtype != FTLE_F32 && dtype != FTLE_F64) fail(FTLE_ERR_INVALID_ARG, "unknown dtype");
        if (n_points < 0) fail(FTLE_ERR_INVALID_ARG, "n_points < 0");
        if (n_points > INT32_MAX) fail(FTLE_ERR_UNSUPPORTED, "n_points > 2^31-1");
        if (n_points > 0 && (!coords || !row_ptr || !col || !ell)) fail(FTLE_ERR_INVALID_ARG, "NULL pointer");
        if (reinterpret_cast<uintptr_t>(ell) % (dim == 2 ? 16 : 8) != 0)
            fail(FTLE_ERR_INVALID_ARG, "ell must be 16-byte (2D) or 8-byte (3D) aligned");
        if (n_points == 0) return;
        int dev = 0;
        check_hip(hipGetDevice(&dev), "hipGetDevice (no usable GPU?)");
        check_hip(launch_axis_ell(dim, dtype == FTLE_F64, coords, row_ptr, col, n_points, ell,
                                  static_cast<hipStream_t>(stream)),
                  "axis list launch");
    });
}

ftle_status ftle_batched_pin_config(int block, int tiles_per_pop, int per_cu_cap)
{
    return guarded([&] {
        if (block != 0) {
            if (!supported_block(block)) fail(FTLE_ERR_INVALID_ARG, "block must be 0, 128, 256 or 512");
            if (tiles_per_pop < 0 || tiles_per_pop > 64) fail(FTLE_ERR_INVALID_ARG, "tiles_per_pop must be in [0, 64]");
            if (tiles_per_pop > 0 && (per_cu_cap < 1 || per_cu_cap > 32))
                fail(FTLE_ERR_INVALID_ARG, "per_cu_cap must be in [1, 32]");
        }
        std::lock_guard<std::mutex> lk(g_batch_mu);
        g_pin = block ? PinnedShape{block, tiles_per_pop, tiles_per_pop ? per_cu_cap : 0} : PinnedShape{};
    });
}

ftle_status ftle_batched_config(int n, const ftle_mesh_t* meshes, int* block, int* tiles_per_pop, int* grid)
{
    return guarded([&] {
        if (n < 1 || !meshes) fail(FTLE_ERR_INVALID_ARG, "bad mesh list");
        std::lock_guard<std::mutex> lk(g_batch_mu);
        auto it = g_plans.find(std::vector<ftle_mesh_t>(meshes, meshes + n));
        if (it == g_plans.end() || !it->second->tuned) fail(FTLE_ERR_INVALID_ARG, "no batched call with these meshes yet");
        if (block) *block = it->second->block;
        if (tiles_per_pop) *tiles_per_pop = it->second->tiles_per_pop;
        if (grid) *grid = it->second->grid;
    });
}

}  // extern "C"
