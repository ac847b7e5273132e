/*
 * FTLE oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, double-precision CPU implementation of what the FTLE hot
 * path computes, written to be checked against the mathematics by eye.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it; the product library never calls it and shares no code,
 * header, table or helper with it.
 *
 * What it follows:
 *  - Neighbour lists are built on the host from the mesh cells (Section 2.2,
 *    the decoupled algorithm: neighbours precomputed once, on the CPU, into a
 *    list of integer point indices; a missing neighbour is encoded as -1).
 *  - The per-point FTLE kernel of UVaFTLE (Section 2, the core computation
 *    behind Table 1): flow-map gradient from the point's neighbours, the
 *    Cauchy-Green tensor C = J^T J, its largest eigenvalue, and
 *    FTLE = ln(sqrt(lambda_max)) / |T| (natural logarithm).
 *  - The paper prints no gradient formula; the reading used here is the
 *    least-squares gradient over the stencil, which equals the central
 *    difference on an axis-aligned symmetric stencil and the one-sided
 *    difference where a slot is -1, and is exact for affine flow maps.
 *  - The adjoint (dL/dflow for L = sum_i g_i FTLE_i) is the chain rule of the
 *    same definition, applied in scatter form.
 *
 * Precision: everything in double (the paper's core is double precision,
 * Section 2.1).  Build with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXD 3

/* ------------------------------------------------------------------------ */
/* Threads                                                                   */
/* ------------------------------------------------------------------------ */

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Stencils (Section 2.2: neighbour list computed once, on the host)          */
/* ------------------------------------------------------------------------ */

static int cmp_i32(const void* a, const void* b)
{
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* Upper bound on the number of directed neighbour entries. */
int64_t oracle_ring1_bound(int dim, int64_t ncells)
{
    int k = dim + 1;
    return ncells * (int64_t)k * (int64_t)(k - 1);
}

/*
 * RING1 stencil: every vertex that shares a cell with i, excluding i itself,
 * without duplicates, in ascending index order.
 * row_ptr has n+1 entries; col must hold oracle_ring1_bound() entries.
 * Returns nnz, or -1 if a cell references a point outside [0, n).
 */
int64_t oracle_ring1(int dim, int64_t n, int64_t ncells, const int32_t* cells,
                     int64_t* row_ptr, int32_t* col)
{
    int k = dim + 1;
    int64_t* start = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t* fill = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!start || !fill) { free(start); free(fill); return -2; }
    for (int64_t c = 0; c < ncells; ++c)
        for (int a = 0; a < k; ++a) {
            int32_t v = cells[c * k + a];
            if (v < 0 || v >= n) { free(start); free(fill); return -1; }
            start[v + 1] += k - 1;
        }
    for (int64_t i = 0; i < n; ++i) start[i + 1] += start[i];
    memcpy(fill, start, ((size_t)n + 1) * sizeof(int64_t));
    for (int64_t c = 0; c < ncells; ++c)
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b)
                if (a != b) {
                    int32_t u = cells[c * k + a];
                    col[fill[u]++] = cells[c * k + b];
                }
    /* sort each row, drop duplicates and the point itself, compact */
    int64_t out = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t s = start[i], e = start[i + 1];
        qsort(col + s, (size_t)(e - s), sizeof(int32_t), cmp_i32);
        int32_t prev = -1;
        for (int64_t p = s; p < e; ++p) {
            int32_t v = col[p];
            if (v == (int32_t)i || v == prev) continue;
            col[out++] = v;
            prev = v;
        }
        row_ptr[i + 1] = out;
    }
    free(start);
    free(fill);
    return out;
}

/*
 * AXIS stencil (the paper's fixed-width list, Section 2.2): 2*dim slots per
 * point, slot 2d is the -x_d direction and slot 2d+1 the +x_d direction.
 * Among the RING1 neighbours j with sigma*(x_j - x_i)_d > 0 the slot holds
 * the one with the largest sigma*(x_j - x_i)_d / |x_j - x_i| (ties: smaller
 * index, i.e. the first met in ascending order); with no candidate it holds -1.
 */
void oracle_axis(int dim, int64_t n, const double* x, const int64_t* row_ptr,
                 const int32_t* col, int32_t* slots)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        for (int d = 0; d < dim; ++d)
            for (int sg = 0; sg < 2; ++sg) {
                double sigma = sg ? 1.0 : -1.0;
                double best = 0.0;
                int32_t arg = -1;
                for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                    int32_t j = col[p];
                    double nrm2 = 0.0;
                    for (int e = 0; e < dim; ++e) {
                        double t = x[(int64_t)j * dim + e] - x[i * dim + e];
                        nrm2 += t * t;
                    }
                    double along = sigma * (x[(int64_t)j * dim + d] - x[i * dim + d]);
                    if (!(along > 0.0)) continue;
                    double cosang = along / sqrt(nrm2);
                    if (arg < 0 || cosang > best) { best = cosang; arg = j; }
                }
                slots[i * 2 * dim + 2 * d + sg] = arg;
            }
    }
}

/* ------------------------------------------------------------------------ */
/* Dense helpers (small D x D, row-major double a[r][c])                     */
/* ------------------------------------------------------------------------ */

/* Solve A Y = R for Y (D x D, D right-hand sides) by Gaussian elimination
 * with partial pivoting.  A and R are overwritten.  Returns 0 on success,
 * -1 if a pivot is exactly zero. */
static int gepp_solve(int D, double A[MAXD][MAXD], double R[MAXD][MAXD], double Y[MAXD][MAXD])
{
    for (int c = 0; c < D; ++c) {
        int piv = c;
        for (int r = c + 1; r < D; ++r)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        if (A[piv][c] == 0.0) return -1;
        if (piv != c) {
            for (int k = 0; k < D; ++k) {
                double t = A[c][k]; A[c][k] = A[piv][k]; A[piv][k] = t;
                t = R[c][k]; R[c][k] = R[piv][k]; R[piv][k] = t;
            }
        }
        for (int r = c + 1; r < D; ++r) {
            double f = A[r][c] / A[c][c];
            for (int k = c; k < D; ++k) A[r][k] -= f * A[c][k];
            for (int k = 0; k < D; ++k) R[r][k] -= f * R[c][k];
        }
    }
    for (int k = 0; k < D; ++k)
        for (int r = D - 1; r >= 0; --r) {
            double s = R[r][k];
            for (int q = r + 1; q < D; ++q) s -= A[r][q] * Y[q][k];
            Y[r][k] = s / A[r][r];
        }
    return 0;
}

static double det_small(int D, double A[MAXD][MAXD])
{
    if (D == 2) return A[0][0] * A[1][1] - A[0][1] * A[1][0];
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
         - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
         + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

/*
 * Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix (textbook
 * two-sided rotations, each zeroing one off-diagonal pair), iterated until
 * the squared off-diagonal mass is <= 1e-30 of the squared Frobenius norm,
 * at most 50 sweeps.  On return a's diagonal holds the eigenvalues and the
 * columns of v the matching unit eigenvectors.
 */
static void jacobi3(double a[3][3], double v[3][3])
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) v[r][c] = (r == c) ? 1.0 : 0.0;
    double fro2 = 0.0;
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) fro2 += a[r][c] * a[r][c];
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off2 = 2.0 * (a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2]);
        if (off2 <= 1e-30 * fro2) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                double apq = a[p][q];
                if (apq == 0.0) continue;
                double theta = (a[q][q] - a[p][p]) / (2.0 * apq);
                double t;
                if (fabs(theta) > 1e150) t = 0.5 / theta;
                else t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int r = 0; r < 3; ++r) {
                    if (r == p || r == q) continue;
                    double arp = a[r][p], arq = a[r][q];
                    a[r][p] = a[p][r] = c * arp - s * arq;
                    a[r][q] = a[q][r] = s * arp + c * arq;
                }
                a[p][p] -= t * apq;
                a[q][q] += t * apq;
                a[p][q] = a[q][p] = 0.0;
                for (int r = 0; r < 3; ++r) {
                    double vrp = v[r][p], vrq = v[r][q];
                    v[r][p] = c * vrp - s * vrq;
                    v[r][q] = s * vrp + c * vrq;
                }
            }
    }
}

/* Exposed for the eigen pins: eigenvalues (ascending) and eigenvectors
 * (columns of vecs, row-major 3x3) of the symmetric matrix m (row-major). */
void oracle_jacobi_eig3(const double* m, double* vals, double* vecs)
{
    double a[3][3], v[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) a[r][c] = 0.5 * (m[r * 3 + c] + m[c * 3 + r]);
    jacobi3(a, v);
    int idx[3] = {0, 1, 2};
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (a[idx[j]][idx[j]] < a[idx[i]][idx[i]]) { int t = idx[i]; idx[i] = idx[j]; idx[j] = t; }
    for (int i = 0; i < 3; ++i) {
        vals[i] = a[idx[i]][idx[i]];
        for (int r = 0; r < 3; ++r) vecs[r * 3 + i] = v[r][idx[i]];
    }
}

/* ------------------------------------------------------------------------ */
/* Per-point FTLE                                                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    int ok;              /* 1 if the stencil has full rank */
    double M[MAXD][MAXD];/* sum dx dx^T */
    double J[MAXD][MAXD];/* flow-map gradient, J[r][c] = d phi_r / d x_c */
    double lam;          /* largest eigenvalue of C = J^T J */
    double lam2;         /* second largest eigenvalue */
    double v[MAXD];      /* unit eigenvector of lam */
    double detratio;     /* det M / (tr M / D)^D */
} point_state;

/*
 * Least-squares flow-map gradient at point i over its stencil (entries -1
 * are absent neighbours and are skipped), then C = J^T J and its top
 * eigenpair.  X = [x_j - x_i] (D x k), F = [phi_j - phi_i] (D x k),
 * M = X X^T, and J = F X^T M^{-1}, obtained by solving M J^T = X F^T.
 */
static void point_eval(int D, int64_t i, const double* x, const double* phi,
                       const int64_t* row_ptr, const int32_t* col, point_state* st)
{
    double M[MAXD][MAXD] = {{0}}, R[MAXD][MAXD] = {{0}}, Y[MAXD][MAXD] = {{0}};
    int k = 0;
    for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
        int64_t j = col[p];
        if (j < 0) continue;
        double dx[MAXD], df[MAXD];
        for (int e = 0; e < D; ++e) {
            dx[e] = x[j * D + e] - x[i * D + e];
            df[e] = phi[j * D + e] - phi[i * D + e];
        }
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) {
                M[r][c] += dx[r] * dx[c];
                R[r][c] += dx[r] * df[c];      /* (X F^T)[r][c] */
            }
        ++k;
    }
    memcpy(st->M, M, sizeof(M));
    double tr = 0.0;
    for (int e = 0; e < D; ++e) tr += M[e][e];
    double det = det_small(D, M);
    double scale = pow(tr / D, D);
    st->detratio = (scale > 0.0) ? det / scale : 0.0;
    st->ok = 0;
    if (k < D || !(det > 1e-12 * scale)) return;
    double A[MAXD][MAXD];
    memcpy(A, M, sizeof(M));
    if (gepp_solve(D, A, R, Y) != 0) return;
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) st->J[r][c] = Y[c][r];
    /* Cauchy-Green tensor */
    double C[MAXD][MAXD];
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) {
            double s = 0.0;
            for (int r = 0; r < D; ++r) s += st->J[r][a] * st->J[r][b];
            C[a][b] = s;
        }
    if (D == 2) {
        /* largest eigenvalue of [[a, b], [b, c]]: m + sqrt(d^2 + b^2) */
        double a = C[0][0], b = C[0][1], c = C[1][1];
        double m = 0.5 * (a + c), d = 0.5 * (a - c), h = hypot(d, b);
        st->lam = m + h;
        st->lam2 = m - h;
        double v0, v1;
        /* (C - lam I) v = 0: rows give v ~ (lam - c, b) = (d + h, b) and
         * v ~ (b, lam - a) = (b, h - d); take the one without cancellation */
        if (d >= 0.0) { v0 = d + h; v1 = b; }
        else          { v0 = b; v1 = h - d; }
        double nv = hypot(v0, v1);
        if (nv > 0.0) { st->v[0] = v0 / nv; st->v[1] = v1 / nv; }
        else          { st->v[0] = 1.0; st->v[1] = 0.0; }
    } else {
        double a[3][3], V[3][3];
        memcpy(a, C, sizeof(a));
        jacobi3(a, V);
        int top = 0;
        for (int e = 1; e < 3; ++e) if (a[e][e] > a[top][top]) top = e;
        st->lam = a[top][top];
        double second = -INFINITY;
        for (int e = 0; e < 3; ++e) if (e != top && a[e][e] > second) second = a[e][e];
        st->lam2 = second;
        for (int r = 0; r < 3; ++r) st->v[r] = V[r][top];
    }
    st->ok = 1;
}

static double ftle_of(double lam, double T)
{
    return 0.5 * log(lam) / fabs(T);
}

/*
 * FTLE for the points listed in sel (nsel of them; sel == NULL means all n
 * points, out[i] for point i).  x, phi: n x dim row-major doubles.  The
 * stencil is a CSR (row_ptr n+1, col) whose -1 entries are skipped.
 * Optional outputs (may be NULL): gap = (lam1 - lam2)/lam1, detratio.
 */
void oracle_ftle(int dim, int64_t n, const double* x, const double* phi,
                 const int64_t* row_ptr, const int32_t* col, double T,
                 int64_t nsel, const int64_t* sel, double* out, double* gap, double* detratio)
{
    int64_t cnt = sel ? nsel : n;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t k = 0; k < cnt; ++k) {
        int64_t i = sel ? sel[k] : k;
        point_state st;
        point_eval(dim, i, x, phi, row_ptr, col, &st);
        out[k] = st.ok ? ftle_of(st.lam, T) : NAN;
        if (gap) gap[k] = st.ok ? (st.lam - st.lam2) / st.lam : NAN;
        if (detratio) detratio[k] = st.detratio;
    }
}

/*
 * Adjoint of L = sum_i g_i FTLE_i with respect to the flow map.
 *   dFTLE_i/dJ_i = (J_i v_i) v_i^T / (|T| lam_i)         (d lam = 2 (Jv)^T dJ v)
 *   G_i = g_i dFTLE_i/dJ_i,  H_i = G_i M_i^{-1}           (J = B M^{-1})
 *   B_i = sum_j (phi_j - phi_i)(x_j - x_i)^T, so each stencil entry adds
 *   H_i (x_j - x_i) to dL/dphi_j and subtracts it from dL/dphi_i.
 * Points whose FTLE is not finite (rank-deficient stencil, lam = 0) add
 * nothing.  grad (n x dim) is overwritten.
 */
void oracle_ftle_grad(int dim, int64_t n, const double* x, const double* phi,
                      const int64_t* row_ptr, const int32_t* col, double T,
                      const double* g, double* grad)
{
    int D = dim;
    double* H = (double*)calloc((size_t)n * D * D, sizeof(double));
    unsigned char* use = (unsigned char*)calloc((size_t)n, 1);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; ++i) {
        point_state st;
        point_eval(D, i, x, phi, row_ptr, col, &st);
        if (!st.ok || !(st.lam > 0.0) || !isfinite(st.lam) || !isfinite(g[i])) continue;
        double Jv[MAXD];
        for (int r = 0; r < D; ++r) {
            double s = 0.0;
            for (int c = 0; c < D; ++c) s += st.J[r][c] * st.v[c];
            Jv[r] = s;
        }
        double coef = g[i] / (fabs(T) * st.lam);
        /* solve M H^T = G^T, i.e. H = G M^{-1} (M symmetric) */
        double A[MAXD][MAXD], R[MAXD][MAXD], Ht[MAXD][MAXD] = {{0}};
        memcpy(A, st.M, sizeof(A));
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) R[r][c] = coef * Jv[c] * st.v[r];  /* G^T[r][c] = G[c][r] */
        if (gepp_solve(D, A, R, Ht) != 0) continue;
        for (int r = 0; r < D; ++r)
            for (int c = 0; c < D; ++c) H[i * D * D + r * D + c] = Ht[c][r];
        use[i] = 1;
    }
    memset(grad, 0, (size_t)n * D * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        if (!use[i]) continue;
        const double* Hi = H + i * D * D;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            int64_t j = col[p];
            if (j < 0) continue;
            double dx[MAXD];
            for (int e = 0; e < D; ++e) dx[e] = x[j * D + e] - x[i * D + e];
            for (int r = 0; r < D; ++r) {
                double s = 0.0;
                for (int c = 0; c < D; ++c) s += Hi[r * D + c] * dx[c];
                grad[j * D + r] += s;
                grad[i * D + r] -= s;
            }
        }
    }
    free(H);
    free(use);
}

/* ------------------------------------------------------------------------ */
/* Flow maps by advection (the step before the FTLE path: the paper's inputs */
/* are precomputed flow maps, Section 2.2)                                   */
/* ------------------------------------------------------------------------ */
/*
 * Velocity of an analytic flow at point p, time t.
 *  kind 0, the double gyre (Shadden, Lekien and Marsden, Physica D 212,
 *    2005), params A, eps, omega: stream function
 *    psi = A sin(pi f(x, t)) sin(pi y), f = eps sin(omega t) x^2 +
 *    (1 - 2 eps sin(omega t)) x; velocity (-dpsi/dy, dpsi/dx).
 *  kind 1, the steady ABC flow, params A, B, C:
 *    (A sin z + C cos y, B sin x + A cos z, C sin y + B cos x).
 */
static void velocity(int kind, const double* prm, const double* p, double t, double* v)
{
    const double pi = 3.14159265358979323846;
    if (kind == 0) {
        const double A = prm[0], eps = prm[1], om = prm[2];
        const double s = sin(om * t);
        const double a = eps * s, b = 1.0 - 2.0 * eps * s;
        const double f = a * p[0] * p[0] + b * p[0];
        const double dfdx = 2.0 * a * p[0] + b;
        v[0] = -pi * A * sin(pi * f) * cos(pi * p[1]);
        v[1] = pi * A * cos(pi * f) * sin(pi * p[1]) * dfdx;
    } else {
        const double A = prm[0], B = prm[1], C = prm[2];
        v[0] = A * sin(p[2]) + C * cos(p[1]);
        v[1] = B * sin(p[0]) + A * cos(p[2]);
        v[2] = C * sin(p[1]) + B * cos(p[0]);
    }
}

/*
 * Flow map phi_i = x_i(t0_i + T_i) by the classical fourth-order Runge-Kutta
 * method: steps = max(1, ceil(|T_i| / dt - 1e-9)) steps of h = T_i / steps.
 * x0, phi: n x dim; t0, T: n values each.
 */
void oracle_advect_rk4(int kind, const double* prm, int64_t n, const double* x0, const double* t0,
                       const double* T, double dt, double* phi)
{
    const int D = kind == 0 ? 2 : 3;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double p[3], q[3], k1[3], k2[3], k3[3], k4[3];
        for (int d = 0; d < D; ++d) p[d] = x0[i * D + d];
        double steps = ceil(fabs(T[i]) / dt - 1e-9);
        if (steps < 1.0) steps = 1.0;
        const double h = T[i] / steps;
        for (int64_t s = 0; s < (int64_t)steps; ++s) {
            const double t = t0[i] + (double)s * h;
            velocity(kind, prm, p, t, k1);
            for (int d = 0; d < D; ++d) q[d] = p[d] + 0.5 * h * k1[d];
            velocity(kind, prm, q, t + 0.5 * h, k2);
            for (int d = 0; d < D; ++d) q[d] = p[d] + 0.5 * h * k2[d];
            velocity(kind, prm, q, t + 0.5 * h, k3);
            for (int d = 0; d < D; ++d) q[d] = p[d] + h * k3[d];
            velocity(kind, prm, q, t + h, k4);
            for (int d = 0; d < D; ++d) p[d] += h / 6.0 * (k1[d] + 2.0 * k2[d] + 2.0 * k3[d] + k4[d]);
        }
        for (int d = 0; d < D; ++d) phi[i * D + d] = p[d];
    }
}

/*
 * A velocity field sampled on a regular grid (the form simulation data
 * comes in): nodes origin[d] + i spacing[d], i = 0 .. shape[d] - 1, along
 * each axis, at times t_first + k t_step, k = 0 .. nt - 1; vel holds the dim
 * components of node (x, y[, z]) at slice k at
 * ((k * nz + z) * ny + y) * nx + x (x fastest).  Between nodes the velocity
 * is multilinear in space (bilinear, trilinear) and linear in time; a point
 * outside the grid's box takes the value at the nearest point of the box, a
 * time before the first slice or after the last that slice's value.
 */
static void grid_velocity(int D, const int64_t* shape, const double* origin, const double* spacing, int64_t nt,
                          double t_first, double t_step, const double* vel, const double* p, double t, double* v)
{
    int64_t cell[3] = {0, 0, 0};
    double f[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < D; ++d) {
        double u = (p[d] - origin[d]) / spacing[d];
        const double top = (double)(shape[d] - 1);
        if (!(u > 0.0)) u = 0.0;   /* also NaN */
        if (u > top) u = top;
        int64_t c = (int64_t)floor(u);
        if (c > shape[d] - 2) c = shape[d] - 2;
        cell[d] = c;
        f[d] = u - (double)c;
    }
    int64_t k = 0;
    double g = 0.0;
    if (nt > 1) {
        double s = (t - t_first) / t_step;
        if (!(s > 0.0)) s = 0.0;
        if (s > (double)(nt - 1)) s = (double)(nt - 1);
        k = (int64_t)floor(s);
        if (k > nt - 2) k = nt - 2;
        g = s - (double)k;
    }
    const int64_t nx = shape[0], ny = shape[1], nz = D == 3 ? shape[2] : 1;
    for (int c = 0; c < D; ++c) v[c] = 0.0;
    for (int slice = 0; slice < (nt > 1 ? 2 : 1); ++slice) {
        const double ws = nt > 1 ? (slice ? g : 1.0 - g) : 1.0;
        for (int corner = 0; corner < (1 << D); ++corner) {
            double w = ws;
            int64_t at[3] = {0, 0, 0};
            for (int d = 0; d < D; ++d) {
                const int bit = (corner >> d) & 1;
                w *= bit ? f[d] : 1.0 - f[d];
                at[d] = cell[d] + bit;
            }
            const int64_t node = (((k + slice) * nz + at[2]) * ny + at[1]) * nx + at[0];
            for (int c = 0; c < D; ++c) v[c] += w * vel[node * D + c];
        }
    }
}

/* oracle_advect_rk4 in a gridded velocity field (grid_velocity above). */
void oracle_advect_rk4_grid(int D, const int64_t* shape, const double* origin, const double* spacing, int64_t nt,
                            double t_first, double t_step, const double* vel, int64_t n, const double* x0,
                            const double* t0, const double* T, double dt, double* phi)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double p[3], q[3], k1[3], k2[3], k3[3], k4[3];
        for (int d = 0; d < D; ++d) p[d] = x0[i * D + d];
        double steps = ceil(fabs(T[i]) / dt - 1e-9);
        if (steps < 1.0) steps = 1.0;
        const double h = T[i] / steps;
        for (int64_t s = 0; s < (int64_t)steps; ++s) {
            const double t = t0[i] + (double)s * h;
            grid_velocity(D, shape, origin, spacing, nt, t_first, t_step, vel, p, t, k1);
            for (int d = 0; d < D; ++d) q[d] = p[d] + 0.5 * h * k1[d];
            grid_velocity(D, shape, origin, spacing, nt, t_first, t_step, vel, q, t + 0.5 * h, k2);
            for (int d = 0; d < D; ++d) q[d] = p[d] + 0.5 * h * k2[d];
            grid_velocity(D, shape, origin, spacing, nt, t_first, t_step, vel, q, t + 0.5 * h, k3);
            for (int d = 0; d < D; ++d) q[d] = p[d] + h * k3[d];
            grid_velocity(D, shape, origin, spacing, nt, t_first, t_step, vel, q, t + h, k4);
            for (int d = 0; d < D; ++d) p[d] += h / 6.0 * (k1[d] + 2.0 * k2[d] + 2.0 * k3[d] + k4[d]);
        }
        for (int d = 0; d < D; ++d) phi[i * D + d] = p[d];
    }
}
