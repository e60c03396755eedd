/*
 * CPU oracle for the shallow-basin PCG solves.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no source with the HIP library:
 * it assembles the P1 operators itself, eliminates Dirichlet nodes explicitly
 * and runs a textbook Jacobi-preconditioned conjugate gradient, all in plain
 * FP64 with no blocking, fusion or reordering.
 *
 * What it computes (paper sections cited per function):
 *   - P1 element matrices on a tetrahedron: the bilinear forms of the
 *     velocity-prediction problem (Sec. 4/5, eq. fofa_velo_pred_h: mass
 *     term and anisotropic viscous term with nu = diag(nu1,nu2,nu3)), of the
 *     pressure-increment problem (eq. fofa_q_cor_h: gradient-gradient term)
 *     and the divergence coupling int (d u_c / d x_c) phi (right-hand side
 *     of eq. fofa_q_cor_h, and the pressure term int p div v of
 *     eq. fofa_velo_pred_h through its transpose);
 *   - assembly of those forms into compressed sparse rows;
 *   - the same mass and anisotropic stiffness forms on the brick elements of
 *     Sec. 5 (Q2 for the velocity, Q1 for the pressure), with a trilinear
 *     geometry map and tensor Gauss quadrature;
 *   - the surface-tension load int_{Gamma_s} theta v ds (eq. fofa_velo_pred_h);
 *   - the explicit advection term int ((u . grad) u_c) phi ds of the same
 *     equation, evaluated at a given velocity;
 *   - preconditioned conjugate gradients with a diagonal preconditioner
 *     (Remark 1 and the DIAG part of Remark 2 at the end of Sec. 5), or with
 *     the inverse of the vertical-line (water column) blocks of the matrix,
 *     a block-diagonal preconditioner the paper does not use: it stands in
 *     for its unavailable line-search preconditioner of Remark 2 and makes
 *     the isotropic pressure operator of eq. fofa_q_cor_h tractable on thin
 *     meshes;
 *   - a dense Cholesky factorisation for tiny systems.
 *
 * Two builds of this one file: the plain one (no OpenMP) is the parity
 * oracle; compiled with -fopenmp it is the multi-core timing baseline of the
 * Jacobi-PCG loop (static row partition of the products and vector updates,
 * dot products as 256 fixed chunks each summed in order, then the chunk sums
 * in order, so results do not depend on the thread count).  The OpenMP
 * pragmas are ignored by the plain build, whose arithmetic they leave as is.
 */
#define _POSIX_C_SOURCE 199309L /* clock_gettime */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_ERR_INVALID (-1)
#define OR_ERR_MESH (-4)
#define OR_ERR_BREAKDOWN (-5)
#define OR_ERR_NOMEM (-3)

/* ------------------------------------------------------------------------ */
/* Element matrices                                                          */
/* ------------------------------------------------------------------------ */

/* Gradients of the four barycentric (P1 hat) functions of a tetrahedron and
 * its signed volume.  With J the 3x3 matrix whose columns are v1-v0, v2-v0,
 * v3-v0, the barycentric coordinates l1,l2,l3 are J^{-1}(x - v0), so grad l_a
 * (a = 1..3) is row a of J^{-1}, and grad l0 = -(grad l1 + grad l2 + grad l3).
 * Returns the signed volume det(J)/6. */
static double tet_gradients(const double X[4][3], double g[4][3])
{
    double J[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            J[r][c] = X[c + 1][r] - X[0][r];
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (det == 0.0) {
        memset(g, 0, sizeof(double) * 12);
        return 0.0;
    }
    /* inverse by the adjugate */
    double inv[3][3];
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    for (int a = 1; a < 4; ++a)
        for (int d = 0; d < 3; ++d)
            g[a][d] = inv[a - 1][d];
    for (int d = 0; d < 3; ++d)
        g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
    return det / 6.0;
}

/* Element matrices of one tetrahedron.
 *   K[a][b]    = vol * sum_d nu[d] g_a[d] g_b[d]     (int (nu grad phi_b).grad phi_a)
 *   M[a][b]    = vol/20 * (1 + delta_ab)              (int phi_a phi_b, exact for P1)
 *   B[c][a][b] = vol/4 * g_b[c]                       (int phi_a d phi_b / d x_c)
 * Any output pointer may be NULL.  Returns the signed volume. */
double or_element(const double *X12, const double *nu, double *K, double *M,
                  double *B)
{
    double X[4][3], g[4][3];
    memcpy(X, X12, sizeof(X));
    double vol = tet_gradients(X, g);
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
            if (K) {
                double s = 0.0;
                for (int d = 0; d < 3; ++d)
                    s += nu[d] * (g[a][d] * g[b][d]);
                K[a * 4 + b] = vol * s;
            }
            if (M)
                M[a * 4 + b] = vol / 20.0 * (a == b ? 2.0 : 1.0);
            if (B)
                for (int c = 0; c < 3; ++c)
                    B[c * 16 + a * 4 + b] = vol / 4.0 * g[b][c];
        }
    return vol;
}

/* ------------------------------------------------------------------------ */
/* Assembly into CSR                                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t n, nnz;
    int64_t *rowptr; /* n+1 */
    int32_t *col;    /* nnz */
    double *val;     /* nnz */
} or_csr;

void or_csr_free(or_csr *A)
{
    if (!A) return;
    free(A->rowptr);
    free(A->col);
    free(A->val);
    free(A);
}

int64_t or_csr_n(const or_csr *A) { return A->n; }
int64_t or_csr_nnz(const or_csr *A) { return A->nnz; }
void or_csr_copy_out(const or_csr *A, int64_t *rowptr, int32_t *col, double *val)
{
    memcpy(rowptr, A->rowptr, sizeof(int64_t) * (A->n + 1));
    memcpy(col, A->col, sizeof(int32_t) * A->nnz);
    memcpy(val, A->val, sizeof(double) * A->nnz);
}

/* Collects element contributions (row, col, value) bucketed by row, then sorts
 * each row by column and sums duplicates.  `nloc` local dofs per element. */
typedef struct {
    int64_t n;
    int64_t *start; /* n+1: bucket offsets */
    int64_t *fill;  /* n: next free slot per bucket */
    int32_t *c;
    double *v;
} triplets;

static int trip_init(triplets *t, int64_t n, int64_t nel, int nloc, const int32_t *conn)
{
    t->n = n;
    t->start = calloc((size_t)n + 1, sizeof(int64_t));
    t->fill = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!t->start || !t->fill) return OR_ERR_NOMEM;
    for (int64_t e = 0; e < nel; ++e)
        for (int a = 0; a < nloc; ++a)
            t->start[conn[e * nloc + a] + 1] += nloc;
    for (int64_t i = 0; i < n; ++i)
        t->start[i + 1] += t->start[i];
    for (int64_t i = 0; i < n; ++i)
        t->fill[i] = t->start[i];
    int64_t tot = t->start[n];
    t->c = malloc(sizeof(int32_t) * (size_t)(tot > 0 ? tot : 1));
    t->v = malloc(sizeof(double) * (size_t)(tot > 0 ? tot : 1));
    if (!t->c || !t->v) return OR_ERR_NOMEM;
    return OR_OK;
}

static void trip_add(triplets *t, int32_t r, int32_t c, double v)
{
    int64_t s = t->fill[r]++;
    t->c[s] = c;
    t->v[s] = v;
}

static void trip_free(triplets *t)
{
    free(t->start);
    free(t->fill);
    free(t->c);
    free(t->v);
}

/* Sort every bucket by column (insertion sort, buckets are short) and sum
 * duplicate columns into a fresh CSR matrix. */
static or_csr *trip_to_csr(triplets *t)
{
    int64_t n = t->n;
    int64_t nnz = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t lo = t->start[i], hi = t->start[i + 1];
        for (int64_t s = lo + 1; s < hi; ++s) {
            int32_t c = t->c[s];
            double v = t->v[s];
            int64_t u = s - 1;
            while (u >= lo && t->c[u] > c) {
                t->c[u + 1] = t->c[u];
                t->v[u + 1] = t->v[u];
                --u;
            }
            t->c[u + 1] = c;
            t->v[u + 1] = v;
        }
        for (int64_t s = lo; s < hi; ++s)
            if (s == lo || t->c[s] != t->c[s - 1]) ++nnz;
    }
    or_csr *A = calloc(1, sizeof(or_csr));
    if (!A) return NULL;
    A->n = n;
    A->nnz = nnz;
    A->rowptr = malloc(sizeof(int64_t) * (size_t)(n + 1));
    A->col = malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    A->val = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!A->rowptr || !A->col || !A->val) {
        or_csr_free(A);
        return NULL;
    }
    int64_t k = 0;
    A->rowptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t lo = t->start[i], hi = t->start[i + 1];
        for (int64_t s = lo; s < hi; ++s) {
            if (s == lo || t->c[s] != t->c[s - 1]) {
                A->col[k] = t->c[s];
                A->val[k] = t->v[s];
                ++k;
            } else {
                A->val[k - 1] += t->v[s];
            }
        }
        A->rowptr[i + 1] = k;
    }
    return A;
}

static int check_conn(int64_t n, int64_t nel, int nloc, const int32_t *conn)
{
    for (int64_t e = 0; e < nel * nloc; ++e)
        if (conn[e] < 0 || conn[e] >= n) return OR_ERR_MESH;
    return OR_OK;
}

/* Assemble one of the volume forms over the tetrahedral mesh.
 *   form 0: c_mass * M + c_stiff * K_nu     with nu = (nu_h, nu_h, nu_v)
 *   form 1: B_c  (c = comp in 0..2), the divergence coupling
 * A tetrahedron with non-positive signed volume is a mesh error. */
int or_assemble(int64_t n, const double *xyz, int64_t ntet, const int32_t *tets,
                int form, double nu_h, double nu_v, double c_mass, double c_stiff,
                int comp, or_csr **out)
{
    *out = NULL;
    if (n <= 0 || ntet < 0) return OR_ERR_INVALID;
    if (check_conn(n, ntet, 4, tets) != OR_OK) return OR_ERR_MESH;
    triplets t;
    memset(&t, 0, sizeof(t));
    if (trip_init(&t, n, ntet, 4, tets) != OR_OK) {
        trip_free(&t);
        return OR_ERR_NOMEM;
    }
    const double nu[3] = {nu_h, nu_h, nu_v};
    for (int64_t e = 0; e < ntet; ++e) {
        double X[12], K[16], M[16], B[48];
        for (int a = 0; a < 4; ++a)
            for (int d = 0; d < 3; ++d)
                X[a * 3 + d] = xyz[(int64_t)tets[e * 4 + a] * 3 + d];
        double vol = or_element(X, nu, K, M, B);
        if (!(vol > 0.0)) {
            trip_free(&t);
            return OR_ERR_MESH;
        }
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                double v = (form == 0) ? c_mass * M[a * 4 + b] + c_stiff * K[a * 4 + b]
                                       : B[comp * 16 + a * 4 + b];
                trip_add(&t, tets[e * 4 + a], tets[e * 4 + b], v);
            }
    }
    *out = trip_to_csr(&t);
    trip_free(&t);
    return *out ? OR_OK : OR_ERR_NOMEM;
}

/* Explicit advection term of the velocity prediction (Sec. 3 eq. pred_velo,
 * Sec. 5 eq. fofa_velo_pred_h): for each component c and node a,
 *   out[c][a] = int ((u . grad) u_c) phi_a dx
 * for the P1 velocity u with nodal values u[c][i] (3 x n, component-major).
 * On a tetrahedron grad u_c is constant, G_c = sum_b u_c(b) grad phi_b, and
 * (u . grad) u_c = sum_b phi_b (u(b) . G_c) is linear, so the integral is the
 * element mass matrix applied to the nodal values s_b = u(b) . G_c. */
int or_advection(int64_t n, const double *xyz, int64_t ntet, const int32_t *tets,
                 const double *u, double *out)
{
    if (n <= 0 || ntet < 0) return OR_ERR_INVALID;
    if (check_conn(n, ntet, 4, tets) != OR_OK) return OR_ERR_MESH;
    for (int64_t i = 0; i < 3 * n; ++i) out[i] = 0.0;
    const double one[3] = {1.0, 1.0, 1.0};
    for (int64_t e = 0; e < ntet; ++e) {
        double X[12], M[16], B[48];
        int64_t v[4];
        for (int a = 0; a < 4; ++a) {
            v[a] = tets[e * 4 + a];
            for (int d = 0; d < 3; ++d) X[a * 3 + d] = xyz[v[a] * 3 + d];
        }
        double vol = or_element(X, one, NULL, M, B);
        if (!(vol > 0.0)) return OR_ERR_MESH;
        /* grad phi_b [d] = B[d][a][b] * 4 / vol for any a */
        double g[4][3];
        for (int b = 0; b < 4; ++b)
            for (int d = 0; d < 3; ++d) g[b][d] = B[d * 16 + b] * 4.0 / vol;
        for (int c = 0; c < 3; ++c) {
            double G[3] = {0.0, 0.0, 0.0};
            for (int b = 0; b < 4; ++b)
                for (int d = 0; d < 3; ++d) G[d] += u[c * n + v[b]] * g[b][d];
            double sv[4];
            for (int b = 0; b < 4; ++b) {
                sv[b] = 0.0;
                for (int d = 0; d < 3; ++d) sv[b] += u[d * n + v[b]] * G[d];
            }
            for (int a = 0; a < 4; ++a) {
                double r = 0.0;
                for (int b = 0; b < 4; ++b) r += M[a * 4 + b] * sv[b];
                out[c * n + v[a]] += r;
            }
        }
    }
    return OR_OK;
}

/* Mass matrix of the surface Gamma_s from its triangles: on a triangle of
 * area A, int phi_a phi_b ds = A/12 * (1 + delta_ab). */
int or_assemble_surface_mass(int64_t n, const double *xyz, int64_t ntri,
                             const int32_t *tris, or_csr **out)
{
    *out = NULL;
    if (check_conn(n, ntri, 3, tris) != OR_OK) return OR_ERR_MESH;
    triplets t;
    memset(&t, 0, sizeof(t));
    if (trip_init(&t, n, ntri, 3, tris) != OR_OK) {
        trip_free(&t);
        return OR_ERR_NOMEM;
    }
    for (int64_t e = 0; e < ntri; ++e) {
        const double *p0 = xyz + 3 * (int64_t)tris[3 * e];
        const double *p1 = xyz + 3 * (int64_t)tris[3 * e + 1];
        const double *p2 = xyz + 3 * (int64_t)tris[3 * e + 2];
        double u[3], w[3], cr[3];
        for (int d = 0; d < 3; ++d) {
            u[d] = p1[d] - p0[d];
            w[d] = p2[d] - p0[d];
        }
        cr[0] = u[1] * w[2] - u[2] * w[1];
        cr[1] = u[2] * w[0] - u[0] * w[2];
        cr[2] = u[0] * w[1] - u[1] * w[0];
        double area = 0.5 * sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        if (!(area > 0.0)) {
            trip_free(&t);
            return OR_ERR_MESH;
        }
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                trip_add(&t, tris[3 * e + a], tris[3 * e + b],
                         area / 12.0 * (a == b ? 2.0 : 1.0));
    }
    *out = trip_to_csr(&t);
    trip_free(&t);
    return *out ? OR_OK : OR_ERR_NOMEM;
}

/* ------------------------------------------------------------------------ */
/* Sparse products and vector helpers                                        */
/* ------------------------------------------------------------------------ */

void or_spmv(const or_csr *A, const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < A->n; ++i) {
        double s = 0.0;
        for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
            s += A->val[k] * x[A->col[k]];
        y[i] = s;
    }
}

/* y = A^T x */
void or_spmv_t(const or_csr *A, const double *x, double *y, int64_t ncols)
{
    for (int64_t j = 0; j < ncols; ++j) y[j] = 0.0;
    for (int64_t i = 0; i < A->n; ++i)
        for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k)
            y[A->col[k]] += A->val[k] * x[i];
}

#ifdef _OPENMP
enum { OR_CHUNKS = 256 };

/* sum_i a[i] b[i] (b == NULL: sum_i a[i]) over OR_CHUNKS contiguous chunks,
 * each summed in order by one thread, then the chunk sums in order */
static double chunked_sum(int64_t n, const double *a, const double *b)
{
    double part[OR_CHUNKS];
#pragma omp parallel for schedule(static)
    for (int c = 0; c < OR_CHUNKS; ++c) {
        int64_t i0 = n * c / OR_CHUNKS, i1 = n * (c + 1) / OR_CHUNKS;
        double s = 0.0;
        if (b)
            for (int64_t i = i0; i < i1; ++i) s += a[i] * b[i];
        else
            for (int64_t i = i0; i < i1; ++i) s += a[i];
        part[c] = s;
    }
    double s = 0.0;
    for (int c = 0; c < OR_CHUNKS; ++c) s += part[c];
    return s;
}
#endif

static double dot(int64_t n, const double *a, const double *b)
{
#ifdef _OPENMP
    return chunked_sum(n, a, b);
#else
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
#endif
}

/* v <- v - mean(v) * 1; returns the mean removed */
static double remove_mean(int64_t n, double *v)
{
#ifdef _OPENMP
    double mean = chunked_sum(n, v, NULL);
#else
    double mean = 0.0;
    for (int64_t i = 0; i < n; ++i) mean += v[i];
#endif
    mean /= (double)n;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) v[i] -= mean;
    return mean;
}

/* Thread count of the timing build (ignored by the plain build) and the wall
 * time of the last PCG iteration loop (set-up and elimination excluded). */
static double g_loop_seconds = 0.0;

void or_set_threads(int threads)
{
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
}

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

double or_last_loop_seconds(void) { return g_loop_seconds; }

static double wall_seconds(void)
{
    struct timespec t;
    clock_gettime(CLOCK_MONOTONIC, &t);
    return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

/* ------------------------------------------------------------------------ */
/* Dirichlet elimination                                                     */
/* ------------------------------------------------------------------------ */

/* Symmetric elimination of homogeneous Dirichlet nodes: a Dirichlet row
 * becomes the identity row, and every entry in a Dirichlet column of a free
 * row is removed, so the free block is unchanged and the matrix stays
 * symmetric.  dirichlet[i] != 0 marks node i. */
or_csr *or_eliminate(const or_csr *A, const uint8_t *dirichlet)
{
    or_csr *E = calloc(1, sizeof(or_csr));
    if (!E) return NULL;
    int64_t n = A->n;
    E->n = n;
    E->rowptr = malloc(sizeof(int64_t) * (size_t)(n + 1));
    E->col = malloc(sizeof(int32_t) * (size_t)(A->nnz > 0 ? A->nnz : 1) + sizeof(int32_t) * (size_t)n);
    E->val = malloc(sizeof(double) * (size_t)(A->nnz > 0 ? A->nnz : 1) + sizeof(double) * (size_t)n);
    if (!E->rowptr || !E->col || !E->val) {
        or_csr_free(E);
        return NULL;
    }
    int64_t k = 0;
    E->rowptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (dirichlet && dirichlet[i]) {
            E->col[k] = (int32_t)i;
            E->val[k] = 1.0;
            ++k;
        } else {
            for (int64_t s = A->rowptr[i]; s < A->rowptr[i + 1]; ++s) {
                int32_t c = A->col[s];
                if (dirichlet && dirichlet[c]) continue;
                E->col[k] = c;
                E->val[k] = A->val[s];
                ++k;
            }
        }
        E->rowptr[i + 1] = k;
    }
    E->nnz = k;
    return E;
}

/* ------------------------------------------------------------------------ */
/* Tridiagonal solve of one water column                                     */
/* ------------------------------------------------------------------------ */

/* Solves T z = r for the symmetric tridiagonal T of order L with diagonal
 * d[0..L-1] and off-diagonal e[0..L-2] (T[k][k+1] = T[k+1][k] = e[k]) by
 * Gaussian elimination from the top of the column down, then substitution
 * from the bottom up (the Thomas algorithm, no pivoting: T is symmetric
 * positive definite here).  Every division is a product with the inverse
 * pivot w[k] = 1 / u[k], so that L = 1 gives z = (1 / d) r exactly as the
 * point Jacobi preconditioner does.  work holds L doubles.  Returns
 * OR_ERR_BREAKDOWN on a non-positive pivot. */
int or_tridiag_solve(int64_t L, const double *d, const double *e, const double *r, double *z,
                     double *work)
{
    double *w = work;
    double u = d[0];
    if (!(u > 0.0)) return OR_ERR_BREAKDOWN;
    w[0] = 1.0 / u;
    z[0] = r[0] * w[0];
    for (int64_t k = 1; k < L; ++k) {
        double c = e[k - 1] * w[k - 1]; /* multiplier of row k-1 */
        u = d[k] - e[k - 1] * c;
        if (!(u > 0.0)) return OR_ERR_BREAKDOWN;
        w[k] = 1.0 / u;
        z[k] = (r[k] - e[k - 1] * z[k - 1]) * w[k];
    }
    for (int64_t k = L - 2; k >= 0; --k) z[k] = z[k] - (e[k] * w[k]) * z[k + 1];
    return OR_OK;
}

/* Column blocks of A: for nodes i = c L + k (column c, level k), ld[i] =
 * A[i][i] and le[i] = A[i][i+1] when i+1 is in the same column, else 0. */
static void column_blocks(const or_csr *A, int64_t L, double *ld, double *le)
{
    for (int64_t i = 0; i < A->n; ++i) {
        ld[i] = 0.0;
        le[i] = 0.0;
        int last = (i % L) == L - 1;
        for (int64_t s = A->rowptr[i]; s < A->rowptr[i + 1]; ++s) {
            if (A->col[s] == i) ld[i] = A->val[s];
            if (!last && A->col[s] == i + 1) le[i] = A->val[s];
        }
    }
}

/* The preconditioner of a PCG run: the inverse diagonal, the inverse of the
 * column blocks (line_len >= 1), or IC(0) in the multicolour order (L set). */
typedef struct {
    int64_t line_len;
    const double *dinv, *ld, *le;
    double *work;
    const or_csr *L;
    const int32_t *perm;
    double *y;
} prec_t;

static int apply_prec_line(int64_t n, int64_t line_len, const double *dinv, const double *ld,
                           const double *le, const double *r, double *z, double *work);
static void ic0_apply(const or_csr *L, const int32_t *perm, const double *r, double *z,
                      double *y);

static int apply_prec(int64_t n, const prec_t *P, const double *r, double *z)
{
    if (P->L) {
        ic0_apply(P->L, P->perm, r, z, P->y);
        return OR_OK;
    }
    return apply_prec_line(n, P->line_len, P->dinv, P->ld, P->le, r, z, P->work);
}

/* z = M^-1 r: the inverse diagonal (line_len == 0) or the inverse of the
 * column blocks (line_len >= 1). */
static int apply_prec_line(int64_t n, int64_t line_len, const double *dinv, const double *ld,
                           const double *le, const double *r, double *z, double *work)
{
    if (line_len == 0) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
        return OR_OK;
    }
    for (int64_t c0 = 0; c0 < n; c0 += line_len) {
        int st = or_tridiag_solve(line_len, ld + c0, le + c0, r + c0, z + c0, work);
        if (st != OR_OK) return st;
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Incomplete Cholesky IC(0) in a multicolour ordering                       */
/* ------------------------------------------------------------------------ */

/* Greedy colouring of the matrix graph in node order: node i takes the
 * smallest colour not taken by a neighbour j < i (j != i with A_ij stored).
 * Returns the number of colours. */
int or_greedy_colors(const or_csr *A, int32_t *color)
{
    int64_t n = A->n;
    int32_t ncol = 0;
    char *used = calloc(64, 1);
    if (!used) return OR_ERR_NOMEM;
    for (int64_t i = 0; i < n; ++i) {
        memset(used, 0, 64);
        for (int64_t s = A->rowptr[i]; s < A->rowptr[i + 1]; ++s) {
            int32_t j = A->col[s];
            if (j < i && color[j] < 64) used[color[j]] = 1;
        }
        int32_t c = 0;
        while (c < 64 && used[c]) ++c;
        if (c >= 64) {
            free(used);
            return OR_ERR_INVALID;
        }
        color[i] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    free(used);
    return ncol;
}

/* The multicolour permutation: nodes sorted by (colour, node); perm[k] is
 * the node at position k, iperm its inverse. */
static void color_order(int64_t n, const int32_t *color, int32_t ncol, int32_t *perm,
                        int32_t *iperm)
{
    int64_t k = 0;
    for (int32_t c = 0; c < ncol; ++c)
        for (int64_t i = 0; i < n; ++i)
            if (color[i] == c) {
                perm[k] = (int32_t)i;
                iperm[i] = (int32_t)k;
                ++k;
            }
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* IC(0) of B = P A P^T (P the permutation above): lower triangular L with the
 * pattern of the lower triangle of B such that (L L^T)_ij = B_ij on that
 * pattern, computed row by row:
 *   L_ij = (B_ij - sum_{k < j} L_ik L_jk) / L_jj     for j < i in the pattern,
 *   L_ii = sqrt(B_ii - sum_{k < i} L_ik^2),
 * the sums running over the stored entries of both rows.  Output: CSR of L
 * (row i of B's order, ascending columns, the diagonal last).  Returns
 * OR_ERR_BREAKDOWN when a pivot is not positive. */
int or_ic0(const or_csr *A, const int32_t *perm, const int32_t *iperm, or_csr **Lout)
{
    *Lout = NULL;
    int64_t n = A->n;
    or_csr *L = calloc(1, sizeof(or_csr));
    if (!L) return OR_ERR_NOMEM;
    L->n = n;
    L->rowptr = malloc(sizeof(int64_t) * (size_t)(n + 1));
    /* lower pattern of B, rows of B in order */
    int64_t cap = A->nnz + n;
    L->col = malloc(sizeof(int32_t) * (size_t)cap);
    L->val = malloc(sizeof(double) * (size_t)cap);
    int32_t *tmpc = malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!L->rowptr || !L->col || !L->val || !tmpc) {
        free(tmpc);
        or_csr_free(L);
        return OR_ERR_NOMEM;
    }
    int64_t k = 0;
    L->rowptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t row = perm[i];
        int64_t m = 0;
        for (int64_t s = A->rowptr[row]; s < A->rowptr[row + 1]; ++s) {
            int32_t j = iperm[A->col[s]];
            if (j < i) tmpc[m++] = j;
        }
        qsort(tmpc, (size_t)m, sizeof(int32_t), cmp_i32);
        for (int64_t t = 0; t < m; ++t) L->col[k + t] = tmpc[t];
        L->col[k + m] = (int32_t)i;
        k += m + 1;
        L->rowptr[i + 1] = k;
    }
    L->nnz = k;
    free(tmpc);
    /* values row by row */
    for (int64_t i = 0; i < n; ++i) {
        int64_t row = perm[i];
        int64_t b0 = L->rowptr[i], b1 = L->rowptr[i + 1] - 1; /* strict lower [b0, b1) */
        double diag = 0.0;
        for (int64_t s = A->rowptr[row]; s < A->rowptr[row + 1]; ++s)
            if (A->col[s] == row) diag = A->val[s];
        for (int64_t t = b0; t < b1; ++t) {
            int32_t j = L->col[t];
            double bij = 0.0;
            for (int64_t s = A->rowptr[row]; s < A->rowptr[row + 1]; ++s)
                if (iperm[A->col[s]] == j) bij = A->val[s];
            /* sum over k < j common to rows i (entries b0..t-1) and j */
            double sum = 0.0;
            int64_t u = b0, v = L->rowptr[j], vend = L->rowptr[j + 1] - 1;
            while (u < t && v < vend) {
                if (L->col[u] == L->col[v]) {
                    sum += L->val[u] * L->val[v];
                    ++u;
                    ++v;
                } else if (L->col[u] < L->col[v]) {
                    ++u;
                } else {
                    ++v;
                }
            }
            L->val[t] = (bij - sum) / L->val[L->rowptr[j + 1] - 1];
        }
        double d = diag;
        for (int64_t t = b0; t < b1; ++t) d -= L->val[t] * L->val[t];
        if (!(d > 0.0)) {
            or_csr_free(L);
            return OR_ERR_BREAKDOWN;
        }
        L->val[b1] = sqrt(d);
    }
    *Lout = L;
    return OR_OK;
}

/* z = P^T (L L^T)^-1 P r: forward substitution with L, backward with L^T
 * (column-oriented over the rows of L), in the permuted order. */
static void ic0_apply(const or_csr *L, const int32_t *perm, const double *r, double *z,
                      double *y)
{
    int64_t n = L->n;
    for (int64_t i = 0; i < n; ++i) {
        double s = r[perm[i]];
        int64_t d = L->rowptr[i + 1] - 1;
        for (int64_t t = L->rowptr[i]; t < d; ++t) s -= L->val[t] * y[L->col[t]];
        y[i] = s / L->val[d];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        int64_t d = L->rowptr[i + 1] - 1;
        y[i] /= L->val[d];
        for (int64_t t = L->rowptr[i]; t < d; ++t) y[L->col[t]] -= L->val[t] * y[i];
    }
    for (int64_t i = 0; i < n; ++i) z[perm[i]] = y[i];
}

/* ------------------------------------------------------------------------ */
/* Jacobi-preconditioned conjugate gradient                                  */
/* ------------------------------------------------------------------------ */

/* Solves A x = b for the symmetric positive (semi-)definite matrix A after
 * eliminating the nodes flagged in `dirichlet` (may be NULL), using
 * conjugate gradients preconditioned by the inverse diagonal.
 *
 * singular != 0: A is the pure-Neumann pressure operator, whose null space is
 * the constants; b is first projected onto the zero-sum vectors (its mean is
 * returned in *removed_mean), every residual computed as b - A x is projected
 * the same way (rounding in A x leaves a small constant part that CG on the
 * singular system could not remove), and, after convergence, the solution is
 * shifted so that its mass-weighted mean sum(m_i x_i) / sum(m_i) is zero,
 * where m = `weights` (the row sums of the mass matrix).  This stands in for
 * the zero-mean constraint of the pressure increment (Sec. 4, q in H^1/R;
 * Remark 2 at the end of Sec. 5).
 *
 * Stopping rule: ||b - A x||_2 <= tol * ||b||_2 for the true residual; the
 * recursively updated residual triggers the check and, if the true residual
 * is still too large, replaces the recursive one (restart).  A tolerance
 * below the rounding floor of the problem would restart forever: after three
 * failed checks in a row none of which halved the smallest true residual
 * seen at a check, the solve ends with OR_NOT_CONVERGED.
 *
 * x holds the initial guess on entry (Dirichlet entries are ignored and set to
 * zero) and the last iterate on exit.  alpha_hist / beta_hist / x_hist may be
 * NULL; otherwise they receive the step lengths, the direction updates and the
 * iterates (maxit rows of n) of each iteration.
 *
 * line_len = 0 selects the inverse diagonal; line_len = L >= 1 selects the
 * inverse of the tridiagonal blocks of the eliminated matrix on the columns
 * {c L, ..., c L + L - 1} (the water columns of the vertical-first node
 * numbering; n must be a multiple of L), applied by or_tridiag_solve.
 * or_pcg is or_pcg_line with line_len = 0.
 */
static int pcg_core(const or_csr *A0, const uint8_t *dirichlet, int singular,
                    const double *weights, const double *b0, double *x, double tol, int maxit,
                    int64_t line_len, int ic0, int *iters_out, double *relres_out,
                    double *removed_mean, double *alpha_hist, double *beta_hist,
                    double *x_hist)
{
    int64_t n = A0->n;
    g_loop_seconds = 0.0;
    if (line_len < 0 || (line_len > 0 && n % line_len != 0)) return OR_ERR_INVALID;
    *iters_out = 0;
    *relres_out = 0.0;
    if (removed_mean) *removed_mean = 0.0;
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(b0[i])) return OR_ERR_INVALID;

    or_csr *A = or_eliminate(A0, dirichlet);
    double *b = malloc(sizeof(double) * (size_t)n);
    double *r = malloc(sizeof(double) * (size_t)n);
    double *z = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n);
    double *q = malloc(sizeof(double) * (size_t)n);
    double *dinv = malloc(sizeof(double) * (size_t)n);
    double *ld = line_len ? malloc(sizeof(double) * (size_t)n) : NULL;
    double *le = line_len ? malloc(sizeof(double) * (size_t)n) : NULL;
    double *work = line_len ? malloc(sizeof(double) * (size_t)line_len) : NULL;
    int32_t *color = ic0 ? malloc(sizeof(int32_t) * (size_t)n) : NULL;
    int32_t *perm = ic0 ? malloc(sizeof(int32_t) * (size_t)n) : NULL;
    int32_t *iperm = ic0 ? malloc(sizeof(int32_t) * (size_t)n) : NULL;
    double *ywork = ic0 ? malloc(sizeof(double) * (size_t)n) : NULL;
    or_csr *L = NULL;
    prec_t P;
    int status = OR_NOT_CONVERGED;
    if (!A || !b || !r || !z || !p || !q || !dinv || (line_len && (!ld || !le || !work)) ||
        (ic0 && (!color || !perm || !iperm || !ywork))) {
        status = OR_ERR_NOMEM;
        goto done;
    }
    for (int64_t i = 0; i < n; ++i) {
        int dir = dirichlet && dirichlet[i];
        b[i] = dir ? 0.0 : b0[i];
        if (dir) x[i] = 0.0;
    }
    if (singular) {
        double mean = remove_mean(n, b);
        if (removed_mean) *removed_mean = mean;
    }
    for (int64_t i = 0; i < n; ++i) {
        double d = 0.0;
        for (int64_t s = A->rowptr[i]; s < A->rowptr[i + 1]; ++s)
            if (A->col[s] == i) d = A->val[s];
        if (!(d > 0.0)) {
            status = OR_ERR_BREAKDOWN;
            goto done;
        }
        dinv[i] = 1.0 / d;
    }
    if (line_len) column_blocks(A, line_len, ld, le);
    if (ic0) {
        int ncol = or_greedy_colors(A, color);
        if (ncol < 0) {
            status = ncol;
            goto done;
        }
        color_order(n, color, ncol, perm, iperm);
        if ((status = or_ic0(A, perm, iperm, &L)) != OR_OK) goto done;
        status = OR_NOT_CONVERGED;
    }
    P.line_len = line_len;
    P.dinv = dinv;
    P.ld = ld;
    P.le = le;
    P.work = work;
    P.L = L;
    P.perm = perm;
    P.y = ywork;
    double bnorm = sqrt(dot(n, b, b));
    if (bnorm == 0.0) {
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        status = OR_OK;
        goto done;
    }
    const double t_loop = wall_seconds();
    or_spmv(A, x, q);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    if (singular) remove_mean(n, r);
    if ((status = apply_prec(n, &P, r, z)) != OR_OK) goto done;
    status = OR_NOT_CONVERGED;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) p[i] = z[i];
    double rho = dot(n, r, z);
    double relres = sqrt(dot(n, r, r)) / bnorm;
    if (relres <= tol) {
        status = OR_OK;
        *relres_out = relres;
        goto normalize;
    }
    int it = 0, stalled = 0;
    double best_true = INFINITY;
    while (it < maxit) {
        or_spmv(A, p, q);
        double gamma = dot(n, p, q);
        if (!(gamma > 0.0) || !isfinite(gamma)) {
            status = OR_ERR_BREAKDOWN;
            break;
        }
        double alpha = rho / gamma;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) x[i] += alpha * p[i];
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) r[i] -= alpha * q[i];
        if (alpha_hist) alpha_hist[it] = alpha;
        if (x_hist) memcpy(x_hist + (int64_t)it * n, x, sizeof(double) * (size_t)n);
        ++it;
        relres = sqrt(dot(n, r, r)) / bnorm;
        if (relres <= tol) {
            or_spmv(A, x, q);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) q[i] = b[i] - q[i];
            if (singular) remove_mean(n, q);
            double true_rel = sqrt(dot(n, q, q)) / bnorm;
            if (true_rel <= tol) {
                relres = true_rel;
                status = OR_OK;
                if (beta_hist) beta_hist[it - 1] = 0.0;
                break;
            }
            /* The rounding floor: three failed checks in a row that do not
             * halve the best true residual so far end the solve. */
            stalled = (true_rel > 0.5 * best_true) ? stalled + 1 : 0;
            if (true_rel < best_true) best_true = true_rel;
            if (stalled >= 3) {
                relres = true_rel;
                if (beta_hist) beta_hist[it - 1] = 0.0;
                break;
            }
            /* restart from the true residual */
            memcpy(r, q, sizeof(double) * (size_t)n);
            if ((status = apply_prec(n, &P, r, z)) != OR_OK) break;
            status = OR_NOT_CONVERGED;
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) p[i] = z[i];
            rho = dot(n, r, z);
            relres = true_rel;
            if (beta_hist) beta_hist[it - 1] = 0.0;
            continue;
        }
        if ((status = apply_prec(n, &P, r, z)) != OR_OK) break;
        status = OR_NOT_CONVERGED;
        double rho_new = dot(n, r, z);
        double beta = rho_new / rho;
        if (beta_hist) beta_hist[it - 1] = beta;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        rho = rho_new;
    }
    g_loop_seconds = wall_seconds() - t_loop;
    *iters_out = it;
    *relres_out = relres;
normalize:
    if (singular && status >= 0 && weights) {
        double wx = 0.0, ws = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            wx += weights[i] * x[i];
            ws += weights[i];
        }
        double shift = wx / ws;
        for (int64_t i = 0; i < n; ++i) x[i] -= shift;
    }
done:
    or_csr_free(A);
    free(b);
    free(r);
    free(z);
    free(p);
    free(q);
    free(dinv);
    free(ld);
    free(le);
    free(work);
    free(color);
    free(perm);
    free(iperm);
    free(ywork);
    or_csr_free(L);
    return status;
}

int or_pcg_line(const or_csr *A0, const uint8_t *dirichlet, int singular,
                const double *weights, const double *b0, double *x, double tol,
                int maxit, int64_t line_len, int *iters_out, double *relres_out,
                double *removed_mean, double *alpha_hist, double *beta_hist,
                double *x_hist)
{
    return pcg_core(A0, dirichlet, singular, weights, b0, x, tol, maxit, line_len, 0, iters_out,
                    relres_out, removed_mean, alpha_hist, beta_hist, x_hist);
}

/* PCG with IC(0) of the eliminated matrix in the greedy multicolour order
 * (or_greedy_colors, or_ic0): the preconditioner of Remark 3 at the end of
 * Sec. 5 for the velocity systems, in an order whose triangular solves run
 * colour by colour. */
int or_pcg_ic0(const or_csr *A0, const uint8_t *dirichlet, int singular,
               const double *weights, const double *b0, double *x, double tol, int maxit,
               int *iters_out, double *relres_out, double *removed_mean, double *alpha_hist,
               double *beta_hist, double *x_hist)
{
    return pcg_core(A0, dirichlet, singular, weights, b0, x, tol, maxit, 0, 1, iters_out,
                    relres_out, removed_mean, alpha_hist, beta_hist, x_hist);
}

/* IC(0) factor of the eliminated matrix in the greedy multicolour order:
 * perm (n) receives the order, L the factor (for tests). */
int or_ic0_factor(const or_csr *A0, const uint8_t *dirichlet, int32_t *perm, or_csr **L)
{
    int64_t n = A0->n;
    *L = NULL;
    or_csr *A = or_eliminate(A0, dirichlet);
    int32_t *color = malloc(sizeof(int32_t) * (size_t)n);
    int32_t *iperm = malloc(sizeof(int32_t) * (size_t)n);
    int st = OR_ERR_NOMEM;
    if (A && color && iperm) {
        int ncol = or_greedy_colors(A, color);
        if (ncol < 0) {
            st = ncol;
        } else {
            color_order(n, color, ncol, perm, iperm);
            st = or_ic0(A, perm, iperm, L);
        }
    }
    free(color);
    free(iperm);
    or_csr_free(A);
    return st;
}

int or_pcg(const or_csr *A0, const uint8_t *dirichlet, int singular, const double *weights,
           const double *b0, double *x, double tol, int maxit, int *iters_out,
           double *relres_out, double *removed_mean, double *alpha_hist, double *beta_hist,
           double *x_hist)
{
    return or_pcg_line(A0, dirichlet, singular, weights, b0, x, tol, maxit, 0, iters_out,
                       relres_out, removed_mean, alpha_hist, beta_hist, x_hist);
}

/* True relative residual ||mask(b - A x)|| / ||mask(b)|| with Dirichlet rows
 * removed (a Dirichlet row's equation is x_i = 0, which the caller checks). */
double or_relres(const or_csr *A, const uint8_t *dirichlet, const double *b,
                 const double *x)
{
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < A->n; ++i) {
        if (dirichlet && dirichlet[i]) continue;
        double s = 0.0;
        for (int64_t k = A->rowptr[i]; k < A->rowptr[i + 1]; ++k) {
            int32_t c = A->col[k];
            if (dirichlet && dirichlet[c]) continue;
            s += A->val[k] * x[c];
        }
        double d = b[i] - s;
        num += d * d;
        den += b[i] * b[i];
    }
    return den > 0.0 ? sqrt(num / den) : sqrt(num);
}

/* ------------------------------------------------------------------------ */
/* Dense Cholesky for tiny systems                                           */
/* ------------------------------------------------------------------------ */

/* Solves the dense SPD system A x = b (row-major n x n) by A = L L^T.
 * Returns OR_ERR_BREAKDOWN if a pivot is not positive. */
int or_cholesky_solve(int64_t n, const double *A, const double *b, double *x)
{
    double *L = calloc((size_t)(n * n), sizeof(double));
    double *y = malloc(sizeof(double) * (size_t)n);
    if (!L || !y) {
        free(L);
        free(y);
        return OR_ERR_NOMEM;
    }
    for (int64_t j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int64_t k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
        if (!(s > 0.0)) {
            free(L);
            free(y);
            return OR_ERR_BREAKDOWN;
        }
        L[j * n + j] = sqrt(s);
        for (int64_t i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int64_t k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = t / L[j * n + j];
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        double t = b[i];
        for (int64_t k = 0; k < i; ++k) t -= L[i * n + k] * y[k];
        y[i] = t / L[i * n + i];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
        double t = y[i];
        for (int64_t k = i + 1; k < n; ++k) t -= L[k * n + i] * x[k];
        x[i] = t / L[i * n + i];
    }
    free(L);
    free(y);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Brick elements: Q2 velocity / Q1 pressure spaces of Sec. 5               */
/* ------------------------------------------------------------------------ */

/* Value and derivative at s of the k-th Lagrange polynomial of degree p
 * through the equispaced points t_m = -1 + 2m/p of [-1, 1]:
 * l_k(s) = prod_{m != k} (s - t_m) / (t_k - t_m), differentiated factor by
 * factor with the product rule. */
static void lagrange_1d(int p, int k, double s, double *val, double *der)
{
    double tk = -1.0 + 2.0 * k / p;
    double v = 1.0, d = 0.0;
    for (int m = 0; m <= p; ++m) {
        if (m == k) continue;
        double tm = -1.0 + 2.0 * m / p;
        double f = (s - tm) / (tk - tm);
        d = d * f + v / (tk - tm);
        v = v * f;
    }
    *val = v;
    *der = d;
}

/* Gauss-Legendre rule with p + 1 points on [-1, 1]: 2 points (exact to
 * degree 3) for p = 1, 3 points (exact to degree 5) for p = 2. */
static void gauss_rule(int p, double *x, double *w)
{
    if (p == 1) {
        x[0] = -1.0 / sqrt(3.0);
        x[1] = 1.0 / sqrt(3.0);
        w[0] = w[1] = 1.0;
    } else {
        x[0] = -sqrt(0.6);
        x[1] = 0.0;
        x[2] = sqrt(0.6);
        w[0] = w[2] = 5.0 / 9.0;
        w[1] = 8.0 / 9.0;
    }
}

static double det3(const double A[3][3])
{
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
         - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
         + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

/* Solves A g = r by Cramer's rule (det(A) given). */
static void cramer3(const double A[3][3], double detA, const double *r, double *g)
{
    for (int k = 0; k < 3; ++k) {
        double Ak[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                Ak[i][j] = (j == k) ? r[i] : A[i][j];
        g[k] = det3(Ak) / detA;
    }
}

/* Element matrices of one brick of order p (1: Q1, 2: Q2), Sec. 5.
 *   X8     the 8 corners, corner (c1, c2, c3) in {0,1}^3 at row c1 + 2 c2 + 4 c3
 *   nu     (nu_1, nu_2, nu_3) of the anisotropic stiffness
 *   K, M   nloc x nloc row-major, nloc = (p+1)^3, local node (a, b, c) (each
 *          0..p, reference point (t_a, t_b, t_c)) at a + (p+1) b + (p+1)^2 c
 * The element is the image of the reference cube [-1,1]^3 under the trilinear
 * map through its corners; the basis functions are the products of the 1D
 * Lagrange polynomials of degree p; the integrals use the tensor Gauss rule
 * with p + 1 points per direction (exact for both forms on parallelepipeds).
 *   M_ab = int phi_a phi_b,   K_ab = int sum_d nu_d (d_d phi_a)(d_d phi_b),
 * with the physical gradient g of a basis function obtained from its
 * reference gradient r through J^T g = r, J_rd = d x_r / d s_d.
 * Returns the smallest Jacobian determinant over the quadrature points. */
double or_hex_element(int p, const double *X8, const double *nu, double *K, double *M)
{
    const int q = p + 1, nloc = q * q * q;
    double gx[3], gw[3];
    gauss_rule(p, gx, gw);
    for (int k = 0; k < nloc * nloc; ++k) {
        K[k] = 0.0;
        M[k] = 0.0;
    }
    double detmin = INFINITY;
    double N[27], G[27][3];
    for (int i3 = 0; i3 < q; ++i3)
        for (int i2 = 0; i2 < q; ++i2)
            for (int i1 = 0; i1 < q; ++i1) {
                const double s[3] = {gx[i1], gx[i2], gx[i3]};
                const double w = gw[i1] * gw[i2] * gw[i3];
                double J[3][3] = {{0.0}};
                for (int c = 0; c < 8; ++c) {
                    int cc[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
                    double lin[3], dlin[3];
                    for (int d = 0; d < 3; ++d) {
                        double sg = cc[d] ? 1.0 : -1.0;
                        lin[d] = 0.5 * (1.0 + sg * s[d]);
                        dlin[d] = 0.5 * sg;
                    }
                    double dG[3] = {dlin[0] * lin[1] * lin[2], lin[0] * dlin[1] * lin[2],
                                    lin[0] * lin[1] * dlin[2]};
                    for (int r = 0; r < 3; ++r)
                        for (int d = 0; d < 3; ++d)
                            J[r][d] += X8[3 * c + r] * dG[d];
                }
                double det = det3(J);
                if (det < detmin) detmin = det;
                double JT[3][3];
                for (int r = 0; r < 3; ++r)
                    for (int d = 0; d < 3; ++d)
                        JT[d][r] = J[r][d];
                for (int c = 0; c < q; ++c)
                    for (int b = 0; b < q; ++b)
                        for (int a = 0; a < q; ++a) {
                            double va, da, vb, db, vc, dc;
                            lagrange_1d(p, a, s[0], &va, &da);
                            lagrange_1d(p, b, s[1], &vb, &db);
                            lagrange_1d(p, c, s[2], &vc, &dc);
                            int l = a + q * b + q * q * c;
                            N[l] = va * vb * vc;
                            double ref[3] = {da * vb * vc, va * db * vc, va * vb * dc};
                            cramer3(JT, det, ref, G[l]);
                        }
                for (int a = 0; a < nloc; ++a)
                    for (int b = 0; b < nloc; ++b) {
                        M[a * nloc + b] += w * det * N[a] * N[b];
                        double k = 0.0;
                        for (int d = 0; d < 3; ++d)
                            k += nu[d] * G[a][d] * G[b][d];
                        K[a * nloc + b] += w * det * k;
                    }
            }
    return detmin;
}

/* Assemble c_mass * M + c_stiff * K_nu (nu = (nu_h, nu_h, nu_v)) over a brick
 * mesh of order p: hex holds (p+1)^3 node ids per element in the local order
 * of or_hex_element.  An element whose Jacobian determinant is not positive
 * at every quadrature point is a mesh error. */
int or_assemble_hex(int64_t n, const double *xyz, int64_t nhex, const int32_t *hex, int p,
                    double nu_h, double nu_v, double c_mass, double c_stiff, or_csr **out)
{
    *out = NULL;
    if (n <= 0 || nhex < 0 || (p != 1 && p != 2)) return OR_ERR_INVALID;
    const int q = p + 1, nloc = q * q * q;
    if (check_conn(n, nhex, nloc, hex) != OR_OK) return OR_ERR_MESH;
    triplets t;
    memset(&t, 0, sizeof(t));
    if (trip_init(&t, n, nhex, nloc, hex) != OR_OK) {
        trip_free(&t);
        return OR_ERR_NOMEM;
    }
    const double nu[3] = {nu_h, nu_h, nu_v};
    double *K = malloc(sizeof(double) * nloc * nloc);
    double *M = malloc(sizeof(double) * nloc * nloc);
    if (!K || !M) {
        free(K);
        free(M);
        trip_free(&t);
        return OR_ERR_NOMEM;
    }
    int st = OR_OK;
    for (int64_t e = 0; e < nhex && st == OR_OK; ++e) {
        const int32_t *h = hex + e * nloc;
        double X8[24];
        for (int c = 0; c < 8; ++c) {
            int l = (c & 1) * p + q * (((c >> 1) & 1) * p) + q * q * ((c >> 2) * p);
            for (int d = 0; d < 3; ++d)
                X8[3 * c + d] = xyz[(int64_t)h[l] * 3 + d];
        }
        if (!(or_hex_element(p, X8, nu, K, M) > 0.0)) {
            st = OR_ERR_MESH;
            break;
        }
        for (int a = 0; a < nloc; ++a)
            for (int b = 0; b < nloc; ++b)
                trip_add(&t, h[a], h[b], c_mass * M[a * nloc + b] + c_stiff * K[a * nloc + b]);
    }
    free(K);
    free(M);
    if (st == OR_OK) {
        *out = trip_to_csr(&t);
        if (!*out) st = OR_ERR_NOMEM;
    }
    trip_free(&t);
    return st;
}
