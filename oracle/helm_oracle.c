/*
 * helm_oracle.c -- plain FP64 CPU oracle for the discrete Helmholtz problem.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU product path links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP library.
 *
 * What it computes (Appendix A.1 of the paper, "Numerical forward model"):
 *   P1 finite elements on a uniform rectangular grid split into triangles,
 *   with nodal quadrature, give
 *       A(m, w) = S - w^2 M(m) - i w B(m),
 *   S the stiffness matrix (equal to the five-point Laplacian with halved
 *   couplings along boundary edges), M = diag(d_k m_k), B = diag(b_k sqrt(m_k)).
 *   The wavefield of a grid-point source s solves A u = e_s; the adjoint
 *   problem is solved with A^* (conjugate transpose).
 *
 * The solve is the plain definition: Gaussian elimination with partial
 * (row) pivoting on the banded matrix (lower and upper bandwidth n_x), stored
 * in LAPACK-style band format, followed by forward/back substitution.  The
 * adjoint solve applies the conjugate-transposed factors.  No blocking.
 *
 * Grid: node k = j*nx + i, x_i = i*hx, z_j = j*hz, j = 0 is the top row.
 * Readings where the paper is silent (stated again in the Python wrapper):
 *   - corner mass weight d = hx*hz/4 (the average of the two triangulation
 *     directions; interior hx*hz, edges hx*hz/2 as in P1 lumping);
 *   - b_k = sum over boundary edges touching node k of half the edge length.
 *
 * Complex numbers are stored interleaved (re, im) as double[2].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double re, im; } cplx;

static inline cplx cmul(cplx a, cplx b) { cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; return r; }
static inline cplx cconj(cplx a) { cplx r = {a.re, -a.im}; return r; }
static inline cplx csub(cplx a, cplx b) { cplx r = {a.re - b.re, a.im - b.im}; return r; }
static inline double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }
static inline cplx cdiv(cplx a, cplx b) {
    /* plain definition a * conj(b) / |b|^2 */
    double den = cabs2(b);
    cplx r = {(a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den};
    return r;
}

/* ------------------------------------------------------------------------ */
/* Quadrature weights (App. A.1): M = diag(d_k m_k), B = diag(b_k sqrt(m_k)) */
/* ------------------------------------------------------------------------ */
static double end_half(int idx, int n) { return (idx == 0 || idx == n - 1) ? 0.5 : 1.0; }

void or_weights(int nx, int nz, double hx, double hz, double* d, double* b) {
    for (int j = 0; j < nz; ++j)
        for (int i = 0; i < nx; ++i) {
            int k = j * nx + i;
            d[k] = hx * hz * end_half(i, nx) * end_half(j, nz);
            double bk = 0.0;
            /* boundary edges along the top and bottom rows (length hx) */
            if (j == 0 || j == nz - 1) {
                if (i > 0) bk += 0.5 * hx;
                if (i < nx - 1) bk += 0.5 * hx;
            }
            /* boundary edges along the left and right columns (length hz) */
            if (i == 0 || i == nx - 1) {
                if (j > 0) bk += 0.5 * hz;
                if (j < nz - 1) bk += 0.5 * hz;
            }
            b[k] = bk;
        }
}

/* Stiffness coupling of a grid edge: hz/hx for an x-edge, hx/hz for a z-edge,
 * halved when the edge lies on the boundary (only one triangle touches it). */
static double xedge_coef(int j, int nz, double hx, double hz) { return (hz / hx) * end_half(j, nz); }
static double zedge_coef(int i, int nx, double hx, double hz) { return (hx / hz) * end_half(i, nx); }

/* Entries of A(m, w) row by row, as a list of (col, value) per row: diag and
 * the four neighbours.  Used for the band fill and for y = A x. */
static int row_entries(int nx, int nz, double hx, double hz, const double* m, double w,
                       const double* d, const double* b, int k, int* cols, cplx* vals) {
    int i = k % nx, j = k / nx, cnt = 0;
    double sdiag = 0.0;
    if (i > 0)      { double c = xedge_coef(j, nz, hx, hz); cols[cnt] = k - 1;  vals[cnt].re = -c; vals[cnt].im = 0; cnt++; sdiag += c; }
    if (i < nx - 1) { double c = xedge_coef(j, nz, hx, hz); cols[cnt] = k + 1;  vals[cnt].re = -c; vals[cnt].im = 0; cnt++; sdiag += c; }
    if (j > 0)      { double c = zedge_coef(i, nx, hx, hz); cols[cnt] = k - nx; vals[cnt].re = -c; vals[cnt].im = 0; cnt++; sdiag += c; }
    if (j < nz - 1) { double c = zedge_coef(i, nx, hx, hz); cols[cnt] = k + nx; vals[cnt].re = -c; vals[cnt].im = 0; cnt++; sdiag += c; }
    cols[cnt] = k;
    vals[cnt].re = sdiag - w * w * d[k] * m[k];
    vals[cnt].im = -w * b[k] * sqrt(m[k]);
    cnt++;
    return cnt;
}

/* y = A x (conj_flag = 0) or y = A^* x (conj_flag = 1), for S columns of length N. */
void or_apply(int nx, int nz, double hx, double hz, const double* m, double w, int conj_flag,
              int S, const double* x, double* y) {
    int N = nx * nz;
    double* d = (double*)malloc(sizeof(double) * N);
    double* b = (double*)malloc(sizeof(double) * N);
    or_weights(nx, nz, hx, hz, d, b);
    const cplx* X = (const cplx*)x;
    cplx* Y = (cplx*)y;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < N; ++k) {
        int cols[5]; cplx vals[5];
        int cnt = row_entries(nx, nz, hx, hz, m, w, d, b, k, cols, vals);
        if (conj_flag) for (int t = 0; t < cnt; ++t) vals[t] = cconj(vals[t]);   /* A symmetric: A^* = conj(A) */
        for (int s = 0; s < S; ++s) {
            cplx acc = {0.0, 0.0};
            for (int t = 0; t < cnt; ++t) {
                cplx p = cmul(vals[t], X[(size_t)s * N + cols[t]]);
                acc.re += p.re; acc.im += p.im;
            }
            Y[(size_t)s * N + k] = acc;
        }
    }
    free(d); free(b);
}

/* ------------------------------------------------------------------------ */
/* Band storage: A(r, c) lives at ab[c*ldab + (kl + ku + r - c)], with        */
/* kl = ku = nx and ldab = 2*kl + ku + 1 (kl extra rows for pivoting fill).  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int nx, nz, N, kl, ku, ldab;
    cplx* ab;
    int* ipiv;
} or_band;

static inline cplx* AB(or_band* f, int r, int c) { return &f->ab[(size_t)c * f->ldab + (f->kl + f->ku + r - c)]; }

size_t or_band_bytes(int nx, int nz) {
    size_t N = (size_t)nx * nz, ldab = 3 * (size_t)nx + 1;
    return ldab * N * sizeof(cplx) + N * sizeof(int);
}

/* Factor A = P L U by Gaussian elimination with partial pivoting.
 * Returns 0, or (1 + column) of the first exactly-zero pivot. */
static int band_factor(or_band* f) {
    int N = f->N, kl = f->kl, ku = f->ku;
    for (int c = 0; c < N; ++c) {
        /* pivot search: the largest |entry| of column c on or below the diagonal */
        int last = c + kl < N - 1 ? c + kl : N - 1;
        int p = c;
        double best = cabs2(*AB(f, c, c));
        for (int r = c + 1; r <= last; ++r) {
            double v = cabs2(*AB(f, r, c));
            if (v > best) { best = v; p = r; }
        }
        f->ipiv[c] = p;
        if (best == 0.0) return c + 1;
        /* columns touched by the pivot row: up to c + kl + ku */
        int clast = c + kl + ku < N - 1 ? c + kl + ku : N - 1;
        if (p != c)
            for (int cc = c; cc <= clast; ++cc) {
                cplx t = *AB(f, c, cc); *AB(f, c, cc) = *AB(f, p, cc); *AB(f, p, cc) = t;
            }
        cplx piv = *AB(f, c, c);
        for (int r = c + 1; r <= last; ++r) *AB(f, r, c) = cdiv(*AB(f, r, c), piv);   /* multipliers l_rc */
        /* rank-one update of the active window; columns are independent */
#pragma omp parallel for schedule(static) if (clast - c > 64)
        for (int cc = c + 1; cc <= clast; ++cc) {
            cplx u = *AB(f, c, cc);
            if (u.re == 0.0 && u.im == 0.0) continue;
            for (int r = c + 1; r <= last; ++r) *AB(f, r, cc) = csub(*AB(f, r, cc), cmul(*AB(f, r, c), u));
        }
    }
    return 0;
}

/* Solve A x = rhs (trans = 0) or A^* x = rhs (trans = 1) in place, one column. */
static void band_solve_one(const or_band* fc, int trans, cplx* x) {
    or_band* f = (or_band*)fc;
    int N = f->N, kl = f->kl, ku = f->ku, w = kl + ku;
    if (!trans) {
        /* L y = P b: interchanges interleaved with the column eliminations */
        for (int c = 0; c < N; ++c) {
            int p = f->ipiv[c];
            if (p != c) { cplx t = x[c]; x[c] = x[p]; x[p] = t; }
            int last = c + kl < N - 1 ? c + kl : N - 1;
            for (int r = c + 1; r <= last; ++r) x[r] = csub(x[r], cmul(*AB(f, r, c), x[c]));
        }
        /* U x = y, back substitution (U has upper bandwidth kl + ku) */
        for (int c = N - 1; c >= 0; --c) {
            x[c] = cdiv(x[c], *AB(f, c, c));
            int first = c - w > 0 ? c - w : 0;
            for (int r = first; r < c; ++r) x[r] = csub(x[r], cmul(*AB(f, r, c), x[c]));
        }
    } else {
        /* A^* = U^* L^* P^T : first U^* y = b (forward substitution) */
        for (int c = 0; c < N; ++c) {
            int first = c - w > 0 ? c - w : 0;
            cplx acc = x[c];
            for (int r = first; r < c; ++r) acc = csub(acc, cmul(cconj(*AB(f, r, c)), x[r]));
            x[c] = cdiv(acc, cconj(*AB(f, c, c)));
        }
        /* then L^* z = y backwards, undoing the interchanges in reverse order */
        for (int c = N - 1; c >= 0; --c) {
            int last = c + kl < N - 1 ? c + kl : N - 1;
            cplx acc = x[c];
            for (int r = c + 1; r <= last; ++r) acc = csub(acc, cmul(cconj(*AB(f, r, c)), x[r]));
            x[c] = acc;
            int p = f->ipiv[c];
            if (p != c) { cplx t = x[c]; x[c] = x[p]; x[p] = t; }
        }
    }
}

/* Opaque factor handle for the Python wrapper. */
void* or_factor(int nx, int nz, double hx, double hz, const double* m, double w, int* status) {
    or_band* f = (or_band*)calloc(1, sizeof(or_band));
    if (!f) { *status = -2; return NULL; }
    f->nx = nx; f->nz = nz; f->N = nx * nz; f->kl = nx; f->ku = nx; f->ldab = 2 * nx + nx + 1;
    f->ab = (cplx*)calloc((size_t)f->ldab * f->N, sizeof(cplx));
    f->ipiv = (int*)malloc(sizeof(int) * f->N);
    if (!f->ab || !f->ipiv) { free(f->ab); free(f->ipiv); free(f); *status = -2; return NULL; }
    double* d = (double*)malloc(sizeof(double) * f->N);
    double* b = (double*)malloc(sizeof(double) * f->N);
    or_weights(nx, nz, hx, hz, d, b);
    for (int k = 0; k < f->N; ++k) {
        int cols[5]; cplx vals[5];
        int cnt = row_entries(nx, nz, hx, hz, m, w, d, b, k, cols, vals);
        for (int t = 0; t < cnt; ++t) *AB(f, k, cols[t]) = vals[t];
    }
    free(d); free(b);
    int info = band_factor(f);
    *status = info;
    return f;
}

void or_factor_free(void* h) {
    or_band* f = (or_band*)h;
    if (!f) return;
    free(f->ab); free(f->ipiv); free(f);
}

/* X[s] = A^{-1} B[s] (trans = 0) or A^{-*} B[s] (trans = 1), S columns of length N. */
void or_solve(void* h, int trans, int S, const double* B, double* X) {
    or_band* f = (or_band*)h;
    size_t N = (size_t)f->N;
    memcpy(X, B, sizeof(cplx) * N * (size_t)S);
#pragma omp parallel for schedule(dynamic, 1)
    for (int s = 0; s < S; ++s) band_solve_one(f, trans, (cplx*)X + (size_t)s * N);
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
