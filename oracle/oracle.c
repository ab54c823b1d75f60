/*
 * oracle.c -- plain FP64 CPU reference for the batched partitioned
 * tridiagonal solves (PDD and PPT) of Ha, Park & You, "A scalable multi-GPU
 * method for semi-implicit fractional-step integration of incompressible
 * Navier-Stokes equations" (arXiv:1812.01178).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the tests, the smoke check and the benchmark's CPU
 * baseline load it.  It shares no code, header or table with the HIP path.
 *
 * Written for readability, not speed: every partition block is copied out,
 * every spike is a separate Thomas solve, the reduced system is assembled as
 * a dense matrix and solved by dense Gaussian elimination with partial
 * pivoting.  Built with -O2 -ffp-contract=off (no fused multiply-add).
 *
 * Notation (0-based in code): a line has n rows
 *     a[j] x[j-1] + b[j] x[j] + c[j] x[j+1] = d[j],   j = 0..n-1,
 * split into P partitions of m = n/P rows; partition r owns rows
 * r*m .. r*m+m-1.  For a non-periodic line a[0] and c[n-1] are not part of
 * the matrix and are never read.  For a periodic line a[0] couples row 0 to
 * row n-1 and c[n-1] couples row n-1 to row 0.
 *
 * Interfaces i = 1..P-1 (and i = P, joining partition P-1 to partition 0,
 * when periodic) sit between partition L(i) = i-1 and R(i) = i mod P.  The
 * paper's reduced unknowns y_{2i-1}, y_{2i} (1-based) are stored at 0-based
 * positions 2i-2 and 2i-1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum {
    ORC_OK = 0,
    ORC_E_ARG = 1,
    ORC_E_SHAPE = 2,
    ORC_E_ZERO_PIVOT = 3,
    ORC_E_NOMEM = 7
};

enum { ORC_EXACT = 0, ORC_PDD = 1, ORC_PPT = 2, ORC_EXACT_LD = 3 };

/* ------------------------------------------------------------------------ */
/* Thomas algorithm (textbook, no pivoting).                                 */
/*   c'_0 = c_0/b_0,  d'_0 = d_0/b_0                                         */
/*   c'_j = c_j/(b_j - a_j c'_{j-1}),  d'_j = (d_j - a_j d'_{j-1})/(same)    */
/*   x_{n-1} = d'_{n-1},  x_j = d'_j - c'_j x_{j+1}                          */
/* a[0] and c[n-1] are not read.  cp is caller scratch of length n.          */
/* ------------------------------------------------------------------------ */
int orc_thomas(int64_t n, const double *a, const double *b, const double *c,
               const double *d, double *x, double *cp)
{
    if (n < 1) return ORC_E_SHAPE;
    double den = b[0];
    if (den == 0.0) return ORC_E_ZERO_PIVOT;
    cp[0] = (n > 1 ? c[0] : 0.0) / den;
    x[0] = d[0] / den;
    for (int64_t j = 1; j < n; ++j) {
        den = b[j] - a[j] * cp[j - 1];
        if (den == 0.0) return ORC_E_ZERO_PIVOT;
        cp[j] = (j < n - 1 ? c[j] : 0.0) / den;
        x[j] = (d[j] - a[j] * x[j - 1]) / den;
    }
    for (int64_t j = n - 2; j >= 0; --j)
        x[j] = x[j] - cp[j] * x[j + 1];
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Periodic (cyclic) tridiagonal system, textbook Sherman-Morrison rank-one  */
/* correction of the Thomas algorithm.  This is the plain exact solution of  */
/* a periodic line and is deliberately a different route from the paper's   */
/* partitioned algebra, so it can pin the periodic PDD/PPT code.             */
/*   A = B + u v^T,  u = (g, 0..0, c_{n-1}),  v = (1, 0..0, a_0/g),         */
/*   B = A with b_0 -= g, b_{n-1} -= a_0 c_{n-1}/g and corners removed,     */
/*   x = p - (v.p)/(1 + v.q) q  with  B p = d, B q = u.                     */
/* work: 5n doubles.                                                         */
/* ------------------------------------------------------------------------ */
int orc_cyclic(int64_t n, const double *a, const double *b, const double *c,
               const double *d, double *x, double *work)
{
    if (n < 3) return ORC_E_SHAPE;
    double *bb = work, *u = work + n, *q = work + 2 * n, *cp = work + 3 * n;
    const double alpha = c[n - 1];   /* couples row n-1 to x_0 */
    const double beta = a[0];        /* couples row 0 to x_{n-1} */
    const double g = -b[0];
    for (int64_t j = 0; j < n; ++j) { bb[j] = b[j]; u[j] = 0.0; }
    bb[0] = b[0] - g;
    bb[n - 1] = b[n - 1] - alpha * beta / g;
    u[0] = g;
    u[n - 1] = alpha;
    int st = orc_thomas(n, a, bb, c, d, x, cp);
    if (st) return st;
    st = orc_thomas(n, a, bb, c, u, q, cp);
    if (st) return st;
    const double vx = x[0] + beta / g * x[n - 1];
    const double vq = q[0] + beta / g * q[n - 1];
    const double den = 1.0 + vq;
    if (den == 0.0) return ORC_E_ZERO_PIVOT;
    const double f = vx / den;
    for (int64_t j = 0; j < n; ++j) x[j] = x[j] - f * q[j];
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The same two exact solves carried out in long double (x87 extended, a    */
/* 64-bit significand): the reference for results that converge to the     */
/* exact A^{-1} d (iterative refinement), whose distance to an FP64 direct  */
/* solve can reach cond(A) * 1e-16.  Inputs and outputs are FP64.           */
/* work: 5n long doubles.                                                    */
/* ------------------------------------------------------------------------ */
static int thomas_ld(int64_t n, const long double *a, const long double *b, const long double *c,
                     const long double *d, long double *x, long double *cp)
{
    long double den = b[0];
    if (den == 0.0L) return ORC_E_ZERO_PIVOT;
    cp[0] = (n > 1 ? c[0] : 0.0L) / den;
    x[0] = d[0] / den;
    for (int64_t j = 1; j < n; ++j) {
        den = b[j] - a[j] * cp[j - 1];
        if (den == 0.0L) return ORC_E_ZERO_PIVOT;
        cp[j] = (j < n - 1 ? c[j] : 0.0L) / den;
        x[j] = (d[j] - a[j] * x[j - 1]) / den;
    }
    for (int64_t j = n - 2; j >= 0; --j) x[j] = x[j] - cp[j] * x[j + 1];
    return ORC_OK;
}

int orc_exact_ld(int64_t n, int periodic, const double *a, const double *b, const double *c,
                 const double *d, double *x)
{
    if (n < 1 || (periodic && n < 3)) return ORC_E_SHAPE;
    long double *w = (long double *)malloc(sizeof(long double) * (size_t)(8 * n));
    if (!w) return ORC_E_NOMEM;
    long double *A = w, *B = w + n, *C = w + 2 * n, *D = w + 3 * n, *X = w + 4 * n;
    long double *cp = w + 5 * n, *U = w + 6 * n, *Q = w + 7 * n;
    for (int64_t j = 0; j < n; ++j) { A[j] = a[j]; B[j] = b[j]; C[j] = c[j]; D[j] = d[j]; }
    int st;
    if (!periodic) {
        st = thomas_ld(n, A, B, C, D, X, cp);
    } else {   /* Sherman-Morrison, as orc_cyclic */
        const long double alpha = C[n - 1], beta = A[0], g = -B[0];
        B[0] -= g;
        B[n - 1] -= alpha * beta / g;
        for (int64_t j = 0; j < n; ++j) U[j] = 0.0L;
        U[0] = g;
        U[n - 1] = alpha;
        st = thomas_ld(n, A, B, C, D, X, cp);
        if (!st) st = thomas_ld(n, A, B, C, U, Q, cp);
        if (!st) {
            const long double vx = X[0] + beta / g * X[n - 1], vq = Q[0] + beta / g * Q[n - 1];
            const long double f = vx / (1.0L + vq);
            for (int64_t j = 0; j < n; ++j) X[j] -= f * Q[j];
        }
    }
    if (!st)
        for (int64_t j = 0; j < n; ++j) x[j] = (double)X[j];
    free(w);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Dense Gaussian elimination with partial pivoting, K x K row-major M       */
/* (destroyed), rhs overwritten by the solution.                             */
/* ------------------------------------------------------------------------ */
static int gepp_solve(int K, double *M, double *rhs)
{
    for (int k = 0; k < K; ++k) {
        int p = k;
        double best = fabs(M[k * K + k]);
        for (int i = k + 1; i < K; ++i)
            if (fabs(M[i * K + k]) > best) { best = fabs(M[i * K + k]); p = i; }
        if (best == 0.0) return ORC_E_ZERO_PIVOT;
        if (p != k) {
            for (int t = 0; t < K; ++t) {
                double s = M[k * K + t]; M[k * K + t] = M[p * K + t]; M[p * K + t] = s;
            }
            double s = rhs[k]; rhs[k] = rhs[p]; rhs[p] = s;
        }
        for (int i = k + 1; i < K; ++i) {
            double l = M[i * K + k] / M[k * K + k];
            if (l == 0.0) continue;
            for (int t = k; t < K; ++t) M[i * K + t] -= l * M[k * K + t];
            rhs[i] -= l * rhs[k];
        }
    }
    for (int k = K - 1; k >= 0; --k) {
        double s = rhs[k];
        for (int t = k + 1; t < K; ++t) s -= M[k * K + t] * rhs[t];
        rhs[k] = s / M[k * K + k];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Local quantities of one line (Sec. 3.2, Eqs. (5) and (6)).                */
/*   xt[r*m + t]  = x~ : the block solve  A~ x~ = d                          */
/*   v [r*m + t]  = A~_r^{-1} (a_{rm} e_0)        (a-corner spike)           */
/*   w [r*m + t]  = A~_r^{-1} (c_{rm+m-1} e_{m-1})  (c-corner spike)         */
/* A~ = A - Delta A: each partition block with the coupling to its           */
/* neighbours removed (its first a and last c set to zero).  A spike that    */
/* has no corner (v of partition 0, w of partition P-1, non-periodic) is 0.  */
/* scratch: 6m doubles.                                                      */
/* ------------------------------------------------------------------------ */
static int local_solves(int64_t n, int P, int periodic, const double *a,
                        const double *b, const double *c, const double *d,
                        double *xt, double *v, double *w, double *scratch)
{
    const int64_t m = n / P;
    double *at = scratch, *bt = scratch + m, *ct = scratch + 2 * m;
    double *e = scratch + 3 * m, *cp = scratch + 4 * m;
    for (int r = 0; r < P; ++r) {
        const int64_t o = (int64_t)r * m;
        for (int64_t t = 0; t < m; ++t) { at[t] = a[o + t]; bt[t] = b[o + t]; ct[t] = c[o + t]; }
        at[0] = 0.0;          /* Delta A: remove the a-corner of the block */
        ct[m - 1] = 0.0;      /* Delta A: remove the c-corner of the block */
        int st = orc_thomas(m, at, bt, ct, d + o, xt + o, cp);            /* Eq. (5) */
        if (st) return st;
        for (int64_t t = 0; t < m; ++t) e[t] = 0.0;
        if (r >= 1 || periodic) e[0] = a[o];                              /* column of V */
        st = orc_thomas(m, at, bt, ct, e, v + o, cp);                     /* Eq. (6) */
        if (st) return st;
        for (int64_t t = 0; t < m; ++t) e[t] = 0.0;
        if (r <= P - 2 || periodic) e[m - 1] = c[o + m - 1];              /* column of V */
        st = orc_thomas(m, at, bt, ct, e, w + o, cp);                     /* Eq. (6) */
        if (st) return st;
    }
    return ORC_OK;
}

/* Number of interfaces and reduced-system size. */
static int n_interfaces(int P, int periodic) { return periodic ? P : P - 1; }

/* ------------------------------------------------------------------------ */
/* Assemble Z = I + E^T A~^{-1} V (Eq. (7)) and E^T x~ for one line.         */
/* Row 2i-1 (1-based) selects x at the last row of L(i); row 2i the first    */
/* row of R(i).  The Y = A~^{-1} V column of unknown 2i-1 is the v spike of  */
/* R(i); the column of unknown 2i is the w spike of L(i).                    */
/* Z is K x K row-major, K = 2 * n_interfaces.                               */
/* ------------------------------------------------------------------------ */
static void assemble_Z(int64_t m, int P, int periodic, const double *xt,
                       const double *v, const double *w, double *Z, double *rhs)
{
    const int NI = n_interfaces(P, periodic), K = 2 * NI;
    for (int t = 0; t < K * K; ++t) Z[t] = 0.0;
    for (int i = 1; i <= NI; ++i) {
        const int L = i - 1, R = i % P;
        const int u1 = 2 * i - 2, u2 = 2 * i - 1;      /* y_{2i-1}, y_{2i} */
        const int64_t lastL = (int64_t)L * m + m - 1, firstR = (int64_t)R * m;
        /* row 2i-1: x at the last row of L */
        Z[u1 * K + u1] += 1.0;
        Z[u1 * K + u2] += w[lastL];                    /* w^(L)_m  */
        if (L >= 1 || periodic) {                      /* v^(L)_m, column of L's left interface */
            const int il = (L >= 1) ? L : P;
            Z[u1 * K + (2 * il - 2)] += v[lastL];
        }
        /* row 2i: x at the first row of R */
        Z[u2 * K + u2] += 1.0;
        Z[u2 * K + u1] += v[firstR];                   /* v^(R)_1  */
        if (R <= P - 2 || periodic) {                  /* w^(R)_1, column of R's right interface */
            const int ir = R + 1;
            Z[u2 * K + (2 * ir - 1)] += w[firstR];
        }
        rhs[u1] = xt[lastL];                           /* E^T x~ */
        rhs[u2] = xt[firstR];
    }
}

/* x = x~ - Y y  (Eq. (8)); partition r uses y_{2r-1} with v^(r) and
 * y_{2r+2} with w^(r) (y_{-1} = y_{2P} = 0 when non-periodic; when periodic
 * partition 0's left interface is the wrap interface P). */
static void correct(int64_t m, int P, int periodic, const double *xt,
                    const double *v, const double *w, const double *y, double *x)
{
    for (int r = 0; r < P; ++r) {
        double yl = 0.0, yr = 0.0;
        if (r >= 1 || periodic) {
            const int il = (r >= 1) ? r : P;
            yl = y[2 * il - 2];
        }
        if (r <= P - 2 || periodic) {
            const int ir = r + 1;
            yr = y[2 * ir - 1];
        }
        const int64_t o = (int64_t)r * m;
        for (int64_t t = 0; t < m; ++t)
            x[o + t] = xt[o + t] - v[o + t] * yl - w[o + t] * yr;
    }
}

static int check_shape(int64_t n, int P, int periodic)
{
    if (n < 1 || P < 1) return ORC_E_SHAPE;
    if (n % P != 0) return ORC_E_SHAPE;
    if (n / P < 2 && !(P == 1 && !periodic)) return ORC_E_SHAPE;
    if (periodic && n < 3) return ORC_E_SHAPE;
    return ORC_OK;
}

/* Work array sizes (doubles) for one line. */
int64_t orc_line_work(int64_t n, int P)
{
    const int K = 2 * P;
    return 6 * n + 6 * (n / (P > 0 ? P : 1)) + 3 * (int64_t)K * K + 4 * K + 16;
}

/* ------------------------------------------------------------------------ */
/* PDD (Sec. 3.2, PDD paragraph; Algorithm 1 steps 3-7): Z keeps only its    */
/* 2x2 diagonal blocks [[1, w^(L)_m], [v^(R)_1, 1]] per interface (the       */
/* entries v^(L)_m and w^(R)_1 are dropped), each solved with the inverse of */
/* a 2x2 matrix; then x = x~ - Y y.                                          */
/* ------------------------------------------------------------------------ */
int orc_pdd(int64_t n, int P, int periodic, const double *a, const double *b,
            const double *c, const double *d, double *x, double *work)
{
    int st = check_shape(n, P, periodic);
    if (st) return st;
    const int64_t m = n / P;
    if (P == 1 && !periodic) return orc_thomas(n, a, b, c, d, x, work);
    double *xt = work, *v = work + n, *w = work + 2 * n, *scratch = work + 3 * n;
    double *y = scratch + 6 * m;
    st = local_solves(n, P, periodic, a, b, c, d, xt, v, w, scratch);
    if (st) return st;
    const int NI = n_interfaces(P, periodic);
    for (int i = 1; i <= NI; ++i) {
        const int L = i - 1, R = i % P;
        const int64_t lastL = (int64_t)L * m + m - 1, firstR = (int64_t)R * m;
        const double z12 = w[lastL], z21 = v[firstR];
        const double r1 = xt[lastL], r2 = xt[firstR];
        const double det = 1.0 - z12 * z21;
        if (det == 0.0) return ORC_E_ZERO_PIVOT;
        y[2 * i - 2] = (r1 - z12 * r2) / det;
        y[2 * i - 1] = (r2 - z21 * r1) / det;
    }
    correct(m, P, periodic, xt, v, w, y, x);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* PPT (Sec. 3.2, Eqs. (9)-(11)): with the pair-swapping permutation P,      */
/* Zbar = P + E^T A~^{-1} V P = Z P is tridiagonal (cyclic when periodic);   */
/* solve Zbar ybar = E^T x~ by Gaussian elimination with partial pivoting,   */
/* then x = x~ - Ybar ybar with Ybar = Y P, i.e. y = P ybar.                 */
/* ------------------------------------------------------------------------ */
static void permute_pairs(int K, const double *in, double *out)
{
    for (int k = 0; k < K; k += 2) { out[k] = in[k + 1]; out[k + 1] = in[k]; }
}

int orc_ppt(int64_t n, int P, int periodic, const double *a, const double *b,
            const double *c, const double *d, double *x, double *work)
{
    int st = check_shape(n, P, periodic);
    if (st) return st;
    const int64_t m = n / P;
    if (P == 1 && !periodic) return orc_thomas(n, a, b, c, d, x, work);
    const int NI = n_interfaces(P, periodic), K = 2 * NI;
    double *xt = work, *v = work + n, *w = work + 2 * n, *scratch = work + 3 * n;
    double *Z = scratch + 6 * m, *Zbar = Z + K * K, *rhs = Zbar + K * K, *ybar = rhs + K;
    double *y = ybar + K;
    st = local_solves(n, P, periodic, a, b, c, d, xt, v, w, scratch);
    if (st) return st;
    assemble_Z(m, P, periodic, xt, v, w, Z, rhs);
    /* Zbar = Z P : swap columns 2i-1 <-> 2i of Z */
    for (int row = 0; row < K; ++row)
        for (int col = 0; col < K; col += 2) {
            Zbar[row * K + col] = Z[row * K + col + 1];
            Zbar[row * K + col + 1] = Z[row * K + col];
        }
    for (int k = 0; k < K; ++k) ybar[k] = rhs[k];
    st = gepp_solve(K, Zbar, ybar);                                    /* Eq. (10) */
    if (st) return st;
    permute_pairs(K, ybar, y);                                         /* Ybar ybar = Y (P ybar) */
    correct(m, P, periodic, xt, v, w, y, x);                           /* Eq. (11) */
    return ORC_OK;
}

/* Exact solution: Thomas (non-periodic) or the Sherman-Morrison cyclic solve. */
int orc_exact(int64_t n, int periodic, const double *a, const double *b,
              const double *c, const double *d, double *x, double *work)
{
    return periodic ? orc_cyclic(n, a, b, c, d, x, work) : orc_thomas(n, a, b, c, d, x, work);
}

/* ------------------------------------------------------------------------ */
/* Diagnostics for the pattern pins: Z, Zbar (K x K each), E^T x~ and the    */
/* spikes of one line.  out_Z, out_Zbar: K*K; out_rhs: K; v_out, w_out: n.   */
/* ------------------------------------------------------------------------ */
int orc_reduced_system(int64_t n, int P, int periodic, const double *a,
                       const double *b, const double *c, const double *d,
                       double *out_Z, double *out_Zbar, double *out_rhs,
                       double *xt_out, double *v_out, double *w_out)
{
    int st = check_shape(n, P, periodic);
    if (st) return st;
    if (P == 1 && !periodic) return ORC_E_SHAPE;
    const int64_t m = n / P;
    const int K = 2 * n_interfaces(P, periodic);
    double *scratch = (double *)malloc(sizeof(double) * (size_t)(6 * m + 8));
    if (!scratch) return ORC_E_NOMEM;
    st = local_solves(n, P, periodic, a, b, c, d, xt_out, v_out, w_out, scratch);
    free(scratch);
    if (st) return st;
    assemble_Z(m, P, periodic, xt_out, v_out, w_out, out_Z, out_rhs);
    for (int row = 0; row < K; ++row)
        for (int col = 0; col < K; col += 2) {
            out_Zbar[row * K + col] = out_Z[row * K + col + 1];
            out_Zbar[row * K + col + 1] = out_Z[row * K + col];
        }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Batched driver.  Line (b0, b1), b0 < nb0, b1 < nb1, has its row j at      */
/*   d[j*s_j + b0*s_b0 + b1*s_b1]                                            */
/* and coefficients at a[j*cs_j + b0*cs_b0 + b1*cs_b1] (stride 0 = shared).  */
/* method: ORC_EXACT, ORC_PDD or ORC_PPT.  d is overwritten by x.            */
/* Returns the first error met (lines after it may be left unsolved).        */
/* ------------------------------------------------------------------------ */
int orc_solve_batch(int method, int64_t n, int P, int periodic,
                    const double *a, const double *b, const double *c,
                    int64_t cs_j, int64_t cs_b0, int64_t cs_b1,
                    double *d, int64_t nb0, int64_t nb1,
                    int64_t s_j, int64_t s_b0, int64_t s_b1, int nthreads)
{
    if (!a || !b || !c || !d) return ORC_E_ARG;
    if (method != ORC_EXACT && method != ORC_EXACT_LD) {
        int st = check_shape(n, P, periodic);
        if (st) return st;
    } else if (n < 1 || (periodic && n < 3)) {
        return ORC_E_SHAPE;
    }
    const int64_t nlines = nb0 * nb1;
    const int64_t lw = orc_line_work(n, P);
    int status = ORC_OK;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * (size_t)(5 * n + lw));
        if (!buf) {
#pragma omp critical
            status = ORC_E_NOMEM;
        } else {
            double *la = buf, *lb = buf + n, *lc = buf + 2 * n, *ld = buf + 3 * n;
            double *lx = buf + 4 * n, *work = buf + 5 * n;
#pragma omp for schedule(static)
            for (int64_t L = 0; L < nlines; ++L) {
                const int64_t b0 = L % nb0, b1 = L / nb0;
                const int64_t o = b0 * s_b0 + b1 * s_b1, co = b0 * cs_b0 + b1 * cs_b1;
                for (int64_t j = 0; j < n; ++j) {
                    la[j] = a[co + j * cs_j];
                    lb[j] = b[co + j * cs_j];
                    lc[j] = c[co + j * cs_j];
                    ld[j] = d[o + j * s_j];
                }
                int st;
                if (method == ORC_PDD) st = orc_pdd(n, P, periodic, la, lb, lc, ld, lx, work);
                else if (method == ORC_PPT) st = orc_ppt(n, P, periodic, la, lb, lc, ld, lx, work);
                else if (method == ORC_EXACT_LD) st = orc_exact_ld(n, periodic, la, lb, lc, ld, lx);
                else st = orc_exact(n, periodic, la, lb, lc, ld, lx, work);
                if (st) {
#pragma omp critical
                    if (status == ORC_OK) status = st;
                    continue;
                }
                for (int64_t j = 0; j < n; ++j) d[o + j * s_j] = lx[j];
            }
            free(buf);
        }
    }
    return status;
}

/* ------------------------------------------------------------------------ */
/* One ADI sweep over u[Nz][Ny][Nx] (x fastest) along direction dir          */
/* (0 = x, 1 = y, 2 = z); a, b, c have the length of that direction and are  */
/* shared by every line (Sec. 2.2: one tridiagonal system per direction).    */
/* ------------------------------------------------------------------------ */
int orc_adi_sweep(int method, int dir, double *u, int64_t Nx, int64_t Ny, int64_t Nz,
                  const double *a, const double *b, const double *c,
                  int P, int periodic, int nthreads)
{
    if (dir == 0)
        return orc_solve_batch(method, Nx, P, periodic, a, b, c, 1, 0, 0,
                               u, Ny, Nz, 1, Nx, Nx * Ny, nthreads);
    if (dir == 1)
        return orc_solve_batch(method, Ny, P, periodic, a, b, c, 1, 0, 0,
                               u, Nx, Nz, Nx, 1, Nx * Ny, nthreads);
    if (dir == 2)
        return orc_solve_batch(method, Nz, P, periodic, a, b, c, 1, 0, 0,
                               u, Nx, Ny, Nx * Ny, 1, Nx, nthreads);
    return ORC_E_ARG;
}

/* ------------------------------------------------------------------------ */
/* Wall-normal Poisson solves per spanwise wavenumber (Sec. 2.2; PPT        */
/* paragraph of Sec. 3.2).  phihat[Nk][Ny][Nx] complex128 interleaved (re,  */
/* im); for wavenumber k the real matrix is a_j = ay_j, c_j = cy_j,          */
/* b_j = -(ay_j + cy_j) - lam_k; real and imaginary parts are independent    */
/* real right-hand sides of the same real matrix.  A mode with lam_k == 0 is */
/* the singular Neumann operator: row 0 is replaced by x_0 = 0.              */
/* ------------------------------------------------------------------------ */
int orc_poisson(int method, double *phihat, int64_t Nx, int64_t Ny, int64_t Nk,
                const double *ay, const double *cy, const double *lam, int P, int nthreads)
{
    if (!phihat || !ay || !cy || !lam) return ORC_E_ARG;
    double *bk = (double *)malloc(sizeof(double) * (size_t)(3 * Ny));
    if (!bk) return ORC_E_NOMEM;
    double *ak = bk + Ny, *ck = bk + 2 * Ny;
    int status = ORC_OK;
    for (int64_t k = 0; k < Nk && status == ORC_OK; ++k) {
        for (int64_t j = 0; j < Ny; ++j) {
            ak[j] = ay[j];
            ck[j] = cy[j];
            bk[j] = -(ay[j] + cy[j]) - lam[k];
        }
        double *plane = phihat + 2 * k * Ny * Nx;
        if (lam[k] == 0.0) {          /* gauge: x_0 = 0 */
            bk[0] = 1.0;
            ck[0] = 0.0;
            for (int64_t i = 0; i < 2 * Nx; ++i) plane[i] = 0.0;
        }
        /* real view: 2*Nx independent real lines, row stride 2*Nx */
        status = orc_solve_batch(method, Ny, P, 0, ak, bk, ck, 1, 0, 0,
                                 plane, 2 * Nx, 1, 2 * Nx, 1, 0, nthreads);
    }
    free(bk);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Wall-normal Poisson solves once both homogeneous directions are          */
/* transformed (Sec. 2.2; PPT paragraph of Sec. 3.2): one real matrix per    */
/* line (k, i) of phihat[Nk][Ny][Nx] complex128, a_j = ay_j, c_j = cy_j,      */
/* b_j = -(ay_j + cy_j) - (lamz_k + lamx_i).  A line whose shift is 0 is the */
/* singular Neumann operator: row 0 is replaced by x_0 = 0.  Real and        */
/* imaginary parts are two right-hand sides of the same matrix, each solved  */
/* by the method given (ORC_PPT, ORC_PDD, ORC_EXACT or ORC_EXACT_LD).        */
/* ------------------------------------------------------------------------ */
int orc_poisson_shifted(int method, double *phihat, int64_t Nx, int64_t Ny, int64_t Nk,
                        const double *ay, const double *cy, const double *lamz,
                        const double *lamx, int P, int nthreads)
{
    if (!phihat || !ay || !cy || !lamz || !lamx) return ORC_E_ARG;
    if (method == ORC_PDD || method == ORC_PPT) {
        int st = check_shape(Ny, P, 0);
        if (st) return st;
    }
    const int64_t n = Ny, lw = orc_line_work(n, P);
    int status = ORC_OK;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * (size_t)(6 * n + lw));
        if (!buf) {
#pragma omp critical
            status = ORC_E_NOMEM;
        } else {
            double *la = buf, *lb = buf + n, *lc = buf + 2 * n, *ld = buf + 3 * n;
            double *lx = buf + 4 * n, *work = buf + 6 * n;
#pragma omp for schedule(static)
            for (int64_t L = 0; L < Nk * Nx; ++L) {
                const int64_t k = L / Nx, i = L % Nx;
                const double sigma = lamz[k] + lamx[i];
                for (int64_t j = 0; j < n; ++j) {
                    la[j] = ay[j];
                    lc[j] = cy[j];
                    lb[j] = -(ay[j] + cy[j]) - sigma;
                }
                if (sigma == 0.0) {           /* gauge: x_0 = 0 */
                    lb[0] = 1.0;
                    lc[0] = 0.0;
                }
                for (int part = 0; part < 2; ++part) {
                    double *base = phihat + 2 * (k * Ny * Nx + i) + part;
                    for (int64_t j = 0; j < n; ++j) ld[j] = base[2 * j * Nx];
                    if (sigma == 0.0) ld[0] = 0.0;
                    int st;
                    if (method == ORC_PDD) st = orc_pdd(n, P, 0, la, lb, lc, ld, lx, work);
                    else if (method == ORC_PPT) st = orc_ppt(n, P, 0, la, lb, lc, ld, lx, work);
                    else if (method == ORC_EXACT_LD) st = orc_exact_ld(n, 0, la, lb, lc, ld, lx);
                    else st = orc_exact(n, 0, la, lb, lc, ld, lx, work);
                    if (st) {
#pragma omp critical
                        if (status == ORC_OK) status = st;
                        break;
                    }
                    for (int64_t j = 0; j < n; ++j) base[2 * j * Nx] = lx[j];
                }
            }
            free(buf);
        }
    }
    return status;
}

/* ------------------------------------------------------------------------ */
/* Diagonal pivoting for one tridiagonal block: the local solver the PPT    */
/* paragraph of Sec. 3.2 names (the parallel solver of Chang et al. that it  */
/* cites), i.e. Gaussian elimination without row interchanges whose pivots  */
/* are 1x1 diagonal entries or 2x2 diagonal blocks.  The paper prints no    */
/* pivot criterion; the one used here is the Bunch-Kaufman test in the      */
/* form given for tridiagonal matrices: with delta the current (eliminated) */
/* diagonal entry of row k and                                               */
/*   sigma = max(|c_k|, |a_{k+1}|, |b_{k+1}|, |c_{k+1}|, |a_{k+2}|)          */
/* (entries outside the block count as 0), row k is a 1x1 pivot when        */
/*   |delta| sigma >= kappa |a_{k+1} c_k|,   kappa = (sqrt(5) - 1)/2,        */
/* else rows k, k+1 form a 2x2 pivot.  The last row is always 1x1.          */
/*                                                                            */
/* After elimination every row reads x_k = p_k - q_k x_{k+s}: s = 1, or     */
/* s = 2 for the first row of a 2x2 pivot (its partner row links to k+2 as  */
/* well).  A 1x1 pivot takes exactly the steps of orc_thomas:               */
/*   delta = b_k - a_k q_{k-1},  q_k = c_k/delta,  p_k = (d_k - a_k p_{k-1})/delta. */
/* A 2x2 pivot with block [[delta, c_k], [a_{k+1}, b_{k+1}]], determinant   */
/* D = delta b_{k+1} - c_k a_{k+1} and r = d_k - a_k p_{k-1}:               */
/*   p_k = (b_{k+1} r - c_k d_{k+1})/D,      q_k = -c_k c_{k+1}/D,           */
/*   p_{k+1} = (delta d_{k+1} - a_{k+1} r)/D, q_{k+1} = delta c_{k+1}/D.      */
/* m rows: a[0] and c[m-1] are not read.  rhs holds nrhs right-hand sides   */
/* of length m one after the other and is overwritten by the solutions      */
/* (all share the pivots).  piv[k] (nullable): 1 for a 1x1 pivot, 2 for the */
/* first row of a 2x2 pivot, 0 for its second row.  work: 2m doubles.       */
/* ------------------------------------------------------------------------ */
static const double kDpKappa = 0.6180339887498948482;   /* (sqrt(5) - 1)/2 */

int orc_dpivot(int64_t m, const double *a, const double *b, const double *c, int nrhs,
               double *rhs, unsigned char *piv, double *work)
{
    if (m < 1 || nrhs < 0) return ORC_E_SHAPE;
    double *q = work;                    /* q_k */
    unsigned char *kind = (unsigned char *)(work + m);   /* pivot kinds (m bytes) */
#define AA(k) ((k) >= 1 && (k) < m ? a[k] : 0.0)
#define CC(k) ((k) >= 0 && (k) < m - 1 ? c[k] : 0.0)
    /* factorisation: pivot kinds and q (shared by every right-hand side) */
    double qprev = 0.0;                  /* q of the row linked (s = 1) to row k */
    int64_t k = 0;
    while (k < m) {
        const double delta = b[k] - AA(k) * qprev;
        int two = 0;
        if (k + 1 < m) {
            double sigma = fabs(CC(k));
            sigma = fmax(sigma, fabs(AA(k + 1)));
            sigma = fmax(sigma, fabs(b[k + 1]));
            sigma = fmax(sigma, fabs(CC(k + 1)));
            sigma = fmax(sigma, fabs(AA(k + 2)));
            two = fabs(delta) * sigma < kDpKappa * fabs(AA(k + 1) * CC(k));
        }
        if (!two) {
            if (delta == 0.0) return ORC_E_ZERO_PIVOT;
            q[k] = CC(k) / delta;
            kind[k] = 1;
            qprev = q[k];
            k += 1;
        } else {
            const double D = delta * b[k + 1] - CC(k) * AA(k + 1);
            if (D == 0.0) return ORC_E_ZERO_PIVOT;
            q[k] = -CC(k) * CC(k + 1) / D;
            q[k + 1] = delta * CC(k + 1) / D;
            kind[k] = 2;
            kind[k + 1] = 0;
            qprev = q[k + 1];
            k += 2;
        }
    }
    /* each right-hand side: forward p, then back substitution */
    for (int s = 0; s < nrhs; ++s) {
        double *x = rhs + (int64_t)s * m;
        double pprev = 0.0, qp = 0.0;
        k = 0;
        while (k < m) {
            if (kind[k] == 1) {
                const double delta = b[k] - AA(k) * qp;
                x[k] = (x[k] - AA(k) * pprev) / delta;
                qp = q[k];
                pprev = x[k];
                k += 1;
            } else {
                const double delta = b[k] - AA(k) * qp;
                const double D = delta * b[k + 1] - CC(k) * AA(k + 1);
                const double r = x[k] - AA(k) * pprev;
                const double dn = x[k + 1];
                x[k] = (b[k + 1] * r - CC(k) * dn) / D;
                x[k + 1] = (delta * dn - AA(k + 1) * r) / D;
                qp = q[k + 1];
                pprev = x[k + 1];
                k += 2;
            }
        }
        for (int64_t t = m - 2; t >= 0; --t) {
            const int64_t link = kind[t] == 2 ? t + 2 : t + 1;
            x[t] = x[t] - q[t] * (link < m ? x[link] : 0.0);
        }
    }
    if (piv)
        for (int64_t t = 0; t < m; ++t) piv[t] = kind[t];
#undef AA
#undef CC
    return ORC_OK;
}

/* Local solves of Eqs. (5), (6) with the diagonal-pivoting block solver:   */
/* the three right-hand sides of partition r (its part of d, the a-corner   */
/* column a_{rm} e_0, the c-corner column c_{rm+m-1} e_{m-1}) go through    */
/* one factorisation of A~_r.  piv: n bytes (nullable).  scratch: 8m.       */
static int local_solves_dp(int64_t n, int P, int periodic, const double *a, const double *b,
                           const double *c, const double *d, double *xt, double *v, double *w,
                           unsigned char *piv, double *scratch)
{
    const int64_t m = n / P;
    double *at = scratch, *ct = scratch + m, *R = scratch + 2 * m, *fw = scratch + 5 * m;
    for (int r = 0; r < P; ++r) {
        const int64_t o = (int64_t)r * m;
        for (int64_t t = 0; t < m; ++t) { at[t] = a[o + t]; ct[t] = c[o + t]; }
        at[0] = 0.0;          /* Delta A: remove the a-corner of the block */
        ct[m - 1] = 0.0;      /* Delta A: remove the c-corner of the block */
        for (int64_t t = 0; t < 3 * m; ++t) R[t] = 0.0;
        for (int64_t t = 0; t < m; ++t) R[t] = d[o + t];
        if (r >= 1 || periodic) R[m] = a[o];
        if (r <= P - 2 || periodic) R[2 * m + m - 1] = c[o + m - 1];
        int st = orc_dpivot(m, at, b + o, ct, 3, R, piv ? piv + o : NULL, fw);
        if (st) return st;
        for (int64_t t = 0; t < m; ++t) {
            xt[o + t] = R[t];
            v[o + t] = R[m + t];
            w[o + t] = R[2 * m + t];
        }
    }
    return ORC_OK;
}

/* PPT (Eqs. (9)-(11)) with diagonal pivoting in the partition blocks: the  */
/* local solves above, then the same Zbar assembly, GEPP and correction as  */
/* orc_ppt.  piv (nullable): the pivot kind of every row of the line.       */
/* work: orc_line_work(n, P) + 2n doubles.                                   */
int orc_ppt_dp(int64_t n, int P, int periodic, const double *a, const double *b,
               const double *c, const double *d, double *x, double *work, unsigned char *piv)
{
    int st = check_shape(n, P, periodic);
    if (st) return st;
    const int64_t m = n / P;
    const int NI = n_interfaces(P, periodic), K = 2 * NI;
    double *xt = work, *v = work + n, *w = work + 2 * n, *scratch = work + 3 * n;
    double *Z = scratch + 8 * m, *Zbar = Z + K * K, *rhs = Zbar + K * K, *ybar = rhs + K;
    double *y = ybar + K;
    st = local_solves_dp(n, P, periodic, a, b, c, d, xt, v, w, piv, scratch);
    if (st) return st;
    if (P == 1 && !periodic) {
        for (int64_t t = 0; t < n; ++t) x[t] = xt[t];
        return ORC_OK;
    }
    assemble_Z(m, P, periodic, xt, v, w, Z, rhs);
    for (int row = 0; row < K; ++row)
        for (int col = 0; col < K; col += 2) {
            Zbar[row * K + col] = Z[row * K + col + 1];
            Zbar[row * K + col + 1] = Z[row * K + col];
        }
    for (int k = 0; k < K; ++k) ybar[k] = rhs[k];
    st = gepp_solve(K, Zbar, ybar);                                    /* Eq. (10) */
    if (st) return st;
    permute_pairs(K, ybar, y);
    correct(m, P, periodic, xt, v, w, y, x);                           /* Eq. (11) */
    return ORC_OK;
}

/* Batched strided driver of orc_ppt_dp (layout as orc_solve_batch, with   */
/* per-line coefficients allowed).  piv (nullable): nb0*nb1*n bytes, line  */
/* (b0, b1) at (b1*nb0 + b0)*n.                                              */
int orc_ppt_dp_batch(int64_t n, int P, int periodic, const double *a, const double *b,
                     const double *c, int64_t cs_j, int64_t cs_b0, int64_t cs_b1, double *d,
                     int64_t nb0, int64_t nb1, int64_t s_j, int64_t s_b0, int64_t s_b1,
                     unsigned char *piv, int nthreads)
{
    if (!a || !b || !c || !d) return ORC_E_ARG;
    int status = check_shape(n, P, periodic);
    if (status) return status;
    const int64_t nlines = nb0 * nb1;
    const int64_t lw = orc_line_work(n, P) + 2 * n + 2 * (n / P);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        double *buf = (double *)malloc(sizeof(double) * (size_t)(5 * n + lw));
        if (!buf) {
#pragma omp critical
            status = ORC_E_NOMEM;
        } else {
            double *la = buf, *lb = buf + n, *lc = buf + 2 * n, *ld = buf + 3 * n;
            double *lx = buf + 4 * n, *work = buf + 5 * n;
#pragma omp for schedule(static)
            for (int64_t L = 0; L < nlines; ++L) {
                const int64_t b0 = L % nb0, b1 = L / nb0;
                const int64_t o = b0 * s_b0 + b1 * s_b1, co = b0 * cs_b0 + b1 * cs_b1;
                for (int64_t j = 0; j < n; ++j) {
                    la[j] = a[co + j * cs_j];
                    lb[j] = b[co + j * cs_j];
                    lc[j] = c[co + j * cs_j];
                    ld[j] = d[o + j * s_j];
                }
                const int st = orc_ppt_dp(n, P, periodic, la, lb, lc, ld, lx, work,
                                          piv ? piv + L * n : NULL);
                if (st) {
#pragma omp critical
                    if (status == ORC_OK) status = st;
                    continue;
                }
                for (int64_t j = 0; j < n; ++j) d[o + j * s_j] = lx[j];
            }
            free(buf);
        }
    }
    return status;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
