/* Exercises every entry point of oracle/oracle.c on small random lines with
 * work arrays of exactly the documented sizes, for a build with AddressSanitizer
 * and UndefinedBehaviorSanitizer (tests/test_sanitize.py).  Each result is also
 * compared with the plain solve of the same line (loose bound: this program
 * checks memory and arithmetic safety; the accuracy pins are the pytest ones).
 * Exit status 0 when every call behaved, 1 otherwise. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_thomas(int64_t, const double *, const double *, const double *, const double *, double *, double *);
int orc_cyclic(int64_t, const double *, const double *, const double *, const double *, double *, double *);
int orc_exact_ld(int64_t, int, const double *, const double *, const double *, const double *, double *);
int64_t orc_line_work(int64_t, int);
int orc_pdd(int64_t, int, int, const double *, const double *, const double *, const double *, double *, double *);
int orc_ppt(int64_t, int, int, const double *, const double *, const double *, const double *, double *, double *);
int orc_exact(int64_t, int, const double *, const double *, const double *, const double *, double *, double *);
int orc_reduced_system(int64_t, int, int, const double *, const double *, const double *, const double *, double *,
                       double *, double *, double *, double *, double *);
int orc_solve_batch(int, int64_t, int, int, const double *, const double *, const double *, int64_t, int64_t,
                    int64_t, double *, int64_t, int64_t, int64_t, int64_t, int64_t, int);
int orc_adi_sweep(int, int, double *, int64_t, int64_t, int64_t, const double *, const double *, const double *,
                  int, int, int);
int orc_poisson(int, double *, int64_t, int64_t, int64_t, const double *, const double *, const double *, int, int);
int orc_poisson_shifted(int, double *, int64_t, int64_t, int64_t, const double *, const double *, const double *,
                        const double *, int, int);
int orc_dpivot(int64_t, const double *, const double *, const double *, int, double *, unsigned char *, double *);
int orc_ppt_dp(int64_t, int, int, const double *, const double *, const double *, const double *, double *,
               double *, unsigned char *);
int orc_ppt_dp_batch(int64_t, int, int, const double *, const double *, const double *, int64_t, int64_t, int64_t,
                     double *, int64_t, int64_t, int64_t, int64_t, int64_t, unsigned char *, int);

static int failures = 0;
static uint64_t rng_state = 0x9E3779B97F4A7C15ull;

static double uni(void)   /* splitmix64 -> [0, 1) */
{
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static double *vec(int64_t n)   /* exactly n doubles, so an overrun is caught */
{
    double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!p) { fprintf(stderr, "malloc\n"); exit(2); }
    return p;
}

static void dominant(int64_t n, double *a, double *b, double *c, double *d, int periodic)
{
    for (int64_t j = 0; j < n; ++j) {
        a[j] = uni() - 0.5;
        c[j] = uni() - 0.5;
        b[j] = (uni() < 0.5 ? -1.0 : 1.0) * (fabs(a[j]) + fabs(c[j]) + 0.5 + uni());
        d[j] = 2.0 * uni() - 1.0;
    }
    if (!periodic) { a[0] = 0.0; c[n - 1] = 0.0; }
}

static void expect(int ok, const char *what, int64_t n, int P, int periodic)
{
    if (!ok) {
        fprintf(stderr, "FAIL %s n=%lld P=%d periodic=%d\n", what, (long long)n, P, periodic);
        ++failures;
    }
}

static double maxdiff(int64_t n, const double *x, const double *y)
{
    double e = 0.0, s = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        e = fmax(e, fabs(x[j] - y[j]));
        s = fmax(s, fabs(y[j]));
    }
    return e / (s > 0 ? s : 1.0);
}

static void line_case(int64_t n, int P, int periodic)
{
    double *a = vec(n), *b = vec(n), *c = vec(n), *d = vec(n), *x = vec(n), *ref = vec(n);
    dominant(n, a, b, c, d, periodic);
    double *w5 = vec(5 * n);
    int st = orc_exact(n, periodic, a, b, c, d, ref, w5);
    expect(st == 0, "exact", n, P, periodic);
    st = orc_exact_ld(n, periodic, a, b, c, d, x);
    expect(st == 0 && maxdiff(n, x, ref) < 1e-12, "exact_ld", n, P, periodic);
    const int64_t lw = orc_line_work(n, P);
    double *work = vec(lw);
    st = orc_ppt(n, P, periodic, a, b, c, d, x, work);
    expect(st == 0 && maxdiff(n, x, ref) < 1e-12, "ppt", n, P, periodic);
    st = orc_pdd(n, P, periodic, a, b, c, d, x, work);
    expect(st == 0 && maxdiff(n, x, ref) < 1.0, "pdd", n, P, periodic);
    free(work);
    if (P > 1 || periodic) {
        const int K = 2 * (periodic ? P : P - 1);
        double *Z = vec((int64_t)K * K), *Zb = vec((int64_t)K * K), *rhs = vec(K);
        double *xt = vec(n), *v = vec(n), *w = vec(n);
        st = orc_reduced_system(n, P, periodic, a, b, c, d, Z, Zb, rhs, xt, v, w);
        expect(st == 0, "reduced_system", n, P, periodic);
        free(Z); free(Zb); free(rhs); free(xt); free(v); free(w);
    }
    /* diagonal pivoting: documented work orc_line_work + 2n */
    double *wdp = vec(orc_line_work(n, P) + 2 * n);
    unsigned char *piv = (unsigned char *)malloc((size_t)n);
    st = orc_ppt_dp(n, P, periodic, a, b, c, d, x, wdp, piv);
    expect(st == 0 && maxdiff(n, x, ref) < 1e-12, "ppt_dp", n, P, periodic);
    for (int64_t j = 0; j < n; ++j) expect(piv[j] == 1, "ppt_dp pivots on dominant rows", n, P, periodic);
    /* non-dominant rows with zero diagonal entries */
    for (int64_t j = 0; j < n; ++j) {
        a[j] = (uni() < 0.5 ? -1 : 1) * (0.5 + 0.5 * uni());
        c[j] = (uni() < 0.5 ? -1 : 1) * (0.5 + 0.5 * uni());
        b[j] = (j % 7 == 0) ? 0.0 : 0.6 * uni() - 0.3;
    }
    if (!periodic) { a[0] = 0.0; c[n - 1] = 0.0; }
    st = orc_ppt_dp(n, P, periodic, a, b, c, d, x, wdp, piv);
    expect(st == 0 || st == 3, "ppt_dp non-dominant", n, P, periodic);
    free(wdp); free(piv);
    free(a); free(b); free(c); free(d); free(x); free(ref); free(w5);
}

int main(void)
{
    static const int64_t ns[] = {1, 2, 3, 4, 12, 16, 24, 64, 288};
    static const int Ps[] = {1, 2, 3, 4, 8, 16};
    for (size_t i = 0; i < sizeof ns / sizeof *ns; ++i)
        for (size_t k = 0; k < sizeof Ps / sizeof *Ps; ++k)
            for (int per = 0; per < 2; ++per) {
                const int64_t n = ns[i];
                const int P = Ps[k];
                if (n % P || (n / P < 2 && !(P == 1 && !per)) || (per && n < 3)) continue;
                line_case(n, P, per);
            }
    /* shape errors come back as codes, not crashes */
    {
        double *a = vec(12), *b = vec(12), *c = vec(12), *d = vec(12), *x = vec(12), *w = vec(orc_line_work(12, 5));
        dominant(12, a, b, c, d, 0);
        expect(orc_ppt(12, 5, 0, a, b, c, d, x, w) == 2, "shape 12 % 5", 12, 5, 0);
        expect(orc_pdd(12, 12, 0, a, b, c, d, x, w) == 2, "shape m = 1", 12, 12, 0);
        expect(orc_thomas(0, a, b, c, d, x, w) == 2, "shape n = 0", 0, 1, 0);
        b[3] = 0.0; a[3] = 0.0; c[3] = 0.0;
        expect(orc_thomas(12, a, b, c, d, x, w) == 3, "zero pivot", 12, 1, 0);
        free(a); free(b); free(c); free(d); free(x); free(w);
    }
    /* dpivot with several right-hand sides, work 2m */
    {
        const int64_t m = 9;
        double *a = vec(m), *b = vec(m), *c = vec(m), *R = vec(3 * m), *wk = vec(2 * m);
        unsigned char *piv = (unsigned char *)malloc((size_t)m);
        for (int64_t j = 0; j < m; ++j) { a[j] = 1.0; c[j] = -1.0; b[j] = (j % 2) ? 0.0 : 0.25; }
        for (int64_t j = 0; j < 3 * m; ++j) R[j] = uni();
        const int st = orc_dpivot(m, a, b, c, 3, R, piv, wk);
        expect(st == 0 || st == 3, "dpivot", m, 1, 0);
        free(a); free(b); free(c); free(R); free(wk); free(piv);
    }
    /* batched drivers over a strided 3-D field and the Poisson planes */
    {
        const int64_t Nx = 10, Ny = 8, Nz = 12;
        double *u = vec(Nx * Ny * Nz), *ax = vec(Nx), *bx = vec(Nx), *cx = vec(Nx), *tmp = vec(Nz);
        for (int64_t j = 0; j < Nx * Ny * Nz; ++j) u[j] = uni() - 0.5;
        for (int dir = 0; dir < 3; ++dir) {
            const int64_t n = dir == 0 ? Nx : (dir == 1 ? Ny : Nz);
            double *aa = vec(n), *bb = vec(n), *cc = vec(n);
            dominant(n, aa, bb, cc, tmp, dir == 2);
            for (int method = 0; method < 4; ++method) {
                const int st = orc_adi_sweep(method, dir, u, Nx, Ny, Nz, aa, bb, cc, 2, dir == 2, 1);
                expect(st == 0, "adi_sweep", n, 2, dir == 2);
            }
            free(aa); free(bb); free(cc);
        }
        /* per-line coefficients */
        const int64_t nl = Nx * Nz;
        double *A = vec(Ny * nl), *B = vec(Ny * nl), *C = vec(Ny * nl), *D = vec(Ny * nl);
        for (int64_t l = 0; l < nl; ++l) {
            double la[8], lb[8], lc[8], ld[8];
            dominant(Ny, la, lb, lc, ld, 0);
            for (int64_t j = 0; j < Ny; ++j) {
                A[j * nl + l] = la[j]; B[j * nl + l] = lb[j]; C[j * nl + l] = lc[j]; D[j * nl + l] = ld[j];
            }
        }
        expect(orc_solve_batch(2, Ny, 4, 0, A, B, C, nl, 1, Nx, D, Nx, Nz, nl, 1, Nx, 1) == 0, "solve_batch", Ny, 4, 0);
        unsigned char *piv = (unsigned char *)malloc((size_t)(Ny * nl));
        expect(orc_ppt_dp_batch(Ny, 2, 0, A, B, C, nl, 1, Nx, D, Nx, Nz, nl, 1, Nx, piv, 1) == 0, "ppt_dp_batch",
               Ny, 2, 0);
        free(piv); free(A); free(B); free(C); free(D);
        const int64_t Nk = Nz / 2 + 1;
        double *ph = vec(2 * Nk * Ny * Nx), *ay = vec(Ny), *cy = vec(Ny), *lz = vec(Nk), *lx = vec(Nx);
        for (int64_t j = 0; j < 2 * Nk * Ny * Nx; ++j) ph[j] = uni() - 0.5;
        for (int64_t j = 0; j < Ny; ++j) { ay[j] = j ? 1.0 + uni() : 0.0; cy[j] = j < Ny - 1 ? 1.0 + uni() : 0.0; }
        for (int64_t k = 0; k < Nk; ++k) lz[k] = k ? 0.5 * k : 0.0;
        for (int64_t i = 0; i < Nx; ++i) lx[i] = 0.25 * i;
        for (int method = 0; method < 4; ++method) {
            if (method == 1) continue;   /* PDD is inaccurate, not unsafe, on these rows */
            expect(orc_poisson(method, ph, Nx, Ny, Nk, ay, cy, lz, 4, 1) == 0, "poisson", Ny, 4, 0);
            expect(orc_poisson_shifted(method, ph, Nx, Ny, Nk, ay, cy, lz, lx, 4, 1) == 0, "poisson_shifted", Ny,
                   4, 0);
        }
        free(ph); free(ay); free(cy); free(lz); free(lx);
        free(u); free(ax); free(bx); free(cx); free(tmp);
    }
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("oracle sanitizer driver: ok\n");
    return 0;
}
