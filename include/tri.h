/*
 * tri.h -- C ABI of libtri: batched partitioned tridiagonal solves with the
 * Parallel Diagonal Dominant (PDD) and Parallel Partition (PPT) methods on
 * AMD Instinct MI355X (gfx950).
 *
 * Method: Ha, Park & You, "A scalable multi-GPU method for semi-implicit
 * fractional-step integration of incompressible Navier-Stokes equations",
 * arXiv:1812.01178, Sec. 3.2 (Eqs. (3)-(11), Algorithm 1).  The paper's
 * domain decomposition of each line over p GPUs becomes P partitions of the
 * line inside one GPU; the paper's neighbour exchange (PDD) and all-gather
 * (PPT) become on-chip exchanges.
 *
 * Conventions shared by every call
 * --------------------------------
 * A line is the tridiagonal system
 *     a_j x_{j-1} + b_j x_j + c_j x_{j+1} = d_j,      j = 0 .. n-1
 * (the paper's A = [a_j, b_j, c_j], Sec. 3.2).  For a non-periodic line a_0
 * and c_{n-1} are not part of the matrix and are never read.  For a periodic
 * line (periodic = 1) a_0 couples row 0 to x_{n-1} and c_{n-1} couples row
 * n-1 to x_0.
 *
 * The line is split into P partitions of m = n/P consecutive rows; n must be
 * divisible by P, and m >= 2 unless P = 1 on a non-periodic line.
 * 1 <= P <= TRI_MAX_PARTITIONS.  PDD's result depends on P (it drops the
 * Z entries v_m and w_1, Sec. 3.2); PPT's does not (Eqs. (9)-(11) are exact).
 *
 * Memory: every array pointer passed to a solve is a DEVICE pointer on the
 * context's device, owned by the caller; the library never frees or keeps it
 * past the call (plans keep the pointers given at creation, see below).
 * Right-hand sides are overwritten in place by the solution (Algorithm 1
 * returns its outputs in d1, d2, d3).  Work is queued on the context's
 * stream and the call returns without waiting, unless a tri_info is passed
 * (then the call waits for the stream to fill it in).  The library's own
 * device memory is allocated only by the set-up calls (tri_create,
 * tri_reserve, tri_plan_create): a solve never allocates or frees memory
 * and waits only to fill a tri_info, so every solve called without one can
 * be recorded into a HIP graph.  One-shot solves with a
 * shared matrix keep its partition factors in the context workspace
 * (64 MiB from tri_create, grown by tri_reserve); a call that needs more
 * returns TRI_E_NOMEM before launching anything.  Calls on one context
 * share that workspace and must be queued on one stream.
 *
 * Errors: argument and shape errors are returned before anything is launched
 * and leave the data untouched.  Conditions found on the device (a zero pivot
 * in a partition block, refinement that did not converge) are recorded in a
 * sticky status word of the context and returned by tri_sync_status().
 * All FP64 arithmetic is IEEE double; FP32 arithmetic is used only where a
 * call's tri_prec asks for it.
 */
#ifndef TRI_H
#define TRI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TRI_MAX_PARTITIONS 16

typedef struct tri_ctx_s *tri_ctx;
typedef struct tri_plan_s *tri_plan;

typedef enum {
    TRI_OK = 0,
    TRI_E_ARG = 1,           /* null pointer, bad enum, negative size            */
    TRI_E_SHAPE = 2,         /* n % P != 0, m < 2, P out of range, n < 3 periodic */
    TRI_E_ZERO_PIVOT = 3,    /* a partition block hit a zero pivot (device)      */
    TRI_E_PDD_UNSAFE = 4,    /* strict PDD: a dropped entry above the tolerance  */
    TRI_E_NOT_CONVERGED = 5, /* FP32 + FP64 refinement did not converge (device) */
    TRI_E_HIP = 6,           /* a HIP runtime call failed                        */
    TRI_E_NOMEM = 7,         /* device or host allocation failed                 */
    TRI_E_UNSUPPORTED = 8    /* valid request outside what the library handles  */
} tri_status;

typedef enum { TRI_F64 = 0, TRI_F32_REFINE = 1 } tri_prec;
typedef enum { TRI_REAL = 0, TRI_COMPLEX = 1 } tri_field;
typedef enum { TRI_PDD = 0, TRI_PPT = 1 } tri_method;
typedef enum { TRI_DIR_X = 0, TRI_DIR_Y = 1, TRI_DIR_Z = 2 } tri_dir;

/* Batch of lines.  Line (b0, b1), 0 <= b0 < nb0, 0 <= b1 < nb1, has row j at
 * element  j*s_j + b0*s_b0 + b1*s_b1  of the field (strides in field
 * elements; a complex element is one interleaved (re, im) pair of doubles).
 * nb0 = 0 or nb1 = 0 is an empty batch (returns TRI_OK, launches nothing).
 * Throughput is best with s_b0 = 1 (lines side by side, rows strided) or
 * s_j = 1 (rows contiguous). */
typedef struct {
    int64_t n, nb0, nb1;
    int64_t s_j, s_b0, s_b1;
} tri_lines;

/* Coefficients: row j of line (b0, b1) reads a/b/c at
 * j*cs_j + b0*cs_b0 + b1*cs_b1.  A zero stride broadcasts: cs_b0 = cs_b1 = 0
 * is one matrix shared by all lines (factored once per call); cs_b0 = 0 with
 * cs_b1 != 0 is one matrix per b1 index.  Coefficients are real FP64 even for
 * complex fields (Sec. 2.2: real matrix, complex right-hand side). */
typedef struct {
    const double *a, *b, *c;
    int64_t cs_j, cs_b0, cs_b1;
} tri_coef;

/* Optional host-side report (pass NULL to keep the call asynchronous). */
typedef struct {
    int sweeps;           /* refinement sweeps done (0 for plain FP64)          */
    double pdd_drop_max;  /* largest |dropped Z entry| (v_m, w_1) over the call; */
                          /* PDD's error is bounded by about 4x this times |x|  */
    double resid_max;     /* FP32+refine: largest estimated remaining error of a */
                          /* line relative to |x| (|last update|^2 / |previous| */
                          /* update| / |x|, max norms); the sweeps stop below   */
                          /* 1e-13                                               */
} tri_info;

/* ---- context ------------------------------------------------------------- */

/* Create a context on HIP device `device`, queueing work on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  Allocates the status
 * word and a 64 MiB workspace (see tri_reserve).  *out receives the
 * handle. */
tri_status tri_create(tri_ctx *out, int device, void *hip_stream);
/* Release the context and its workspace (waits for its stream). */
tri_status tri_destroy(tri_ctx ctx);
/* Change the stream later calls queue on. */
tri_status tri_set_stream(tri_ctx ctx, void *hip_stream);
/* Grow the context workspace so that one-shot solves (tri_pdd_solve,
 * tri_ppt_solve, adi_sweep, poisson_wavenumber_solve, projection_step) with
 * up to `matrices` distinct shared matrices (a Poisson call has one per
 * wavenumber; a matrix per b1 index counts nb1) of up to n rows at up to P
 * partitions fit; never shrinks.  Waits for the context stream, then
 * reallocates (a set-up call: never between the launches of a graph
 * capture).  TRI_E_ARG for n < 1, P outside 1..TRI_MAX_PARTITIONS or
 * matrices < 1; TRI_E_NOMEM if the device allocation fails (the context
 * then holds no workspace until a later tri_reserve succeeds). */
tri_status tri_reserve(tri_ctx ctx, int64_t n, int P, int64_t matrices);
/* Strict PDD (Sec. 3.2 holds PDD accurate only where the entries it drops
 * from Z are negligible): with tol > 0, every later PDD solve of this
 * context -- one-shot calls, poisson_shifted_solve with TRI_PDD, and plans
 * created afterwards -- whose dropped reduced-system entries (v at a
 * partition's last row, w at its first) exceed tol sets the status word,
 * and tri_sync_status returns TRI_E_PDD_UNSAFE (the solve itself still
 * runs; nothing synchronises).  A plan's items (all shared-matrix) are
 * checked once, when tri_plan_create computes their tables; the next
 * tri_sync_status reports it.
 * TRI_F32_REFINE solves are not checked: their refinement converges to
 * A^-1 d, not to the truncated system.
 * tol = 0 (the default) turns the check off; the largest dropped entry of
 * a shared-matrix call is reported in tri_info.pdd_drop_max either way.
 * TRI_E_ARG for a negative or NaN tol. */
tri_status tri_set_pdd_tolerance(tri_ctx ctx, double tol);
/* Wait for the stream, read and clear the sticky device status word:
 * TRI_OK, TRI_E_ZERO_PIVOT, TRI_E_NOT_CONVERGED or TRI_E_PDD_UNSAFE. */
tri_status tri_sync_status(tri_ctx ctx);
/* Static English text for a status code. */
const char *tri_status_string(int status);
/* Text of the last error that this context returned (validation detail). */
const char *tri_last_error(tri_ctx ctx);

/* ---- the four solves ------------------------------------------------------ */

/* PDD over a batch of lines (Sec. 3.2, PDD paragraph; Algorithm 1 steps 1-7):
 * per partition the local solves A~ x~ = d and A~ Y = V (Eqs. (5), (6)), the
 * 2x2 interface systems of the block-diagonal part of Z (Eq. (7) with v_m and
 * w_1 dropped), and x = x~ - Y y (Eq. (8)).  field: TRI_REAL (d_inout is
 * double*) or TRI_COMPLEX (d_inout is interleaved complex128, s_b0 must be 1).
 * prec: TRI_F64, or TRI_F32_REFINE (FP32 elimination + FP64 residual
 * refinement towards the exact A^{-1} d, at most 3 refinement sweeps after
 * the first FP32 solve; TRI_E_NOT_CONVERGED from tri_sync_status if a line's
 * estimated error is still above 1e-13; strided rows only). */
tri_status tri_pdd_solve(tri_ctx ctx, const tri_coef *coef, const tri_lines *lines,
                         tri_field field, void *d_inout, int P, int periodic,
                         tri_prec prec, tri_info *info);

/* PPT over a batch of lines (Sec. 3.2, Eqs. (9)-(11)): the same local
 * solves, the tridiagonal (cyclic when periodic) system Zbar y = E^T x~ solved
 * with partial pivoting in FP64, and x = x~ - Ybar y.  Exact for any P.
 * With coefficients per line (any cs_b0/cs_b1 != 0) and TRI_F64, the
 * partition blocks are factored with diagonal pivoting (1x1 or 2x2 pivots,
 * the local solver the PPT paragraph names), so general tridiagonal systems
 * that are not diagonally dominant solve as long as every block is
 * nonsingular; diagonally dominant rows always take 1x1 pivots.  Shared
 * matrices and PDD use 1x1 pivots.  Arguments as tri_pdd_solve. */
tri_status tri_ppt_solve(tri_ctx ctx, const tri_coef *coef, const tri_lines *lines,
                         tri_field field, void *d_inout, int P, int periodic,
                         tri_prec prec, tri_info *info);

/* The per-line PPT solve of tri_ppt_solve (TRI_REAL, TRI_F64, coefficients
 * per line: coef->cs_b0 != 0) that also records the decision of the
 * diagonal-pivoting local solver (PPT paragraph of Sec. 3.2) at every row,
 * for callers that check those decisions.  piv: device array of
 * nb0*nb1*n bytes, caller-owned; line (b0, b1) at (b1*nb0 + b0)*n, row j at
 * +j: 1 = 1x1 pivot, 2 = first row of a 2x2 pivot, 0 = its second row.
 * d_inout is overwritten by x exactly as tri_ppt_solve would.  Errors as
 * tri_ppt_solve; TRI_E_UNSUPPORTED for a shared matrix (cs_b0 == 0, whose
 * tables hold 1x1 pivots), TRI_E_ARG for a null piv with lines to solve. */
tri_status tri_ppt_pivots(tri_ctx ctx, const tri_coef *coef, const tri_lines *lines,
                          double *d_inout, int P, int periodic, unsigned char *piv);

/* One ADI sweep (Sec. 2.2, Sec. 3: one tridiagonal system per direction) over
 * the field u[Nz][Ny][Nx] (x fastest), in place.  dir: TRI_DIR_X (lines of
 * length Nx, rows contiguous), TRI_DIR_Y (length Ny, row stride Nx) or
 * TRI_DIR_Z (length Nz, row stride Nx*Ny).  a, b, c: device arrays of the
 * length of that direction, shared by every line.  method: TRI_PDD or
 * TRI_PPT.  periodic: 1 for the spanwise (z) direction of the paper. */
tri_status adi_sweep(tri_ctx ctx, int dir, double *u_inout, int64_t Nx, int64_t Ny,
                     int64_t Nz, const double *a, const double *b, const double *c,
                     int P, int periodic, int method, tri_prec prec, tri_info *info);

/* adi_sweep for callers that cannot allocate device memory or wait (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same sweep, kernels and result as adi_sweep without a
 * tri_info, with the partition factor tables in the library's static device
 * scratch of TRI_NOALLOC_SCRATCH_BYTES per GPU instead of the context
 * workspace.  Calls no hipMalloc/hipFree and never synchronises.  A sweep
 * whose tables do not fit (about 84 bytes per row of the sweep direction,
 * plus 32 P^2 bytes) returns TRI_E_NOMEM before any launch, data untouched.
 * Every call on one GPU, from any context or stream, shares that scratch:
 * calls that overlap in time race on it and must be serialised by the
 * caller (calls queued on one stream are).  Other errors as adi_sweep. */
#define TRI_NOALLOC_SCRATCH_BYTES (1u << 20)
tri_status adi_sweep_noalloc(tri_ctx ctx, int dir, double *u_inout, int64_t Nx, int64_t Ny,
                             int64_t Nz, const double *a, const double *b, const double *c,
                             int P, int periodic, int method, tri_prec prec);

/* Wall-normal Poisson solves per spanwise wavenumber (Sec. 2.2; PPT
 * paragraph of Sec. 3.2), in place on phihat[Nk][Ny][Nx] complex128
 * (interleaved re, im).  For mode k and every x-station the real matrix is
 *     a_j = ay_j,  c_j = cy_j,  b_j = -(ay_j + cy_j) - lam_k,
 * with ay_0 = cy_{Ny-1} = 0 for the Neumann ends (device arrays of length
 * Ny; lam: device array of Nk modified wavenumbers >= 0).  A mode with
 * lam_k == 0 is singular; it is gauge pinned by replacing row 0 with
 * x_0 = 0.  Solved by PPT with P partitions.  With prec = TRI_F32_REFINE,
 * modes k <= fp64_kmax stay in plain FP64. */
tri_status poisson_wavenumber_solve(tri_ctx ctx, double *phihat_inout, int64_t Nx,
                                    int64_t Ny, int64_t Nk, const double *ay,
                                    const double *cy, const double *lam, int P,
                                    tri_prec prec, int fp64_kmax, tri_info *info);

/* Wall-normal Poisson solves with a shift per x-station as well (Sec. 2.2:
 * the pressure equation transformed in both homogeneous directions; PPT
 * paragraph of Sec. 3.2), in place on phihat[Nk][Ny][Nx] complex128.  For
 * mode k and station i the real matrix is
 *     a_j = ay_j,  c_j = cy_j,  b_j = -(ay_j + cy_j) - (lamz_k + lamx_i),
 * every line with its own matrix, factored on the fly (nothing is stored).
 * A line with lamz_k + lamx_i == 0 is gauge pinned (row 0 replaced by
 * x_0 = 0).  ay, cy: device arrays of Ny (ay_0 = cy_{Ny-1} = 0); lamz: Nk,
 * lamx: Nx device arrays of shifts >= 0.  method TRI_PPT or TRI_PDD with P
 * partitions; Ny/P <= 32 rows per partition (<= 16 if P = 16), else
 * TRI_E_UNSUPPORTED.  FP64 only; asynchronous, allocates nothing; zero pivots
 * set the status word read by tri_sync_status. */
tri_status poisson_shifted_solve(tri_ctx ctx, double *phihat, int64_t Nx, int64_t Ny, int64_t Nk,
                                 const double *ay, const double *cy, const double *lamz,
                                 const double *lamx, int P, int method);

/* ---- the pressure step around the Poisson solves (Sec. 2.2) -------------
 *
 * The fractional step ends every sub-step with a projection: the divergence
 * of the intermediate velocity is Fourier transformed in the periodic
 * spanwise direction, the wall-normal Poisson systems of every wavenumber
 * are solved (poisson_wavenumber_solve), and the transformed back
 * pseudo-pressure phi corrects the velocity by its gradient.  Grid
 * (staggered in y and z, every x-station independent): cells j < Ny of
 * widths dy_j, k < Nz (periodic, width dz); v[Nz][Ny+1][Nx] on the y-faces
 * (face j below cell j; faces 0 and Ny are the walls), w[Nz][Ny][Nx] on the
 * z-faces (face k between cells k-1 and k), phi[Nz][Ny][Nx] at the cells.
 * All arrays are FP64 device arrays owned by the caller, x fastest, 8-byte
 * aligned; spectra are [Nz/2+1][Ny][Nx] complex128 (interleaved re, im),
 * 16-byte aligned (they are moved as 16-byte vectors).
 * Nz must be even with Nz/2 = 2^a 3^b 5^c <= 512 (TRI_E_SHAPE for odd or
 * Nz < 2, TRI_E_UNSUPPORTED otherwise).  Arrays one call reads and writes
 * must not overlap (TRI_E_ARG), except where stated.  Calls are
 * asynchronous on the context stream and allocate nothing. */

/* Real FFT along z of `lines` independent stations: for every station g,
 * xhat[k][g] = sum_n x[n][g] exp(-2 pi i k n / Nz), k = 0..Nz/2, with x of
 * shape [Nz][lines] (lines = Ny*Nx for a field). */
tri_status spanwise_rfft(tri_ctx ctx, const double *x, double *xhat, int64_t lines, int64_t Nz);

/* Inverse of spanwise_rfft: x[n][g] = (1/Nz) sum over the Hermitian
 * extension of xhat[.][g] (the imaginary parts of modes 0 and Nz/2 are
 * ignored). */
tri_status spanwise_irfft(tri_ctx ctx, const double *xhat, double *x, int64_t lines, int64_t Nz);

/* dhat = spanwise_rfft(D), D = (v_{j+1} - v_j)/dy_j + (w_{k+1} - w_k)/dz at
 * every cell (w periodic in k): the right-hand side of the Poisson
 * equation, fused into the transform (D is never stored).  dy: device array
 * of Ny cell widths. */
tri_status projection_divergence_rfft(tri_ctx ctx, const double *v, const double *w,
                                      const double *dy, double dz, double *dhat, int64_t Nx,
                                      int64_t Ny, int64_t Nz);

/* phi = spanwise_irfft(phihat); then the velocity correction by the
 * gradient of phi: w_k -= (phi_k - phi_{k-1})/dz (periodic) and, on the
 * interior y-faces j = 1..Ny-1, v_j -= (phi_j - phi_{j-1})/h_j with
 * h_j = (dy_{j-1} + dy_j)/2 (the wall faces are left as they are).  v and w
 * are updated in place; phihat is read only. */
tri_status projection_correct(tri_ctx ctx, const double *phihat, double *phi, double *v,
                              double *w, const double *dy, double dz, int64_t Nx, int64_t Ny,
                              int64_t Nz);

/* The whole projection: projection_divergence_rfft into phihat (workspace
 * of (Nz/2+1) Ny Nx complex128, owned by the caller), poisson_wavenumber_solve
 * on it in FP64 with P partitions (ay, cy, lam as there; for the corrected
 * velocity to be divergence free they must be the metric of this grid:
 * ay_j = 1/(dy_j h_j), cy_j = 1/(dy_j h_{j+1}), lam_k = (4/dz^2) sin^2(pi k/Nz)),
 * then projection_correct into phi.  The Poisson factors are computed on
 * every call, in the context workspace (TRI_E_NOMEM before any launch if it
 * is too small, see tri_reserve); a plan holding a Poisson item factors
 * them once. */
tri_status projection_step(tri_ctx ctx, double *v, double *w, const double *dy, double dz,
                           const double *ay, const double *cy, const double *lam, double *phihat,
                           double *phi, int64_t Nx, int64_t Ny, int64_t Nz, int P);

/* ---- the 3-D pressure step: cosine transform in x as well (Sec. 2.2) -------
 *
 * With walls at both x-ends (u = 0 on the faces i = 0 and i = Nx, Neumann
 * for phi), the pressure equation is diagonalised in x by the cosine
 * transform and in z by the Fourier transform; what remains are the shifted
 * wall-normal systems of poisson_shifted_solve with
 * lamx_i = (4/dx^2) sin^2(pi i/(2 Nx)).  u[Nz][Ny][Nx+1] lives on the
 * x-faces; everything else as for the spanwise-only step above. */

/* In place on `rows` rows of Nx complex128 values (contiguous rows, 16-byte
 * aligned): X_k = sum_n x_n cos(pi k (2n+1)/(2 Nx)), k < Nx, real and
 * imaginary parts alike.  Nx even, 2^a 3^b 5^c <= 4096 (TRI_E_SHAPE for odd
 * or Nx < 2, TRI_E_UNSUPPORTED otherwise). */
tri_status streamwise_dct(tri_ctx ctx, double *xhat, int64_t Nx, int64_t rows);
/* Its exact inverse: x_n = (X_0 + 2 sum_{k>0} X_k cos(pi k (2n+1)/(2 Nx)))/Nx. */
tri_status streamwise_idct(tri_ctx ctx, double *xhat, int64_t Nx, int64_t rows);

/* dhat = spanwise_rfft(D), D = (u_{i+1} - u_i)/dx + (v_{j+1} - v_j)/dy_j
 * + (w_{k+1} - w_k)/dz, fused into the transform. */
tri_status projection3d_divergence_rfft(tri_ctx ctx, const double *u, const double *v,
                                        const double *w, double dx, const double *dy, double dz,
                                        double *dhat, int64_t Nx, int64_t Ny, int64_t Nz);

/* projection_correct, then u_i -= (phi_i - phi_{i-1})/dx on the interior
 * x-faces i = 1..Nx-1 (the end faces are left as they are). */
tri_status projection3d_correct(tri_ctx ctx, const double *phihat, double *phi, double *u,
                                double *v, double *w, double dx, const double *dy, double dz,
                                int64_t Nx, int64_t Ny, int64_t Nz);

/* The whole 3-D projection: projection3d_divergence_rfft into phihat,
 * streamwise_dct, poisson_shifted_solve (PPT, P partitions; ay, cy, lamz,
 * lamx the metric of this grid for the result to be divergence free),
 * streamwise_idct, projection3d_correct into phi.  Every argument is checked
 * before the first launch (TRI_E_SHAPE for an odd Nx or a P that does not
 * split Ny as the solves require; TRI_E_UNSUPPORTED for an Nx that is not
 * 2^a 3^b 5^c <= 4096 or more than 32 rows a partition); allocates nothing. */
tri_status projection3d_step(tri_ctx ctx, double *u, double *v, double *w, double dx,
                             const double *dy, double dz, const double *ay, const double *cy,
                             const double *lamz, const double *lamx, double *phihat, double *phi,
                             int64_t Nx, int64_t Ny, int64_t Nz, int P);

/* ---- the fractional-step time step (Sec. 2.1-2.2) -------------------------
 *
 * One time step of the semi-implicit fractional-step method on the staggered
 * grid of the 3-D pressure step (u[Nz][Ny][Nx+1] on x-faces, v[Nz][Ny+1][Nx]
 * on y-faces, w[Nz][Ny][Nx] on z-faces, p[Nz][Ny][Nx] at cells; walls at both
 * x-ends and at y = 0, the top at y = Ny, z periodic): three sub-steps of the
 * low-storage third-order Runge-Kutta scheme (gamma = 8/15, 5/12, 3/4,
 * zeta = 0, -17/60, -5/12, alpha = gamma + zeta) for the convection terms
 * -d(u_i u_j)/dx_j (second-order central differences), Crank-Nicolson for the
 * viscous terms nu L u, approximately factored into x, y, z tridiagonal sweeps
 * of every velocity component (PDD, the paper's ADI), the previous pressure in
 * the predictor, the 3-D projection (projection3d_step, PPT shifted solves)
 * and the pressure update p += phi / (alpha dt).  Tangential components:
 * no-slip at y = 0, stress-free at the top, slip at the x-ends.  The wall faces
 * (u at i = 0, Nx; v at j = 0, Ny) must hold 0 and are left as they are. */
typedef struct tri_ns_s *tri_ns;
typedef struct {
    int64_t Nx, Ny, Nz;      /* cells                                               */
    double dx, dz;           /* uniform spacings                                    */
    const double *dy;        /* HOST array of Ny cell widths (read at ns_create)     */
    double dt, nu;           /* time step, kinematic viscosity (1/Re)               */
    int P_adi[3];            /* PDD partitions of the x, y, z sweeps                */
    int P_poisson;           /* PPT partitions of the shifted wall-normal solves    */
} tri_ns_config;
/* Set-up: validate the grid (Nx even and 2^a 3^b 5^c <= 4096, Nz even with
 * Nz/2 = 2^a 3^b 5^c <= 512, P_poisson splitting Ny into <= 32 rows, P_adi as
 * the sweeps require), allocate the metric, sweep coefficients and work fields
 * (7 fields of Nx Ny Nz doubles and one spectrum) and create two sweep plans
 * per sub-step (x and y sweeps; z sweeps; factors computed here; their
 * strided solves of one kernel instance batched).  Where the z sweeps run
 * the strided kernel with at most 24 rows a partition chunk, they add their
 * solutions into u, v, w directly (the velocity update fused into their
 * stores; the same arithmetic, one add per unknown): two lines per lane into
 * v and w where the plan chose that shape and the step's v, w are 16-byte
 * aligned, one line per lane otherwise; else a separate update kernel does.
 * The pressure update is made by the projection's last kernel.  Environment:
 * TRI_NS_FUSE=0 forces the separate update, TRI_NS_FUSE=1 makes ns_create
 * return TRI_E_UNSUPPORTED where the fused form is not available.
 * Synchronises the context stream. */
tri_status ns_create(tri_ctx ctx, const tri_ns_config *cfg, tri_ns *out);
/* One time step, in place on the caller's device fields u, v, w, p (disjoint,
 * 8-byte aligned); asynchronous on the context stream, allocates nothing.
 * Zero pivots and PDD checks are reported by tri_sync_status. */
tri_status ns_step(tri_ns ns, double *u, double *v, double *w, double *p);
tri_status ns_destroy(tri_ns ns);

/* ---- plans: factor once, execute many times, capture as a HIP graph ------ */

typedef enum { TRI_ITEM_ADI_X = 0, TRI_ITEM_ADI_Y = 1, TRI_ITEM_ADI_Z = 2,
               TRI_ITEM_POISSON = 3 } tri_item_kind;

/* One piece of a time step's tridiagonal work.  field: u (ADI, double
 * [Nz][Ny][Nx]) or phihat (POISSON, complex128 [Nz][Ny][Nx] with Nz = Nk
 * modes).  ADI: a, b, c of the sweep direction; POISSON: a = ay, c = cy,
 * lam = modified wavenumbers, b unused.  method is TRI_PDD or TRI_PPT
 * (POISSON always uses PPT).  P = 0 lets the plan choose the partition
 * count: every P in {1, 2, 4, 8, 16} dividing the line is factored and
 * timed, and a PDD item only admits a P whose dropped reduced-system
 * entries (the spike tips PDD neglects) are at most 1e-15, so that its
 * result is the exact solution to round-off (P = 1 is plain Thomas).
 * The coefficient arrays are read once, at creation; the field pointer is
 * kept and solved in place at every execution. */
typedef struct {
    int kind;
    void *field;
    int64_t Nx, Ny, Nz;
    const double *a, *b, *c, *lam;
    int P;
    int periodic;
    int method;
} tri_item;

/* Validate the items, allocate the plan's device tables, factor every
 * matrix (partition factors, spikes, reduced-system inverses) and choose
 * the launch shapes.  All allocation happens here.  Unless the environment
 * sets TRI_AUTOTUNE=0, each item's launch shape (rows per wavefront chunk,
 * rows per lane, kernel variant) is chosen by timing the candidates on a
 * scratch copy of the item's layout (never on the caller's data);
 * TRI_AUTOTUNE_CACHE=<file> keeps the choices across processes, and the
 * read-only table tune_gfx950.txt next to libtri.so holds the tuner's MI355X
 * choices for common shapes (listed shapes are not re-timed;
 * TRI_TUNE_TABLE=<file> reads another table, TRI_TUNE_TABLE=off none).
 * Strided candidates: chunks per partition x workgroup order (line groups
 * in order, or a contiguous range of them per XCD).
 * Execution order: the items behave as if run one after another in the
 * given order; launches that touch disjoint memory are grouped into
 * dependency levels.  TRI_BATCH selects how a level is launched.  2 (the
 * default): in a plan of several FP64 items, every solve of a level -- x,
 * y and z sweeps and Poisson modes alike, each at its own partition count
 * -- runs in ONE launch of the level kernel (512-lane workgroups, each
 * holding blocks of one solve, with that solve's elimination); the tuner
 * then times partition counts and launch shapes as level entries and
 * admits only shapes the level kernel has (strided: at most 8 wavefronts
 * a block, chunks of at most 40 rows; contiguous: the register-factor
 * body with 4 rows per lane where the line splits that way), so a time
 * step is one launch per dependency level.  1: the strided solves of a
 * level that use the same kernel instance run as one batched launch, the
 * others by themselves (single-item and TRI_F32_REFINE plans always
 * group this way).  0: every solve by itself.  Synchronises the context
 * stream. */
tri_status tri_plan_create(tri_ctx ctx, const tri_item *items, int n_items, tri_prec prec,
                           tri_plan *out);
/* Queue every item's solve on the context stream (no allocation, no host
 * synchronisation). */
tri_status tri_plan_execute(tri_plan plan);
/* Record tri_plan_execute into a HIP graph and instantiate it; *graph_exec_out
 * receives the hipGraphExec_t, owned by the plan. */
tri_status tri_plan_capture(tri_plan plan, void **graph_exec_out);
/* Launch the captured graph on the context stream. */
tri_status tri_plan_graph_launch(tri_plan plan);
/* Partition count the plan uses for item i (after tuning), or -1. */
int tri_plan_item_partitions(tri_plan plan, int i);
/* Human-readable launch shape of item i (kernel, chunking, tuned value)
 * written to buf (at most len bytes, NUL-terminated); returns the length
 * the full text needs, or -1 on a bad argument. */
int tri_plan_item_describe(tri_plan plan, int i, char *buf, int len);
/* Kernel launches one tri_plan_execute queues, or -1 for a null plan. */
int tri_plan_launch_count(tri_plan plan);
tri_status tri_plan_destroy(tri_plan plan);

/* Reference copy (measurement aid; not a step of the method).  Every solve
 * reads each unknown from HBM once and writes it back once (16 B per real
 * unknown), so the rate of a plain copy on the same device bounds what any
 * solve kernel can attain; this entry point is that copy, written as the
 * fastest streaming copy on gfx950 (one pass, 16-byte non-temporal loads and
 * stores).  Copies n doubles from src to dst on the context stream,
 * asynchronously.  dst and src are device pointers owned by the caller,
 * 16-byte aligned, either equal (in place) or non-overlapping.  n = 0 does
 * nothing.  Errors (returned before any launch): TRI_E_ARG for a null
 * context, n < 0, a null or misaligned pointer with n > 0, or partially
 * overlapping ranges; TRI_E_HIP if the launch fails. */
tri_status tri_stream_copy(tri_ctx ctx, double *dst, const double *src, int64_t n);

#ifdef __cplusplus
}
#endif

#endif /* TRI_H */
