// tri_internal.h -- internal layouts shared by the host API and the HIP
// kernels of libtri (not installed, not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tri.h"

namespace tri {

constexpr int kPMax = TRI_MAX_PARTITIONS;
constexpr int kNumFactors = 5;   // beta, alpha, cp, v, w

// ---------------------------------------------------------------------------
// Factor tables of G shared matrices with n rows split into P partitions.
//
// F  [(g*5 + f)*n + J]   row J = r*m + t of matrix g:
//    f = 0: beta_J  = 1/den_J,  den_J = b_J - a~_J cp_{J-1}   (Thomas pivot)
//    f = 1: alpha_J = a~_J beta_J                              (forward mult.)
//    f = 2: cp_J    = c~_J beta_J                              (backward mult.)
//    f = 3: v_J     spike A~_r^{-1}(a_{rm} e_0)      (Eq. (6), a-corner)
//    f = 4: w_J     spike A~_r^{-1}(c_{rm+m-1} e_{m-1})  (Eq. (6), c-corner)
//    where a~, c~ are a, c with each partition's corner couplings removed.
//    Forward:  g_t = beta_t d_t - alpha_t g_{t-1};  back: x_t = g_t - cp_t x_{t+1}.
//
// IT [((g*P + r)*2 + side)*(2P) + q]   reduced-system rows of partition r:
//    side 0 gives y_left  (the paper's y_{2r-1}, multiplies v^(r)),
//    side 1 gives y_right (the paper's y_{2r+2}, multiplies w^(r)),
//    as linear combinations of the tip vector T of the line:
//    T[2q] = x~ at the first row of partition q, T[2q+1] = x~ at its last row.
//    PDD: the two nonzeros per side come from one 2x2 interface block.
//    PPT: a dense row of (pair-swap) * Zbar^{-1}, Zbar^{-1} from GEPP.
//
// flags[g]: bit 0 = mode pinned (Poisson lam == 0: row 0 replaced by x_0 = 0,
//           the right-hand side of row 0 is read as 0).
// drop[g]:  largest |v_m^(L)|, |w_1^(R)| over the interfaces (entries PDD drops).
// ---------------------------------------------------------------------------
//
// F32  [(g*5 + f)*n + J]  the same factors rounded to FP32 (refinement's
//                          inner solve).
// ORIG [(g*3 + f)*n + J]  the true matrix rows for the refinement residual,
//                          as a_J, e_J = a_J + b_J + c_J (rounded once), c_J
//                          (FP64): the residual is formed as
//                          d - a (x_{J-1} - x_J) - c (x_{J+1} - x_J) - e x_J,
//                          which avoids cancelling |b x| against |a x + c x|
//                          on nearly balanced rows; a_0 and c_{n-1} are zero
//                          unless periodic; a pinned row reads (0, 1, 0).
struct Tables {
    double *F = nullptr;
    double *IT = nullptr;
    int *flags = nullptr;
    double *drop = nullptr;
    float *F32 = nullptr;
    double *ORIG = nullptr;
    int64_t G = 0, n = 0;
    int P = 0;
    int periodic = 0;
    int method = 0;
    double pdd_tol = 0.0;    // > 0: PDD tables with a dropped entry above it set kStatusPddUnsafe
};

inline size_t tables_bytes_F(int64_t G, int64_t n) { return sizeof(double) * (size_t)(G * kNumFactors * n); }
inline size_t tables_bytes_IT(int64_t G, int P) { return sizeof(double) * (size_t)(G * P * 2 * 2 * P); }
inline size_t tables_bytes_F32(int64_t G, int64_t n) { return sizeof(float) * (size_t)(G * kNumFactors * n); }
inline size_t tables_bytes_ORIG(int64_t G, int64_t n) { return sizeof(double) * (size_t)(G * 3 * n); }

// Source of the G matrices for the factor kernel.
struct MatSrc {
    const double *a, *b, *c;   // row J of matrix g at J*cs_j + g*cs_g
    int64_t cs_j, cs_g;
    const double *lam;         // Poisson mode when non-null: b_J = -(a_J + c_J) - lam[g]
};

// Lines of a solve, after complex fields are unfolded into real lines
// (b0' = 2*b0 + component, all strides doubled).
struct LineSet {
    double *d;
    int64_t n, nb0, nb1, s_j, s_b0, s_b1;
};

struct SolveArgs {
    double *d;
    int64_t n;
    int m, P, periodic;
    int64_t s_j, nb0, nb1, s_b0, s_b1;
    int64_t ngroups0;      // strided kernel: ceil(nb0 / 64)
    int kc;                // strided kernel: chunks (wavefronts) per partition
    int blk_map;           // strided kernel: workgroup -> (line group, b1) order, see strided_block
    int lpl;               // strided kernel: lines per lane (1, or 2 with 16-byte accesses)
    int Cs;                // strided kernel: rows per chunk, m / kc
    int64_t zero;          // always 0 (keeps the compiler from caching factor loads across passes)
    int64_t g_b1;          // matrix index = b1 * g_b1 + g_off (g_b1 = 0: one shared matrix)
    int64_t g_off;
    const double *F;
    const double *IT;
    const int *flags;
    // contiguous kernel
    int C;                 // rows per lane
    int Lp;                // lanes per partition (power of two <= 64)
    int LL;                // lanes per line = P * Lp
    int LPB;               // lines per block
    int64_t nlines;        // nb0 * nb1
    // persistent LDS-staged contiguous kernel
    int stage_stride;      // doubles between staging planes
    int lines_linear;      // 1: line L starts at L * s_b0 (s_b1 == nb0 * s_b0)
    // strided kernel (one line per lane), accumulating instances only: the
    // solution is added to acc[j a_j + b0 a_b0 + b1 a_b1] instead of being
    // stored over d
    double *acc;
    int64_t a_j, a_b0, a_b1;
    // (the register-factor contiguous kernel uses C, Lp, LL, stage_stride,
    // nlines and lines_linear, one line per workgroup)
};

// FP32 elimination + FP64 residual refinement (strided layout).
struct RefineArgs {
    const float *F32;
    const double *ORIG;
    int max_sweeps;        // refinement sweeps after the first FP32 solve
    double tol;            // converged when max|update| <= tol * max|x| on a line
    int *status;
    int *sweeps_used;      // atomicMax of the refinement sweeps done, for tri_info
    unsigned long long *resid_bits;   // atomicMax of the last relative update (double bits)
    // > 0: a bound of the infinity-norm condition number of every matrix of the
    // launch (strictly diagonally dominant rows: max row sum / min dominance
    // margin); a line is then also accepted after one refinement when
    // kappa (|delta_1| / |x|)^2 <= tol
    double kappa = 0.0;
};

// One entry of a ragged batch of strided solves run by a single launch:
// workgroups [begin, begin + ngroups0 * nb1) of the launch solve `a` (with
// refinement arguments R in a refinement batch).
struct BatchEntry {
    SolveArgs a;
    RefineArgs R;
    int64_t begin;
    int method;
};

// One entry of a dependency level run by a single launch of kLevelThreads-lane
// workgroups (k_level): the entry's blocks -- the workgroups its own launch
// would use, of 64 * wpb lanes each -- are packed `sub` to a workgroup, and
// workgroups [begin, begin + ceil(nblocks / sub)) of the launch run them with
// the kernel body `body` (instance rows cmax, method, chunked or not).
enum { kLevelStrided = 0, kLevelStrided2 = 1, kLevelContig = 2, kLevelContigReg = 3 };
constexpr int kLevelThreads = 512;
constexpr int kLevelWaves = kLevelThreads / 64;
struct LevelEntry {
    SolveArgs a;
    int64_t begin;
    int64_t nblocks;
    int body, cmax, method, chunked;
    int wpb;          // wavefronts per block
    int sub;          // blocks per workgroup
    int lds_sub;      // doubles of LDS per block
    int lines;        // register-factor body: consecutive lines per block
};

// Per-line (general) coefficients.
struct GeneralArgs {
    double *d;
    int64_t n;
    int m, P, periodic, cplx;
    int64_t s_j, nb0, nb1, s_b0, s_b1;
    int64_t ngroups0;
    const double *a, *b, *c;
    int64_t cs_j, cs_b0, cs_b1;
    int *status;
    // Shifted Poisson systems (set together, with cs_b0 = cs_b1 = 0 and b
    // unused): a = ay, c = cy shared by every line, b = -(ay + cy) - sigma with
    // sigma = lamz[b1] + lamx[b0 >> cplx] per line; a line with sigma == 0 is
    // gauge pinned (row 0 replaced by x_0 = 0).
    const double *lamz = nullptr, *lamx = nullptr;
    double pdd_tol = 0.0;    // > 0: PDD lines with a dropped entry above it set kStatusPddUnsafe
    // PPT with diagonal pivoting only (nullable): every row's pivot kind, line
    // (b0, b1) at (b1 nb0 + b0) n: 1 = 1x1 pivot, 2 = first row of a 2x2 pivot,
    // 0 = its second row
    unsigned char *piv = nullptr;
};

// Host launchers (tri_kernels.hip).  All return hipError_t of the launch.
hipError_t launch_factor(const MatSrc &src, const Tables &T, int *status, hipStream_t s);
hipError_t launch_strided(const SolveArgs &a, int method, int chunk_max, hipStream_t s);
// whether launch_strided has an accumulating instance (a.acc set, lpl = 1)
bool strided_acc_supported(int method, int chunk_max);
size_t strided_lds_bytes(const SolveArgs &a);
// Two lines per lane (adjacent lines, s_b0 = 1, 16-byte aligned pairs), one
// chunk per partition (kc = 1), m <= 24.
hipError_t launch_strided2(const SolveArgs &a, int method, int chunk_max, hipStream_t s);
// Ragged batch (device table of `count` entries, sorted by begin; every
// entry would run the single-problem kernel instance <cmax, method,
// chunked> with P * kc == wavefronts).
hipError_t launch_strided_batch(const BatchEntry *entries, int count, int64_t blocks, int wavefronts, int cmax,
                                int method, bool chunked, size_t lds, hipStream_t s);
hipError_t launch_contig(const SolveArgs &a, int method, hipStream_t s);
// One dependency level in one launch (device table of `count` entries sorted
// by begin, `blocks` workgroups, `lds` bytes of LDS per workgroup).
hipError_t launch_level(const LevelEntry *entries, int count, int64_t blocks, size_t lds, hipStream_t s);
// Persistent LDS-staged variant for shared matrices (m % C == 0, C even).
hipError_t launch_contig_staged(const SolveArgs &a, int method, int grid, hipStream_t s);
size_t contig_staged_lds_bytes(const SolveArgs &a);
// Persistent grid: resident workgroups per CU x CUs (0 if the query fails).
int contig_staged_grid(const SolveArgs &a, int method);
// Persistent contiguous variant with the factors in registers (one line per
// workgroup; C in {4, 8}, P * Lp a multiple of 64 and <= 512).
hipError_t launch_contig_reg(const SolveArgs &a, int method, int grid, hipStream_t s);
// ---------------------------------------------------------------------------
// Spanwise real FFT and the projection step (tri_fft.hip).  Nz = 2M points,
// M = 2^a 3^b 5^c <= kFftMaxM; passes in the order 4, 2, 3, 5.
constexpr int kFftMaxM = 512;
constexpr int kFftMaxPasses = 12;
struct FftShape {
    int M = 0;
    int npass = 0;
    int radix[kFftMaxPasses] = {};
};
struct FftArgs {
    FftShape S;
    int64_t lines = 0;                  // stations per z-plane (Ny Nx)
    int64_t Nx = 0;                     // divergence producer: stations per y-row
    const double *x = nullptr;          // forward input rows [Nz][lines]
    const double *v = nullptr;          // divergence: v[Nz][Ny+1][Nx] (y-faces)
    const double *w = nullptr;          // divergence: w[Nz][Ny][Nx] (z-faces)
    const double *dy = nullptr;         // cell widths [Ny]
    double dz = 0.0;
    const double *u = nullptr;          // 3-D divergence: u[Nz][Ny][Nx+1] (x-faces)
    double dx = 0.0;
    double *xhat = nullptr;             // forward output [M+1][lines] complex
    const double *xhat_in = nullptr;    // inverse input [M+1][lines] complex
    double *x_out = nullptr;            // inverse output rows [Nz][lines]
    double *w_io = nullptr;             // inverse with correction: w, in place
};
enum { kFftForward = 0, kFftDivergence = 1, kFftInverse = 2, kFftInverseCorrect = 3, kFftDivergence3 = 4 };
// Streamwise cosine transform of complex rows (N = 2^a 3^b 5^c, even,
// <= kDctMaxN); S.M holds N.
constexpr int kDctMaxN = 4096;
struct DctArgs {
    FftShape S;
    double *x = nullptr;                // rows of N complex128, transformed in place
    int64_t rows = 0;
    int64_t row_stride = 0;             // complex elements between rows
};
bool dct_shape(int64_t N, FftShape &S);
hipError_t launch_dct(const DctArgs &A, bool inverse, hipStream_t s);
hipError_t launch_grad_xy(double *u, double *v, const double *phi, const double *dy, double dx, int64_t Nx,
                          int64_t Ny, int64_t Nz, hipStream_t s);
bool fft_shape(int64_t Nz, FftShape &S);
hipError_t launch_fft(const FftArgs &A, int kind, hipStream_t s);
hipError_t launch_grad_y(double *v, const double *phi, const double *dy, int64_t Nx, int64_t Ny, int64_t Nz,
                         hipStream_t s);

// Reference copy of n doubles (16-byte aligned, disjoint or equal ranges).
hipError_t launch_stream_copy(double *dst, const double *src, int64_t n, hipStream_t s);
size_t contig_reg_lds_bytes(const SolveArgs &a);
int contig_reg_grid(const SolveArgs &a, int method);
hipError_t launch_general(const GeneralArgs &a, int method, hipStream_t s);
hipError_t launch_strided_refine(const SolveArgs &a, const RefineArgs &R, int method, int chunk_max, hipStream_t s);
size_t strided_refine_lds_bytes(const SolveArgs &a);
// Ragged batch of refinement solves (same rule with the refinement kernel);
// exact: every entry's chunks have exactly cmax rows.
hipError_t launch_strided_refine_batch(const BatchEntry *entries, int count, int64_t blocks, int wavefronts,
                                       int cmax, int method, bool exact, size_t lds, hipStream_t s);
// Refinement for contiguous rows (one shared matrix; register-factor layout).
hipError_t launch_contig_refine(const SolveArgs &a, const RefineArgs &R, int method, int grid, hipStream_t s);
size_t contig_refine_lds_bytes(const SolveArgs &a);
int contig_refine_grid(const SolveArgs &a, int method);
// Refinement for per-line coefficients (general layout, m <= kGeneralRefineMaxM, P <= 8).
hipError_t launch_general_refine(const GeneralArgs &a, const RefineArgs &R, int method, hipStream_t s);
// Zero the refinement counters with a kernel (safe inside graph capture).
hipError_t launch_reset_counters(int *sweeps, unsigned long long *resid, hipStream_t s);
constexpr int kRefineMaxSweeps = 3;
constexpr int kPoissonFp64Kmax = 2;     // plans: Poisson modes k <= 2 stay FP64 under TRI_F32_REFINE
constexpr double kRefineTol = 1e-13;

// Largest m the register-resident kernels accept.
constexpr int kStridedMaxC = 80;     // rows per wavefront chunk
constexpr int kContigMaxC = 16;
constexpr int kGeneralMaxM = 32;
constexpr int kGeneralRefineMaxM = 16;
constexpr int kGeneralPPTMaxP = 8;

// Status word bits (device).
constexpr int kStatusZeroPivot = 1;
constexpr int kStatusNotConverged = 2;
constexpr int kStatusPddUnsafe = 4;       // a PDD dropped entry above the context's tolerance

}  // namespace tri
