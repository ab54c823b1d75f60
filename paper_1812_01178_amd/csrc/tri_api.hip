// tri_api.hip -- host side of the libtri C ABI (include/tri.h): argument
// validation, contexts, workspace, kernel selection, plans and HIP graphs.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "tri_internal.h"
#include "tri_ns.h"

using namespace tri;

struct tri_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    int *status_dev = nullptr;            // sticky status word
    int *sweeps_dev = nullptr;            // refinement counters (same allocation)
    unsigned long long *resid_dev = nullptr;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    double pdd_tol = 0.0;                 // strict PDD: > 0 reports dropped entries above it
    void *scratch = nullptr;              // this device's static scratch (adi_sweep_noalloc)
    std::string last_error;
};

namespace {

tri_status fail(tri_ctx ctx, tri_status st, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->last_error = buf;
    }
    return st;
}

#define HIP_TRY(ctx, expr)                                                              \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail((ctx), TRI_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// One solve request after validation, in the real view of the field.
struct Problem {
    int method = TRI_PDD;
    int P = 1, periodic = 0, cplx = 0;
    LineSet L{};
    bool general = false;
    // shared / per-b1 matrices
    MatSrc src{};
    int64_t G = 1, g_b1 = 0;
    int fp64_kmax = -1;   // Poisson: matrices g <= fp64_kmax stay FP64 under TRI_F32_REFINE
    // per-line coefficients
    const double *ga = nullptr, *gb = nullptr, *gc = nullptr;
    int64_t cs_j = 0, cs_b0 = 0, cs_b1 = 0;
    unsigned char *piv = nullptr;   // per-line PPT: pivot kinds out (nullable)
};

// Kernel choice for a shared-matrix problem.
struct Launch {
    int kind = 0;          // 0 strided, 1 contiguous, 2 contiguous staged (persistent),
                           // 3 contiguous with register factors (persistent)
    int chunk_max = 0;     // strided: CMAX instance
    int grid = 0;          // staged: persistent grid
    SolveArgs args{};
    bool refine = false;   // FP32 elimination + FP64 refinement (strided)
    RefineArgs R{};
};

// Lanes per partition and rows per lane for the staged contiguous kernel:
// C = m / Lp even, Lp a power of two <= 64 dividing m, C as close to 8 as
// allowed (<= 16).  Returns false if m has no such split.
bool staged_split(int m, int &Lp, int &C, int want_c = 0)
{
    for (int l = 1; l <= 64; l <<= 1)
        if (want_c > 0 && m % l == 0 && m / l == want_c && want_c % 2 == 0 && want_c <= 16) {
            Lp = l;
            C = want_c;
            return true;
        }
    if (want_c > 0) return false;
    for (int cap : {8, 16})
        for (int l = 1; l <= 64; l <<= 1)
            if (m % l == 0 && (m / l) % 2 == 0 && m / l <= cap) {
                Lp = l;
                C = m / l;
                return true;
            }
    return false;
}

// Split for the register-factor contiguous kernel: C rows per lane (4 or 8),
// Lp = m / C a power of two <= 64, one line of P * Lp lanes (a multiple of
// 64, at most 512) per workgroup.
bool reg_split(int m, int P, int C, int &Lp)
{
    if ((C != 4 && C != 8) || m % C != 0) return false;
    Lp = m / C;
    if (Lp > 64 || (Lp & (Lp - 1)) != 0) return false;
    const int LL = P * Lp;
    return LL % 64 == 0 && LL <= 512;
}

// Tuning values of the contiguous kernels: C (rows per lane) selects the
// LDS-staged kernel, kRegTune + C the register-factor kernel.
constexpr int kRegTune = 100;

int env_int(const char *name, int dflt)
{
    const char *v = getenv(name);
    return (v && *v) ? atoi(v) : dflt;
}

// Grouping of a plan level's launches (TRI_BATCH overrides): 0 = one launch
// each, 1 = strided launches of one kernel instance batched, 2 = one level
// launch in plans of several FP64 items (others as 1).
constexpr int kDefaultBatchMode = 2;
int batch_mode() { return env_int("TRI_BATCH", kDefaultBatchMode); }

// Whether the plan being created runs its levels as level launches: batch
// mode 2 and a plan of several FP64 items (a single item has nothing to share
// a launch with and keeps the shapes of its own kernels).  Set by
// tri_plan_create for the duration of the call; the tuner and the schedule
// read it.
thread_local bool t_level_plan = false;
bool level_plan() { return t_level_plan; }

// Chunks per partition for the refinement kernel, which keeps d and x in
// FP64 and the work vector in FP32 (5 VGPRs per row): chunks of at most 16
// rows when possible, at most 40; more than 16 rows need P*kc <= 8.
int pick_kc_refine(int m, int P, int want_kc)
{
    auto valid = [&](int kc) {
        if (kc < 1 || m % kc != 0 || P * kc > 16) return false;
        const int c = m / kc;
        // up to 16 wavefronts of up to 16 rows (128 VGPRs a lane), else up to
        // 8 wavefronts of up to 40 rows
        return c <= 40 && (c <= 16 || P * kc <= 8);
    };
    if (want_kc > 0) return valid(want_kc) ? want_kc : 0;
    for (int kc = 1; kc <= 16; ++kc)
        if (valid(kc) && m / kc <= 16) return kc;
    for (int kc = 1; kc <= 16; ++kc)
        if (valid(kc)) return kc;
    return 0;
}

tri_status check_partition(tri_ctx ctx, int64_t n, int P, int periodic)
{
    if (P < 1 || P > TRI_MAX_PARTITIONS)
        return fail(ctx, TRI_E_SHAPE, "P = %d outside 1..%d", P, TRI_MAX_PARTITIONS);
    if (n < 1) return fail(ctx, TRI_E_SHAPE, "n = %lld < 1", (long long)n);
    if (n % P != 0)
        return fail(ctx, TRI_E_SHAPE, "n = %lld not divisible by P = %d", (long long)n, P);
    const int64_t m = n / P;
    if (m < 2 && !(P == 1 && !periodic))
        return fail(ctx, TRI_E_SHAPE, "partition size m = n/P = %lld < 2", (long long)m);
    if (periodic && n < 3) return fail(ctx, TRI_E_SHAPE, "periodic line needs n >= 3");
    return TRI_OK;
}

// Two lines per lane (k_strided2): neighbouring lines adjacent in memory,
// pairs 16-byte aligned, one wavefront per partition of at most 24 rows.
bool strided2_ok(const Problem &pb, int m)
{
    return pb.L.s_b0 == 1 && pb.L.s_j % 2 == 0 && (uintptr_t)pb.L.d % 16 == 0 &&
           (pb.L.nb1 == 1 || pb.L.s_b1 % 2 == 0) && m <= 24 && pb.P <= 16;
}

int pick_chunk(int c)
{
    static const int inst[] = {8, 16, 24, 32, 40, 48, 56, 64, 72, 80};
    for (int v : inst)
        if (c <= v) return v;
    return 0;
}

// Chunks per partition for the strided kernel: kc divides m, P*kc <= 16
// wavefronts, m/kc <= 80 rows per wavefront (<= 40 when P*kc > 8).  With
// want_kc > 0 that value is used if valid; otherwise the smallest kc giving
// chunks of at most 40 rows (enough occupancy to saturate HBM), else the
// smallest valid kc.  Returns 0 if none.
int pick_kc(int m, int P, int want_kc)
{
    auto valid = [&](int kc) {
        if (kc < 1 || m % kc != 0 || P * kc > 16) return false;
        const int c = m / kc;
        return c <= kStridedMaxC && (c <= 40 || P * kc <= 8);
    };
    if (want_kc > 0) return valid(want_kc) ? want_kc : 0;
    for (int kc = 1; kc <= 16; ++kc)
        if (valid(kc) && m / kc <= 40) return kc;
    for (int kc = 1; kc <= 16; ++kc)
        if (valid(kc)) return kc;
    return 0;
}

// want: forced tuning value (strided: chunks per partition; contiguous:
// rows per lane), 0 = heuristic.  TRI_FORCE_KC / TRI_FORCE_C override it.
tri_status plan_launch(tri_ctx ctx, const Problem &pb, const Tables &T, Launch &out, int want = 0)
{
    // strided tuning values: chunks per partition + 100 * workgroup order
    // (+ 1000: two lines per lane)
    const int want_kc = want ? want % 100 : env_int("TRI_FORCE_KC", 0);
    const int want_map = want ? (want / 100) % 10 : env_int("TRI_BLK_MAP", 0);
    const int want_lpl = want ? 1 + want / 1000 : 1 + (env_int("TRI_LPL", 1) == 2);
    const int want_c = want ? want : env_int("TRI_FORCE_C", 0);
    const int64_t n = pb.L.n;
    const int P = pb.P;
    const int m = (int)(n / P);
    SolveArgs a{};
    a.d = pb.L.d;
    a.n = n;
    a.m = m;
    a.P = P;
    a.periodic = pb.periodic;
    a.s_j = pb.L.s_j;
    a.nb0 = pb.L.nb0;
    a.nb1 = pb.L.nb1;
    a.s_b0 = pb.L.s_b0;
    a.s_b1 = pb.L.s_b1;
    a.g_b1 = pb.g_b1;
    a.F = T.F;
    a.IT = T.IT;
    a.flags = T.flags;
    a.nlines = pb.L.nb0 * pb.L.nb1;
    int sLp = 0, sC = 0;
    const bool aligned = ((uintptr_t)pb.L.d % 16 == 0) && pb.L.s_b0 % 2 == 0 &&
                         (pb.L.nb1 == 1 || pb.L.s_b1 % 2 == 0);
    const bool contig_shared = pb.L.s_j == 1 && n > 1 && pb.g_b1 == 0 && n % 2 == 0 && aligned;
    a.lines_linear = (pb.L.nb1 == 1 || pb.L.s_b1 == pb.L.nb0 * pb.L.s_b0) ? 1 : 0;
    int rC = 0, rLp = 0;
    if (contig_shared) {
        if (want_c > kRegTune) {
            if (!reg_split(m, P, want_c - kRegTune, rLp))
                return fail(ctx, TRI_E_UNSUPPORTED, "register-factor kernel: no split of m = %d with C = %d", m,
                            want_c - kRegTune);
            rC = want_c - kRegTune;
        } else if (want_c == 0) {
            for (int c : {8, 4})
                if (reg_split(m, P, c, rLp)) {
                    rC = c;
                    break;
                }
        }
    }
    if (rC > 0) {
        // contiguous rows, one shared matrix: factors in registers, one line
        // per workgroup; staging planes padded against LDS bank conflicts
        a.C = rC;
        a.Lp = rLp;
        a.LL = P * rLp;
        a.LPB = 1;
        a.stage_stride = 2 * a.LL + (rC == 8 ? 8 : 16);
        out.kind = 3;
        out.args = a;
        out.grid = contig_reg_grid(a, pb.method);
        if (out.grid <= 0) return fail(ctx, TRI_E_HIP, "occupancy query for the contiguous kernel failed");
        return TRI_OK;
    }
    if (contig_shared && want_c <= kRegTune && staged_split(m, sLp, sC, want_c) && P * sLp <= 1024) {
        // contiguous rows, one shared matrix: persistent LDS-staged kernel;
        // as many lines per workgroup as fit in 1024 lanes and ~150 KB of LDS
        a.C = sC;
        a.Lp = sLp;
        a.LL = P * sLp;
        for (a.LPB = std::max(1, 1024 / a.LL); a.LPB >= 1; --a.LPB) {
            const int NT = a.LPB * a.LL;
            a.stage_stride = NT * 2 + ((8 - (NT * 2) % 32) + 32) % 32;
            if (contig_staged_lds_bytes(a) <= 150 * 1024) break;
        }
        if (a.LPB >= 1) {
            out.kind = 2;
            out.args = a;
            out.grid = contig_staged_grid(a, pb.method);
            if (out.grid <= 0) return fail(ctx, TRI_E_HIP, "occupancy query for the contiguous kernel failed");
            return TRI_OK;
        }
    }
    if (pb.L.s_j == 1 && n > 1) {
        // contiguous rows: lanes own C consecutive rows, Lp lanes per partition
        int Lp = 1;
        while (Lp < 64 && (m + Lp - 1) / Lp > 8) Lp <<= 1;
        const int C = (m + Lp - 1) / Lp;
        if (C > kContigMaxC)
            return fail(ctx, TRI_E_UNSUPPORTED, "contiguous lines with m = %d > %d", m, 64 * kContigMaxC);
        const int LL = P * Lp;
        if (LL > 1024) return fail(ctx, TRI_E_UNSUPPORTED, "contiguous line needs %d lanes", LL);
        if (C > 8 && LL > 256)
            return fail(ctx, TRI_E_UNSUPPORTED, "contiguous line with m = %d needs P <= 4", m);
        a.C = C;
        a.Lp = Lp;
        a.LL = LL;
        a.LPB = std::max(1, 256 / LL);
        out.kind = 1;
    } else {
        const int kc = pick_kc(m, P, want_kc);
        if (kc == 0)
            return fail(ctx, TRI_E_UNSUPPORTED, "strided lines: no chunking of m = %d rows over P = %d partitions", m, P);
        a.kc = kc;
        a.Cs = m / kc;
        const int cmax = pick_chunk(a.Cs);
        a.lpl = 1;
        if (want_lpl == 2) {
            if (!strided2_ok(pb, m))
                return fail(ctx, TRI_E_UNSUPPORTED, "two lines per lane need adjacent 16-byte pairs, m = %d <= 24", m);
            a.lpl = 2;
            a.kc = 1;
            a.Cs = m;
        }
        a.ngroups0 = (pb.L.nb0 + 64 * a.lpl - 1) / (64 * a.lpl);
        a.blk_map = (want_map == 1 || want_map == 2) ? want_map : 0;
        out.kind = 0;
        out.chunk_max = a.lpl == 2 ? pick_chunk(m) : cmax;
    }
    out.args = a;
    return TRI_OK;
}

hipError_t run_launch(const Launch &l, int method, hipStream_t s)
{
    if (l.args.nlines == 0) return hipSuccess;
    if (l.refine && l.kind == 3) return launch_contig_refine(l.args, l.R, method, l.grid, s);
    if (l.refine) return launch_strided_refine(l.args, l.R, method, l.chunk_max, s);
    if (l.kind == 2) return launch_contig_staged(l.args, method, l.grid, s);
    if (l.kind == 3) return launch_contig_reg(l.args, method, l.grid, s);
    if (l.kind == 0 && l.args.lpl == 2) return launch_strided2(l.args, method, l.chunk_max, s);
    return l.kind == 1 ? launch_contig(l.args, method, s) : launch_strided(l.args, method, l.chunk_max, s);
}

// The infinity-norm condition bound of a problem's shared matrices for the
// one-refinement acceptance: max_j (|a_j| + |b_j| + |c_j|) / min_j (|b_j| -
// |a_j| - |c_j|) over every matrix (||A^-1|| <= 1 / min margin for strictly
// diagonally dominant rows), or 0 where a row is not strictly dominant or the
// matrices are formed on the fly (Poisson modes) or too many to read.  Reads
// the coefficients to the host: plan creation only.
double dominance_kappa(const Problem &pb)
{
    if (pb.general || pb.src.lam || !pb.src.b || pb.G < 1 || pb.G > 64) return 0.0;
    const int64_t n = pb.L.n;
    const int64_t span = (n - 1) * pb.src.cs_j + (pb.G - 1) * pb.src.cs_g + 1;
    std::vector<double> a((size_t)span), b((size_t)span), c((size_t)span);
    if (hipMemcpy(a.data(), pb.src.a, sizeof(double) * (size_t)span, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(b.data(), pb.src.b, sizeof(double) * (size_t)span, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(c.data(), pb.src.c, sizeof(double) * (size_t)span, hipMemcpyDeviceToHost) != hipSuccess)
        return 0.0;
    double rowmax = 0.0, margin = 1e300;
    for (int64_t g = 0; g < pb.G; ++g)
        for (int64_t j = 0; j < n; ++j) {
            const int64_t J = j * pb.src.cs_j + g * pb.src.cs_g;
            const double aa = (j == 0 && !pb.periodic) ? 0.0 : std::fabs(a[(size_t)J]);
            const double cc = (j == n - 1 && !pb.periodic) ? 0.0 : std::fabs(c[(size_t)J]);
            const double bb = std::fabs(b[(size_t)J]);
            if (!std::isfinite(aa + bb + cc)) return 0.0;
            rowmax = std::max(rowmax, aa + bb + cc);
            margin = std::min(margin, bb - aa - cc);
        }
    return margin > 0.0 ? rowmax / margin : 0.0;
}

// Launch of the refinement kernel over a (sub-)problem.
tri_status plan_refine_launch(tri_ctx ctx, const Problem &pb, const Tables &T, Launch &out, int want = 0)
{
    const int64_t n = pb.L.n;
    const int P = pb.P;
    const int m = (int)(n / P);
    const int kc = pick_kc_refine(m, P, want ? want : env_int("TRI_FORCE_KC", 0));
    if (kc == 0)
        return fail(ctx, TRI_E_UNSUPPORTED, "refinement: no chunking of m = %d rows over P = %d partitions", m, P);
    SolveArgs a{};
    a.d = pb.L.d;
    a.n = n;
    a.m = m;
    a.P = P;
    a.periodic = pb.periodic;
    a.s_j = pb.L.s_j;
    a.nb0 = pb.L.nb0;
    a.nb1 = pb.L.nb1;
    a.s_b0 = pb.L.s_b0;
    a.s_b1 = pb.L.s_b1;
    a.g_b1 = pb.g_b1;
    a.F = T.F;
    a.IT = T.IT;
    a.flags = T.flags;
    a.nlines = pb.L.nb0 * pb.L.nb1;
    a.kc = kc;
    a.Cs = m / kc;
    a.ngroups0 = (pb.L.nb0 + 63) / 64;
    out.kind = 0;
    // (the instance for chunks of exactly 36 rows: the spanwise lines at P = 8)
    out.chunk_max = a.Cs <= 8 ? 8 : (a.Cs <= 16 ? 16 : (a.Cs <= 24 ? 24 : (a.Cs <= 32 ? 32 : (a.Cs == 36 ? 36 : 40))));
    out.refine = true;
    out.R = RefineArgs{T.F32, T.ORIG, kRefineMaxSweeps, kRefineTol, ctx->status_dev, ctx->sweeps_dev,
                       ctx->resid_dev};
    out.args = a;
    return TRI_OK;
}

// Refinement launch for contiguous rows: the register-factor layout (one line
// per workgroup, C = 8 or 4 rows per lane), FP32 factors and true rows in
// registers.
tri_status plan_contig_refine_launch(tri_ctx ctx, const Problem &pb, const Tables &T, Launch &out)
{
    const int64_t n = pb.L.n;
    const int P = pb.P;
    const int m = (int)(n / P);
    const bool aligned = ((uintptr_t)pb.L.d % 16 == 0) && pb.L.s_b0 % 2 == 0 &&
                         (pb.L.nb1 == 1 || pb.L.s_b1 % 2 == 0);
    if (!(pb.L.s_j == 1 && n > 1 && pb.g_b1 == 0 && n % 2 == 0 && aligned))
        return fail(ctx, TRI_E_UNSUPPORTED,
                    "TRI_F32_REFINE for contiguous rows needs one shared matrix and aligned lines of even length");
    int Lp = 0, C = 0;
    for (int c : {8, 4})
        if (reg_split(m, P, c, Lp)) {
            C = c;
            break;
        }
    if (C == 0)
        return fail(ctx, TRI_E_UNSUPPORTED, "TRI_F32_REFINE for contiguous rows: no split of m = %d over P = %d", m,
                    P);
    SolveArgs a{};
    a.d = pb.L.d;
    a.n = n;
    a.m = m;
    a.P = P;
    a.periodic = pb.periodic;
    a.s_j = 1;
    a.nb0 = pb.L.nb0;
    a.nb1 = pb.L.nb1;
    a.s_b0 = pb.L.s_b0;
    a.s_b1 = pb.L.s_b1;
    a.F = T.F;
    a.IT = T.IT;
    a.flags = T.flags;
    a.nlines = pb.L.nb0 * pb.L.nb1;
    a.lines_linear = (pb.L.nb1 == 1 || pb.L.s_b1 == pb.L.nb0 * pb.L.s_b0) ? 1 : 0;
    a.C = C;
    a.Lp = Lp;
    a.LL = P * Lp;
    a.LPB = 1;
    a.stage_stride = 2 * a.LL + (C == 8 ? 8 : 16);
    out.kind = 3;
    out.refine = true;
    out.R = RefineArgs{T.F32, T.ORIG, kRefineMaxSweeps, kRefineTol, ctx->status_dev, ctx->sweeps_dev,
                       ctx->resid_dev};
    out.args = a;
    out.grid = contig_refine_grid(a, pb.method);
    if (out.grid <= 0) return fail(ctx, TRI_E_HIP, "occupancy query for the contiguous refinement kernel failed");
    return TRI_OK;
}

// Restrict a shared-matrix problem to the b1 range [b1_lo, b1_hi).
Problem sub_b1(const Problem &pb, int64_t b1_lo, int64_t b1_hi)
{
    Problem q = pb;
    q.L.d = pb.L.d + b1_lo * pb.L.s_b1;
    q.L.nb1 = b1_hi - b1_lo;
    return q;
}

// All launches of one solve request (one, or two for Poisson under
// TRI_F32_REFINE: low wavenumbers in FP64, the rest refined).
tri_status build_launches(tri_ctx ctx, const Problem &pb, const Tables &T, tri_prec prec,
                          std::vector<Launch> &out, int want = 0)
{
    out.clear();
    if (prec == TRI_F64) {
        Launch l;
        tri_status st = plan_launch(ctx, pb, T, l, want);
        if (st) return st;
        out.push_back(l);
        return TRI_OK;
    }
    if (prec != TRI_F32_REFINE) return fail(ctx, TRI_E_ARG, "bad precision %d", (int)prec);
    if (pb.L.s_j == 1 && pb.L.n > 1) {
        Launch l;
        tri_status st = plan_contig_refine_launch(ctx, pb, T, l);
        if (st) return st;
        out.push_back(l);
        return TRI_OK;
    }
    int64_t split = 0;
    if (pb.fp64_kmax >= 0 && pb.g_b1 == 1) split = std::min<int64_t>(pb.L.nb1, (int64_t)pb.fp64_kmax + 1);
    if (split > 0) {
        Launch l;
        tri_status st = plan_launch(ctx, sub_b1(pb, 0, split), T, l);
        if (st) return st;
        out.push_back(l);
    }
    if (split < pb.L.nb1) {
        Launch l;
        tri_status st = plan_refine_launch(ctx, sub_b1(pb, split, pb.L.nb1), T, l, want);
        if (st) return st;
        l.args.g_off = split;
        out.push_back(l);
    }
    return TRI_OK;
}

size_t tables_bytes(int64_t G, int64_t n, int P)
{
    return tables_bytes_F(G, n) + tables_bytes_IT(G, P) + tables_bytes_ORIG(G, n) + tables_bytes_F32(G, n) +
           sizeof(double) * (size_t)G + sizeof(int) * (size_t)G + 256;
}

Tables carve_tables(void *base, int64_t G, int64_t n, int P, int periodic, int method)
{
    Tables T;
    char *p = (char *)base;
    T.F = (double *)p;
    p += tables_bytes_F(G, n);
    T.IT = (double *)p;
    p += tables_bytes_IT(G, P);
    T.ORIG = (double *)p;
    p += tables_bytes_ORIG(G, n);
    T.drop = (double *)p;
    p += sizeof(double) * (size_t)G;
    T.F32 = (float *)p;
    p += tables_bytes_F32(G, n);
    T.flags = (int *)p;
    T.G = G;
    T.n = n;
    T.P = P;
    T.periodic = periodic;
    T.method = method;
    return T;
}

// The context workspace is allocated by tri_create and grown only by
// tri_reserve (both set-up calls that may wait for the stream); a solve that
// needs more refuses before its first launch instead of reallocating, so no
// solve allocates, frees or waits.
constexpr size_t kDefaultWorkspaceBytes = size_t(64) << 20;

tri_status grow_ws(tri_ctx ctx, size_t bytes)
{
    if (bytes <= ctx->ws_bytes) return TRI_OK;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->ws) HIP_TRY(ctx, hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
    void *p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return fail(ctx, TRI_E_NOMEM, "workspace of %zu bytes", bytes);
    ctx->ws = p;
    ctx->ws_bytes = bytes;
    return TRI_OK;
}

tri_status need_ws(tri_ctx ctx, size_t bytes)
{
    if (bytes <= ctx->ws_bytes) return TRI_OK;
    return fail(ctx, TRI_E_NOMEM,
                "the call needs %zu workspace bytes, the context holds %zu: reserve them with tri_reserve", bytes,
                ctx->ws_bytes);
}

tri_status fill_info(tri_ctx ctx, const Tables *T, tri_info *info, bool refined = false)
{
    if (!info) return TRI_OK;
    info->sweeps = 0;
    info->resid_max = 0.0;
    info->pdd_drop_max = 0.0;
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (refined) {
        int sw = 0;
        unsigned long long rb = 0;
        HIP_TRY(ctx, hipMemcpy(&sw, ctx->sweeps_dev, sizeof(int), hipMemcpyDeviceToHost));
        HIP_TRY(ctx, hipMemcpy(&rb, ctx->resid_dev, sizeof(rb), hipMemcpyDeviceToHost));
        double rv;
        memcpy(&rv, &rb, sizeof rv);
        info->sweeps = sw;
        info->resid_max = rv;
    }
    if (T && T->G > 0) {
        std::vector<double> h((size_t)T->G);
        HIP_TRY(ctx, hipMemcpy(h.data(), T->drop, sizeof(double) * (size_t)T->G, hipMemcpyDeviceToHost));
        for (double v : h) info->pdd_drop_max = std::max(info->pdd_drop_max, v);
    }
    return TRI_OK;
}

// Run one validated problem through the context workspace, or, when `tables`
// is given, with the factor tables in that memory of `tables_cap` bytes.
tri_status run_problem(tri_ctx ctx, const Problem &pb, tri_prec prec, tri_info *info, void *tables = nullptr,
                       size_t tables_cap = 0)
{
    if (prec != TRI_F64 && prec != TRI_F32_REFINE) return fail(ctx, TRI_E_ARG, "bad precision %d", (int)prec);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const int64_t nlines = pb.L.nb0 * pb.L.nb1;
    if (nlines == 0) {
        if (info) *info = tri_info{0, 0.0, 0.0};
        return TRI_OK;
    }
    const int m = (int)(pb.L.n / pb.P);
    if (pb.general) {
        if (m > kGeneralMaxM)
            return fail(ctx, TRI_E_UNSUPPORTED, "per-line coefficients with m = %d > %d", m, kGeneralMaxM);
        if (m > 16 && pb.P > 8)
            return fail(ctx, TRI_E_UNSUPPORTED, "per-line coefficients with m = %d > 16 need P <= 8", m);
        if (pb.method == TRI_PPT && pb.periodic && pb.P > 4)
            return fail(ctx, TRI_E_UNSUPPORTED, "per-line periodic PPT needs P <= 4");
        GeneralArgs g{};
        g.d = pb.L.d;
        g.n = pb.L.n;
        g.m = m;
        g.P = pb.P;
        g.periodic = pb.periodic;
        g.cplx = pb.cplx;
        g.s_j = pb.L.s_j;
        g.nb0 = pb.L.nb0;
        g.nb1 = pb.L.nb1;
        g.s_b0 = pb.L.s_b0;
        g.s_b1 = pb.L.s_b1;
        g.ngroups0 = (pb.L.nb0 + 63) / 64;
        g.a = pb.ga;
        g.b = pb.gb;
        g.c = pb.gc;
        g.cs_j = pb.cs_j;
        g.cs_b0 = pb.cs_b0;
        g.cs_b1 = pb.cs_b1;
        g.status = ctx->status_dev;
        g.pdd_tol = ctx->pdd_tol;
        g.piv = pb.piv;
        if (prec == TRI_F32_REFINE) {
            if (m > kGeneralRefineMaxM || pb.P > 8)
                return fail(ctx, TRI_E_UNSUPPORTED, "TRI_F32_REFINE with per-line coefficients needs m <= %d, P <= 8",
                            kGeneralRefineMaxM);
            const RefineArgs R{nullptr, nullptr, kRefineMaxSweeps, kRefineTol, ctx->status_dev, ctx->sweeps_dev,
                               ctx->resid_dev};
            HIP_TRY(ctx, launch_reset_counters(ctx->sweeps_dev, ctx->resid_dev, ctx->stream));
            HIP_TRY(ctx, launch_general_refine(g, R, pb.method, ctx->stream));
            return fill_info(ctx, nullptr, info, true);
        }
        HIP_TRY(ctx, launch_general(g, pb.method, ctx->stream));
        return fill_info(ctx, nullptr, info);
    }
    const size_t tb = tables_bytes(pb.G, pb.L.n, pb.P);
    tri_status st = TRI_OK;
    if (tables && tb > tables_cap)
        return fail(ctx, TRI_E_NOMEM, "the factor tables need %zu bytes, the static scratch holds %zu", tb, tables_cap);
    if (!tables) st = need_ws(ctx, tb);
    if (st) return st;
    Tables T = carve_tables(tables ? tables : ctx->ws, pb.G, pb.L.n, pb.P, pb.periodic, pb.method);
    T.pdd_tol = prec == TRI_F32_REFINE ? 0.0 : ctx->pdd_tol;   // refinement reaches A^-1 d
    std::vector<Launch> ls;
    st = build_launches(ctx, pb, T, prec, ls);
    if (st) return st;
    HIP_TRY(ctx, launch_factor(pb.src, T, ctx->status_dev, ctx->stream));
    if (prec == TRI_F32_REFINE) HIP_TRY(ctx, launch_reset_counters(ctx->sweeps_dev, ctx->resid_dev, ctx->stream));
    for (const Launch &l : ls) HIP_TRY(ctx, run_launch(l, pb.method, ctx->stream));
    return fill_info(ctx, &T, info, prec == TRI_F32_REFINE);
}

// Validate a tri_coef/tri_lines request and build its Problem.
tri_status make_problem(tri_ctx ctx, int method, const tri_coef *coef, const tri_lines *lines,
                        tri_field field, void *d, int P, int periodic, Problem &pb)
{
    if (!coef || !lines) return fail(ctx, TRI_E_ARG, "null coef or lines");
    if (field != TRI_REAL && field != TRI_COMPLEX) return fail(ctx, TRI_E_ARG, "bad field %d", (int)field);
    if (periodic != 0 && periodic != 1) return fail(ctx, TRI_E_ARG, "periodic must be 0 or 1");
    if (lines->nb0 < 0 || lines->nb1 < 0) return fail(ctx, TRI_E_ARG, "negative batch extent");
    tri_status st = check_partition(ctx, lines->n, P, periodic);
    if (st) return st;
    const bool empty = lines->nb0 == 0 || lines->nb1 == 0;
    if (!empty && (!d || !coef->a || !coef->b || !coef->c))
        return fail(ctx, TRI_E_ARG, "null data or coefficient pointer");
    pb.method = method;
    pb.P = P;
    pb.periodic = periodic;
    pb.cplx = field == TRI_COMPLEX;
    LineSet L{(double *)d, lines->n, lines->nb0, lines->nb1, lines->s_j, lines->s_b0, lines->s_b1};
    if (pb.cplx) {
        if (lines->s_b0 != 1 && lines->nb0 > 1)
            return fail(ctx, TRI_E_UNSUPPORTED, "complex fields need s_b0 = 1");
        L.nb0 = 2 * lines->nb0;
        L.s_b0 = 1;
        L.s_j = 2 * lines->s_j;
        L.s_b1 = 2 * lines->s_b1;
    }
    pb.L = L;
    if (coef->cs_b0 == 0) {
        pb.general = false;
        pb.src = MatSrc{coef->a, coef->b, coef->c, coef->cs_j, coef->cs_b1, nullptr};
        pb.G = (coef->cs_b1 == 0) ? 1 : lines->nb1;
        pb.g_b1 = (coef->cs_b1 == 0) ? 0 : 1;
    } else {
        pb.general = true;
        pb.ga = coef->a;
        pb.gb = coef->b;
        pb.gc = coef->c;
        pb.cs_j = coef->cs_j;
        pb.cs_b0 = coef->cs_b0;
        pb.cs_b1 = coef->cs_b1;
    }
    return TRI_OK;
}

tri_status adi_problem(tri_ctx ctx, int dir, double *u, int64_t Nx, int64_t Ny, int64_t Nz,
                       const double *a, const double *b, const double *c, int P, int periodic,
                       int method, Problem &pb)
{
    if (Nx < 0 || Ny < 0 || Nz < 0) return fail(ctx, TRI_E_ARG, "negative grid extent");
    if (method != TRI_PDD && method != TRI_PPT) return fail(ctx, TRI_E_ARG, "bad method %d", method);
    tri_lines L{};
    if (dir == TRI_DIR_X) L = tri_lines{Nx, Ny, Nz, 1, Nx, Nx * Ny};
    else if (dir == TRI_DIR_Y) L = tri_lines{Ny, Nx, Nz, Nx, 1, Nx * Ny};
    else if (dir == TRI_DIR_Z) L = tri_lines{Nz, Nx, Ny, Nx * Ny, 1, Nx};
    else return fail(ctx, TRI_E_ARG, "bad direction %d", dir);
    if (L.n == 0) return fail(ctx, TRI_E_SHAPE, "empty sweep direction");
    tri_coef C{a, b, c, 1, 0, 0};
    return make_problem(ctx, method, &C, &L, TRI_REAL, u, P, periodic, pb);
}

tri_status poisson_problem(tri_ctx ctx, double *phihat, int64_t Nx, int64_t Ny, int64_t Nk,
                           const double *ay, const double *cy, const double *lam, int P, Problem &pb,
                           int fp64_kmax = -1)
{
    if (Nx < 0 || Ny < 1 || Nk < 0) return fail(ctx, TRI_E_ARG, "bad Poisson extents");
    tri_status st = check_partition(ctx, Ny, P, 0);
    if (st) return st;
    const bool empty = Nx == 0 || Nk == 0;
    if (!empty && (!phihat || !ay || !cy || !lam)) return fail(ctx, TRI_E_ARG, "null Poisson pointer");
    pb.method = TRI_PPT;
    pb.P = P;
    pb.periodic = 0;
    pb.cplx = 1;
    pb.L = LineSet{phihat, Ny, 2 * Nx, Nk, 2 * Nx, 1, 2 * Nx * Ny};
    pb.general = false;
    pb.src = MatSrc{ay, nullptr, cy, 1, 0, lam};
    pb.G = Nk;
    pb.g_b1 = 1;
    pb.fp64_kmax = fp64_kmax;
    return TRI_OK;
}

// ---------------------------------------------------------------------------
// Static scratch of adi_sweep_noalloc: the factor tables of one call live in
// this file-scope device array instead of the context workspace, so that the
// call allocates nothing.  Each GPU the library runs on holds its own copy
// until the process ends.  Host code never passes the array's name to a
// kernel or a copy (on the host it is only a stand-in, not a device address):
// tri_create looks up the device address once per device with
// hipGetSymbolAddress, with that device current, and every use goes through
// that address.  Calls on one GPU share the array: calls that overlap in time
// (other streams or contexts) race on it.  The factor kernel writes every
// table entry a solve reads, so nothing needs clearing between calls.
constexpr size_t kNoallocScratchBytes = TRI_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxScratchDevices] = {};

// The device address of this device's scratch (the device must be current);
// nullptr for device ordinals beyond the table.
tri_status bind_scratch(int device, void **out)
{
    *out = nullptr;
    if (device >= kMaxScratchDevices) return TRI_OK;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return TRI_E_HIP;
        g_scratch_dev[device] = p;
    }
    *out = g_scratch_dev[device];
    return TRI_OK;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char *tri_status_string(int status)
{
    switch (status) {
    case TRI_OK: return "success";
    case TRI_E_ARG: return "invalid argument";
    case TRI_E_SHAPE: return "invalid shape (n, P or partition size)";
    case TRI_E_ZERO_PIVOT: return "zero pivot in a partition block";
    case TRI_E_PDD_UNSAFE: return "PDD truncation above tolerance";
    case TRI_E_NOT_CONVERGED: return "iterative refinement did not converge";
    case TRI_E_HIP: return "HIP runtime error";
    case TRI_E_NOMEM: return "out of memory";
    case TRI_E_UNSUPPORTED: return "unsupported request";
    default: return "unknown status";
    }
}

const char *tri_last_error(tri_ctx ctx) { return ctx ? ctx->last_error.c_str() : "null context"; }

tri_status tri_create(tri_ctx *out, int device, void *hip_stream)
{
    if (!out) return TRI_E_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0) return TRI_E_HIP;
    if (device < 0 || device >= count) return TRI_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return TRI_E_HIP;
    void *scr = nullptr;
    if (bind_scratch(device, &scr) != TRI_OK) return TRI_E_HIP;
    tri_ctx ctx = new (std::nothrow) tri_ctx_s;
    if (!ctx) return TRI_E_NOMEM;
    ctx->device = device;
    ctx->scratch = scr;
    ctx->stream = (hipStream_t)hip_stream;
    void *words = nullptr;
    if (hipMalloc(&words, 64) != hipSuccess) {
        delete ctx;
        return TRI_E_NOMEM;
    }
    ctx->status_dev = (int *)words;
    ctx->sweeps_dev = (int *)((char *)words + 16);
    ctx->resid_dev = (unsigned long long *)((char *)words + 32);
    if (hipMemsetAsync(words, 0, 64, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
        (void)hipFree(ctx->status_dev);
        delete ctx;
        return TRI_E_HIP;
    }
    if (grow_ws(ctx, kDefaultWorkspaceBytes) != TRI_OK) {
        (void)hipFree(ctx->status_dev);
        delete ctx;
        return TRI_E_NOMEM;
    }
    *out = ctx;
    return TRI_OK;
}

tri_status tri_reserve(tri_ctx ctx, int64_t n, int P, int64_t matrices)
{
    if (!ctx) return TRI_E_ARG;
    if (n < 1 || P < 1 || P > TRI_MAX_PARTITIONS || matrices < 1)
        return fail(ctx, TRI_E_ARG, "tri_reserve: n = %lld, P = %d, matrices = %lld", (long long)n, P,
                    (long long)matrices);
    if (n > (int64_t(1) << 32) || matrices > (int64_t(1) << 32) || n * matrices > (int64_t(1) << 34))
        return fail(ctx, TRI_E_NOMEM, "tri_reserve: %lld matrices of %lld rows", (long long)matrices, (long long)n);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    return grow_ws(ctx, tables_bytes(matrices, n, P));
}

tri_status tri_destroy(tri_ctx ctx)
{
    if (!ctx) return TRI_E_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->status_dev) (void)hipFree(ctx->status_dev);
    delete ctx;
    return TRI_OK;
}

tri_status tri_stream_copy(tri_ctx ctx, double *dst, const double *src, int64_t n)
{
    if (!ctx) return TRI_E_ARG;
    if (n < 0) return fail(ctx, TRI_E_ARG, "tri_stream_copy: n = %lld < 0", (long long)n);
    if (n == 0) return TRI_OK;
    if (!dst || !src) return fail(ctx, TRI_E_ARG, "tri_stream_copy: null pointer");
    if (((uintptr_t)dst | (uintptr_t)src) & 15)
        return fail(ctx, TRI_E_ARG, "tri_stream_copy: pointers must be 16-byte aligned");
    const uintptr_t d0 = (uintptr_t)dst, s0 = (uintptr_t)src, len = (uintptr_t)n * sizeof(double);
    if (d0 != s0 && d0 < s0 + len && s0 < d0 + len)
        return fail(ctx, TRI_E_ARG, "tri_stream_copy: source and destination partially overlap");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_stream_copy(dst, src, n, ctx->stream));
    return TRI_OK;
}

tri_status tri_set_pdd_tolerance(tri_ctx ctx, double tol)
{
    if (!ctx) return TRI_E_ARG;
    if (!(tol >= 0.0)) return fail(ctx, TRI_E_ARG, "tri_set_pdd_tolerance: tolerance %g must be >= 0", tol);
    ctx->pdd_tol = tol;
    return TRI_OK;
}

tri_status tri_set_stream(tri_ctx ctx, void *hip_stream)
{
    if (!ctx) return TRI_E_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return TRI_OK;
}

tri_status tri_sync_status(tri_ctx ctx)
{
    if (!ctx) return TRI_E_ARG;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    int h = 0;
    HIP_TRY(ctx, hipMemcpy(&h, ctx->status_dev, sizeof(int), hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemset(ctx->status_dev, 0, sizeof(int)));
    if (h & kStatusZeroPivot) return fail(ctx, TRI_E_ZERO_PIVOT, "zero pivot reported by a kernel");
    if (h & kStatusNotConverged) return fail(ctx, TRI_E_NOT_CONVERGED, "refinement did not converge");
    if (h & kStatusPddUnsafe)
        return fail(ctx, TRI_E_PDD_UNSAFE, "a PDD dropped entry exceeds the tolerance %.3g", ctx->pdd_tol);
    return TRI_OK;
}

tri_status tri_pdd_solve(tri_ctx ctx, const tri_coef *coef, const tri_lines *lines, tri_field field,
                         void *d_inout, int P, int periodic, tri_prec prec, tri_info *info)
{
    if (!ctx) return TRI_E_ARG;
    Problem pb;
    tri_status st = make_problem(ctx, TRI_PDD, coef, lines, field, d_inout, P, periodic, pb);
    if (st) return st;
    return run_problem(ctx, pb, prec, info);
}

tri_status tri_ppt_solve(tri_ctx ctx, const tri_coef *coef, const tri_lines *lines, tri_field field,
                         void *d_inout, int P, int periodic, tri_prec prec, tri_info *info)
{
    if (!ctx) return TRI_E_ARG;
    Problem pb;
    tri_status st = make_problem(ctx, TRI_PPT, coef, lines, field, d_inout, P, periodic, pb);
    if (st) return st;
    return run_problem(ctx, pb, prec, info);
}

tri_status tri_ppt_pivots(tri_ctx ctx, const tri_coef *coef, const tri_lines *lines, double *d_inout, int P,
                          int periodic, unsigned char *piv)
{
    if (!ctx) return TRI_E_ARG;
    Problem pb;
    tri_status st = make_problem(ctx, TRI_PPT, coef, lines, TRI_REAL, d_inout, P, periodic, pb);
    if (st) return st;
    if (!pb.general) return fail(ctx, TRI_E_UNSUPPORTED, "pivot kinds are recorded for per-line coefficients only");
    if (pb.L.nb0 * pb.L.nb1 > 0 && !piv) return fail(ctx, TRI_E_ARG, "null pivot array");
    pb.piv = piv;
    return run_problem(ctx, pb, TRI_F64, nullptr);
}

tri_status adi_sweep(tri_ctx ctx, int dir, double *u_inout, int64_t Nx, int64_t Ny, int64_t Nz,
                     const double *a, const double *b, const double *c, int P, int periodic,
                     int method, tri_prec prec, tri_info *info)
{
    if (!ctx) return TRI_E_ARG;
    Problem pb;
    tri_status st = adi_problem(ctx, dir, u_inout, Nx, Ny, Nz, a, b, c, P, periodic, method, pb);
    if (st) return st;
    return run_problem(ctx, pb, prec, info);
}

tri_status adi_sweep_noalloc(tri_ctx ctx, int dir, double *u_inout, int64_t Nx, int64_t Ny, int64_t Nz,
                             const double *a, const double *b, const double *c, int P, int periodic, int method,
                             tri_prec prec)
{
    if (!ctx) return TRI_E_ARG;
    Problem pb;
    tri_status st = adi_problem(ctx, dir, u_inout, Nx, Ny, Nz, a, b, c, P, periodic, method, pb);
    if (st) return st;
    if (!ctx->scratch)
        return fail(ctx, TRI_E_UNSUPPORTED, "adi_sweep_noalloc: no static scratch on device %d", ctx->device);
    return run_problem(ctx, pb, prec, nullptr, ctx->scratch, kNoallocScratchBytes);
}

tri_status poisson_wavenumber_solve(tri_ctx ctx, double *phihat_inout, int64_t Nx, int64_t Ny,
                                    int64_t Nk, const double *ay, const double *cy,
                                    const double *lam, int P, tri_prec prec, int fp64_kmax,
                                    tri_info *info)
{
    if (!ctx) return TRI_E_ARG;
    Problem pb;
    tri_status st = poisson_problem(ctx, phihat_inout, Nx, Ny, Nk, ay, cy, lam, P, pb, fp64_kmax);
    if (st) return st;
    return run_problem(ctx, pb, prec, info);
}

tri_status poisson_shifted_solve(tri_ctx ctx, double *phihat, int64_t Nx, int64_t Ny, int64_t Nk, const double *ay,
                                 const double *cy, const double *lamz, const double *lamx, int P, int method)
{
    if (!ctx) return TRI_E_ARG;
    if (Nx < 0 || Ny < 1 || Nk < 0) return fail(ctx, TRI_E_ARG, "bad Poisson extents");
    if (method != TRI_PDD && method != TRI_PPT) return fail(ctx, TRI_E_ARG, "bad method %d", method);
    tri_status st = check_partition(ctx, Ny, P, 0);
    if (st) return st;
    if (Nx == 0 || Nk == 0) return TRI_OK;
    if (!phihat || !ay || !cy || !lamz || !lamx) return fail(ctx, TRI_E_ARG, "null Poisson pointer");
    const int m = (int)(Ny / P);
    if (m > kGeneralMaxM)
        return fail(ctx, TRI_E_UNSUPPORTED, "shifted Poisson systems with m = %d > %d rows per partition", m,
                    kGeneralMaxM);
    if (m > 16 && P > 8) return fail(ctx, TRI_E_UNSUPPORTED, "shifted Poisson systems with m = %d > 16 need P <= 8", m);
    if ((2 * Nx + 31) / 32 * Nk > 0x7fffffffLL) return fail(ctx, TRI_E_UNSUPPORTED, "too many lines");
    GeneralArgs g{};
    g.d = phihat;
    g.n = Ny;
    g.m = m;
    g.P = P;
    g.periodic = 0;
    g.cplx = 1;
    g.s_j = 2 * Nx;
    g.nb0 = 2 * Nx;
    g.nb1 = Nk;
    g.s_b0 = 1;
    g.s_b1 = 2 * Nx * Ny;
    g.ngroups0 = (2 * Nx + 63) / 64;
    g.a = ay;
    g.b = nullptr;
    g.c = cy;
    g.cs_j = 1;
    g.cs_b0 = 0;
    g.cs_b1 = 0;
    g.status = ctx->status_dev;
    g.pdd_tol = ctx->pdd_tol;
    g.lamz = lamz;
    g.lamx = lamx;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_general(g, method, ctx->stream));
    return TRI_OK;
}

// ---- pressure step ---------------------------------------------------------

static bool ranges_overlap(const void *p, int64_t pbytes, const void *q, int64_t qbytes)
{
    const uintptr_t a = (uintptr_t)p, b = (uintptr_t)q;
    return pbytes > 0 && qbytes > 0 && a < b + (uintptr_t)qbytes && b < a + (uintptr_t)pbytes;
}

static tri_status fft_check(tri_ctx ctx, int64_t lines, int64_t Nz, FftShape &S, const char *who)
{
    if (lines < 0) return fail(ctx, TRI_E_ARG, "%s: lines = %lld < 0", who, (long long)lines);
    if (Nz < 2 || (Nz & 1)) return fail(ctx, TRI_E_SHAPE, "%s: Nz = %lld must be even and >= 2", who, (long long)Nz);
    if (!fft_shape(Nz, S))
        return fail(ctx, TRI_E_UNSUPPORTED, "%s: Nz/2 = %lld is not 2^a 3^b 5^c <= %d", who, (long long)(Nz / 2),
                    kFftMaxM);
    return TRI_OK;
}

static bool misaligned(const void *p) { return ((uintptr_t)p & 7) != 0; }

// The arrays a whole projection writes (phihat, phi, [u,] v, w) must be
// pairwise disjoint and disjoint from dy; checked before its first launch.
static tri_status projection_arrays_disjoint(tri_ctx ctx, const char *who, const double *phihat, const double *phi,
                                             const double *u, const double *v, const double *w, const double *dy,
                                             int64_t Nx, int64_t Ny, int64_t Nz)
{
    const int64_t lines = Nx * Ny;
    const void *p[6] = {phihat, phi, v, w, u, dy};
    const int64_t nb[6] = {16 * (Nz / 2 + 1) * lines, 8 * Nz * lines, 8 * Nz * (lines + Nx), 8 * Nz * lines,
                           u ? 8 * Nz * (lines + Ny) : 0, 8 * Ny};
    for (int i = 0; i < 6; ++i)
        for (int j = i + 1; j < 5; ++j)
            if (ranges_overlap(p[i], nb[i], p[j], nb[j])) return fail(ctx, TRI_E_ARG, "%s: arrays overlap", who);
    for (int i = 0; i < 5; ++i)
        if (ranges_overlap(p[i], nb[i], dy, nb[5])) return fail(ctx, TRI_E_ARG, "%s: dy overlaps an output", who);
    return TRI_OK;
}
static bool misaligned16(const void *p) { return ((uintptr_t)p & 15) != 0; }   // complex128 spectra

tri_status spanwise_rfft(tri_ctx ctx, const double *x, double *xhat, int64_t lines, int64_t Nz)
{
    if (!ctx) return TRI_E_ARG;
    FftArgs A;
    tri_status st = fft_check(ctx, lines, Nz, A.S, "spanwise_rfft");
    if (st) return st;
    if (lines == 0) return TRI_OK;
    if (!x || !xhat || misaligned(x) || misaligned16(xhat))
        return fail(ctx, TRI_E_ARG, "spanwise_rfft: null or misaligned array");
    if (ranges_overlap(x, 8 * Nz * lines, xhat, 16 * (Nz / 2 + 1) * lines))
        return fail(ctx, TRI_E_ARG, "spanwise_rfft: x and xhat overlap");
    A.lines = lines;
    A.x = x;
    A.xhat = xhat;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_fft(A, kFftForward, ctx->stream));
    return TRI_OK;
}

tri_status spanwise_irfft(tri_ctx ctx, const double *xhat, double *x, int64_t lines, int64_t Nz)
{
    if (!ctx) return TRI_E_ARG;
    FftArgs A;
    tri_status st = fft_check(ctx, lines, Nz, A.S, "spanwise_irfft");
    if (st) return st;
    if (lines == 0) return TRI_OK;
    if (!x || !xhat || misaligned(x) || misaligned16(xhat))
        return fail(ctx, TRI_E_ARG, "spanwise_irfft: null or misaligned array");
    if (ranges_overlap(x, 8 * Nz * lines, xhat, 16 * (Nz / 2 + 1) * lines))
        return fail(ctx, TRI_E_ARG, "spanwise_irfft: x and xhat overlap");
    A.lines = lines;
    A.xhat_in = xhat;
    A.x_out = x;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_fft(A, kFftInverse, ctx->stream));
    return TRI_OK;
}

static tri_status grid_check(tri_ctx ctx, int64_t Nx, int64_t Ny, int64_t Nz, const double *dy, double dz,
                             FftShape &S, const char *who)
{
    if (Nx < 1 || Ny < 1) return fail(ctx, TRI_E_SHAPE, "%s: Nx = %lld, Ny = %lld", who, (long long)Nx, (long long)Ny);
    if (Nx > INT32_MAX || Ny > INT32_MAX || Nx * Ny > ((int64_t)1 << 40))
        return fail(ctx, TRI_E_UNSUPPORTED, "%s: grid too large", who);
    if (!dy || misaligned(dy)) return fail(ctx, TRI_E_ARG, "%s: null or misaligned dy", who);
    if (!(dz > 0.0)) return fail(ctx, TRI_E_ARG, "%s: dz must be > 0", who);
    return fft_check(ctx, Nx * Ny, Nz, S, who);
}

tri_status projection_divergence_rfft(tri_ctx ctx, const double *v, const double *w, const double *dy, double dz,
                                      double *dhat, int64_t Nx, int64_t Ny, int64_t Nz)
{
    if (!ctx) return TRI_E_ARG;
    FftArgs A;
    tri_status st = grid_check(ctx, Nx, Ny, Nz, dy, dz, A.S, "projection_divergence_rfft");
    if (st) return st;
    if (!v || !w || !dhat || misaligned(v) || misaligned(w) || misaligned16(dhat))
        return fail(ctx, TRI_E_ARG, "projection_divergence_rfft: null or misaligned array");
    const int64_t lines = Nx * Ny;
    const int64_t hb = 16 * (Nz / 2 + 1) * lines;
    if (ranges_overlap(dhat, hb, v, 8 * Nz * (lines + Nx)) || ranges_overlap(dhat, hb, w, 8 * Nz * lines) ||
        ranges_overlap(dhat, hb, dy, 8 * Ny))
        return fail(ctx, TRI_E_ARG, "projection_divergence_rfft: dhat overlaps an input");
    A.lines = lines;
    A.Nx = Nx;
    A.v = v;
    A.w = w;
    A.dy = dy;
    A.dz = dz;
    A.xhat = dhat;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_fft(A, kFftDivergence, ctx->stream));
    return TRI_OK;
}

tri_status projection_correct(tri_ctx ctx, const double *phihat, double *phi, double *v, double *w,
                              const double *dy, double dz, int64_t Nx, int64_t Ny, int64_t Nz)
{
    if (!ctx) return TRI_E_ARG;
    FftArgs A;
    tri_status st = grid_check(ctx, Nx, Ny, Nz, dy, dz, A.S, "projection_correct");
    if (st) return st;
    if (!phihat || !phi || !v || !w || misaligned16(phihat) || misaligned(phi) || misaligned(v) || misaligned(w))
        return fail(ctx, TRI_E_ARG, "projection_correct: null or misaligned array");
    const int64_t lines = Nx * Ny;
    const void *p[5] = {phihat, phi, v, w, dy};
    const int64_t nb[5] = {16 * (Nz / 2 + 1) * lines, 8 * Nz * lines, 8 * Nz * (lines + Nx), 8 * Nz * lines, 8 * Ny};
    for (int i = 0; i < 5; ++i)
        for (int j = i + 1; j < 5; ++j) {
            if (i == 0 && j == 4) continue;   // phihat and dy are both read only
            if (ranges_overlap(p[i], nb[i], p[j], nb[j]))
                return fail(ctx, TRI_E_ARG, "projection_correct: arrays overlap");
        }
    A.lines = lines;
    A.Nx = Nx;
    A.dz = dz;
    A.xhat_in = phihat;
    A.x_out = phi;
    A.w_io = w;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_fft(A, kFftInverseCorrect, ctx->stream));
    HIP_TRY(ctx, launch_grad_y(v, phi, dy, Nx, Ny, Nz, ctx->stream));
    return TRI_OK;
}

static tri_status dct_call(tri_ctx ctx, double *xhat, int64_t Nx, int64_t rows, bool inverse, const char *who)
{
    if (!ctx) return TRI_E_ARG;
    if (rows < 0) return fail(ctx, TRI_E_ARG, "%s: rows = %lld < 0", who, (long long)rows);
    if (Nx < 2 || (Nx & 1)) return fail(ctx, TRI_E_SHAPE, "%s: Nx = %lld must be even and >= 2", who, (long long)Nx);
    DctArgs A;
    if (!dct_shape(Nx, A.S))
        return fail(ctx, TRI_E_UNSUPPORTED, "%s: Nx = %lld is not 2^a 3^b 5^c <= %d", who, (long long)Nx, kDctMaxN);
    if (rows == 0) return TRI_OK;
    if (!xhat || misaligned16(xhat)) return fail(ctx, TRI_E_ARG, "%s: null or misaligned array", who);
    A.x = xhat;
    A.rows = rows;
    A.row_stride = Nx;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_dct(A, inverse, ctx->stream));
    return TRI_OK;
}

tri_status streamwise_dct(tri_ctx ctx, double *xhat, int64_t Nx, int64_t rows)
{
    return dct_call(ctx, xhat, Nx, rows, false, "streamwise_dct");
}

tri_status streamwise_idct(tri_ctx ctx, double *xhat, int64_t Nx, int64_t rows)
{
    return dct_call(ctx, xhat, Nx, rows, true, "streamwise_idct");
}

tri_status projection3d_divergence_rfft(tri_ctx ctx, const double *u, const double *v, const double *w, double dx,
                                        const double *dy, double dz, double *dhat, int64_t Nx, int64_t Ny,
                                        int64_t Nz)
{
    if (!ctx) return TRI_E_ARG;
    FftArgs A;
    tri_status st = grid_check(ctx, Nx, Ny, Nz, dy, dz, A.S, "projection3d_divergence_rfft");
    if (st) return st;
    if (!(dx > 0.0)) return fail(ctx, TRI_E_ARG, "projection3d_divergence_rfft: dx must be > 0");
    if (!u || !v || !w || !dhat || misaligned(u) || misaligned(v) || misaligned(w) || misaligned16(dhat))
        return fail(ctx, TRI_E_ARG, "projection3d_divergence_rfft: null or misaligned array");
    const int64_t lines = Nx * Ny;
    const int64_t hb = 16 * (Nz / 2 + 1) * lines;
    if (ranges_overlap(dhat, hb, u, 8 * Nz * (lines + Ny)) || ranges_overlap(dhat, hb, v, 8 * Nz * (lines + Nx)) ||
        ranges_overlap(dhat, hb, w, 8 * Nz * lines) || ranges_overlap(dhat, hb, dy, 8 * Ny))
        return fail(ctx, TRI_E_ARG, "projection3d_divergence_rfft: dhat overlaps an input");
    A.lines = lines;
    A.Nx = Nx;
    A.u = u;
    A.dx = dx;
    A.v = v;
    A.w = w;
    A.dy = dy;
    A.dz = dz;
    A.xhat = dhat;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_fft(A, kFftDivergence3, ctx->stream));
    return TRI_OK;
}

}  // extern "C"

namespace {

// projection3d_correct; with press also press += phi * pscale (the
// fractional step's pressure update, from the same read of phi).
tri_status projection3d_correct_p(tri_ctx ctx, const double *phihat, double *phi, double *u, double *v, double *w,
                                  double dx, const double *dy, double dz, int64_t Nx, int64_t Ny, int64_t Nz,
                                  double *press, double pscale)
{
    if (!ctx) return TRI_E_ARG;
    if (!(dx > 0.0)) return fail(ctx, TRI_E_ARG, "projection3d_correct: dx must be > 0");
    if (!u || misaligned(u)) return fail(ctx, TRI_E_ARG, "projection3d_correct: null or misaligned u");
    FftArgs A;
    tri_status st = grid_check(ctx, Nx, Ny, Nz, dy, dz, A.S, "projection3d_correct");
    if (st) return st;
    if (!phihat || !phi || !v || !w || misaligned16(phihat) || misaligned(phi) || misaligned(v) || misaligned(w))
        return fail(ctx, TRI_E_ARG, "projection3d_correct: null or misaligned array");
    st = projection_arrays_disjoint(ctx, "projection3d_correct", phihat, phi, u, v, w, dy, Nx, Ny, Nz);
    if (st) return st;
    A.lines = Nx * Ny;
    A.Nx = Nx;
    A.dz = dz;
    A.xhat_in = phihat;
    A.x_out = phi;
    A.w_io = w;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, launch_fft(A, kFftInverseCorrect, ctx->stream));
    if (press) HIP_TRY(ctx, launch_grad_xy_pressure(u, v, phi, dy, dx, Nx, Ny, Nz, press, pscale, ctx->stream));
    else HIP_TRY(ctx, launch_grad_xy(u, v, phi, dy, dx, Nx, Ny, Nz, ctx->stream));
    return TRI_OK;
}

// projection3d_step; with press the last kernel also adds phi * pscale to it.
tri_status projection3d_step_p(tri_ctx ctx, double *u, double *v, double *w, double dx, const double *dy, double dz,
                               const double *ay, const double *cy, const double *lamz, const double *lamx,
                               double *phihat, double *phi, int64_t Nx, int64_t Ny, int64_t Nz, int P, double *press,
                               double pscale)
{
    if (!ctx) return TRI_E_ARG;
    FftShape S, Sx;
    tri_status st = grid_check(ctx, Nx, Ny, Nz, dy, dz, S, "projection3d_step");
    if (st) return st;
    if (Nx < 2 || (Nx & 1)) return fail(ctx, TRI_E_SHAPE, "projection3d_step: Nx = %lld must be even", (long long)Nx);
    if (!dct_shape(Nx, Sx))
        return fail(ctx, TRI_E_UNSUPPORTED, "projection3d_step: Nx = %lld is not 2^a 3^b 5^c <= %d",
                    (long long)Nx, kDctMaxN);
    st = check_partition(ctx, Ny, P, 0);
    if (st) return st;
    const int m = (int)(Ny / P);
    if (m > kGeneralMaxM || (m > 16 && P > 8))
        return fail(ctx, TRI_E_UNSUPPORTED, "projection3d_step: P = %d does not split Ny = %lld into <= 32 rows", P,
                    (long long)Ny);
    if (!ay || !cy || !lamz || !lamx || !phihat || !phi || !u || !v || !w)
        return fail(ctx, TRI_E_ARG, "projection3d_step: null array");
    if (misaligned16(phihat) || misaligned(phi) || misaligned(u) || misaligned(v) || misaligned(w))
        return fail(ctx, TRI_E_ARG, "projection3d_step: misaligned array");
    if (!(dx > 0.0)) return fail(ctx, TRI_E_ARG, "projection3d_step: dx must be > 0");
    st = projection_arrays_disjoint(ctx, "projection3d_step", phihat, phi, u, v, w, dy, Nx, Ny, Nz);
    if (st) return st;
    st = projection3d_divergence_rfft(ctx, u, v, w, dx, dy, dz, phihat, Nx, Ny, Nz);
    if (st) return st;
    const int64_t nk = Nz / 2 + 1;
    st = streamwise_dct(ctx, phihat, Nx, nk * Ny);
    if (st) return st;
    st = poisson_shifted_solve(ctx, phihat, Nx, Ny, nk, ay, cy, lamz, lamx, P, TRI_PPT);
    if (st) return st;
    st = streamwise_idct(ctx, phihat, Nx, nk * Ny);
    if (st) return st;
    return projection3d_correct_p(ctx, phihat, phi, u, v, w, dx, dy, dz, Nx, Ny, Nz, press, pscale);
}

}  // namespace

extern "C" {

tri_status projection3d_correct(tri_ctx ctx, const double *phihat, double *phi, double *u, double *v, double *w,
                                double dx, const double *dy, double dz, int64_t Nx, int64_t Ny, int64_t Nz)
{
    return projection3d_correct_p(ctx, phihat, phi, u, v, w, dx, dy, dz, Nx, Ny, Nz, nullptr, 0.0);
}

tri_status projection3d_step(tri_ctx ctx, double *u, double *v, double *w, double dx, const double *dy, double dz,
                             const double *ay, const double *cy, const double *lamz, const double *lamx,
                             double *phihat, double *phi, int64_t Nx, int64_t Ny, int64_t Nz, int P)
{
    return projection3d_step_p(ctx, u, v, w, dx, dy, dz, ay, cy, lamz, lamx, phihat, phi, Nx, Ny, Nz, P, nullptr,
                               0.0);
}

tri_status projection_step(tri_ctx ctx, double *v, double *w, const double *dy, double dz, const double *ay,
                           const double *cy, const double *lam, double *phihat, double *phi, int64_t Nx,
                           int64_t Ny, int64_t Nz, int P)
{
    if (!ctx) return TRI_E_ARG;
    FftShape S;
    tri_status st = grid_check(ctx, Nx, Ny, Nz, dy, dz, S, "projection_step");
    if (st) return st;
    // every argument is validated before the first launch
    Problem pb;
    st = poisson_problem(ctx, phihat, Nx, Ny, Nz / 2 + 1, ay, cy, lam, P, pb, 0);
    if (st) return st;
    if (!phi || !v || !w) return fail(ctx, TRI_E_ARG, "projection_step: null array");
    if (misaligned16(phihat) || misaligned(phi) || misaligned(v) || misaligned(w))
        return fail(ctx, TRI_E_ARG, "projection_step: misaligned array");
    st = projection_arrays_disjoint(ctx, "projection_step", phihat, phi, nullptr, v, w, dy, Nx, Ny, Nz);
    if (st) return st;
    st = projection_divergence_rfft(ctx, v, w, dy, dz, phihat, Nx, Ny, Nz);
    if (st) return st;
    st = run_problem(ctx, pb, TRI_F64, nullptr);
    if (st) return st;
    return projection_correct(ctx, phihat, phi, v, w, dy, dz, Nx, Ny, Nz);
}

}  // extern "C"

// ============================================================================
// Autotuner: launch shape of one plan item, picked by timing the candidates
// on a zero-filled scratch field with the item's exact strides (the caller's
// data is never touched).  Results are cached per process and, if
// TRI_AUTOTUNE_CACHE names a file, across processes.
// ============================================================================
namespace {

std::mutex g_tune_mu;
std::map<std::string, int> g_tune_cache;
bool g_tune_loaded = false;

std::string tune_key(const Problem &pb, int kind)
{
    char buf[256];
    snprintf(buf, sizeof buf, "k%d m%d P%d per%d n%lld nb0 %lld nb1 %lld sj%lld sb0 %lld sb1 %lld g%lld",
             kind, pb.method, pb.P, pb.periodic, (long long)pb.L.n, (long long)pb.L.nb0,
             (long long)pb.L.nb1, (long long)pb.L.s_j, (long long)pb.L.s_b0, (long long)pb.L.s_b1,
             (long long)pb.g_b1);
    // level launches keep their own choices (only shapes the level kernel runs)
    return level_plan() ? std::string(buf) + " L" : std::string(buf);
}

void tune_cache_read(const char *path)
{
    FILE *fp = fopen(path, "r");
    if (!fp) return;
    char line[512];
    while (fgets(line, sizeof line, fp)) {
        if (line[0] == '#') continue;
        char *bar = strrchr(line, '|');
        if (!bar) continue;
        *bar = 0;
        g_tune_cache[line] = atoi(bar + 1);
    }
    fclose(fp);
}

// Tuning choices known before any timing: the table shipped next to the
// library (results of this tuner on MI355X for common shapes, read-only),
// then TRI_AUTOTUNE_CACHE, whose entries take precedence.
void tune_cache_load()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    Dl_info info;
    const char *table = getenv("TRI_TUNE_TABLE");   // another table, or "off"
    if (table && *table) {
        if (strcmp(table, "off") != 0) tune_cache_read(table);
    } else if (dladdr((void *)&tune_cache_read, &info) && info.dli_fname) {
        std::string dir(info.dli_fname);
        const size_t slash = dir.rfind('/');
        dir = slash == std::string::npos ? std::string(".") : dir.substr(0, slash);
        tune_cache_read((dir + "/tune_gfx950.txt").c_str());
    }
    const char *f = getenv("TRI_AUTOTUNE_CACHE");
    if (f && *f) tune_cache_read(f);
}

void tune_cache_store(const std::string &key, int v)
{
    g_tune_cache[key] = v;
    const char *f = getenv("TRI_AUTOTUNE_CACHE");
    if (!f || !*f) return;
    FILE *fp = fopen(f, "a");
    if (!fp) return;
    fprintf(fp, "%s|%d\n", key.c_str(), v);
    fclose(fp);
}

constexpr size_t kLevelMaxLds = 64 * 1024;   // bytes of LDS a level workgroup may take

// The level kernel's entry for an FP64 launch, if it has a body there:
// strided launches of at most 8 wavefronts with chunks of at most 40 rows
// (24 with two lines per lane) keep their launch shape; contiguous launches
// of a shared matrix run the register-factor body with 4 rows per lane where
// the line splits that way, other contiguous launches the plain body with at
// most 8 rows per lane and as many lines per workgroup as fit.
bool level_entry(const Launch &l, int method, LevelEntry &e)
{
    if (l.refine || l.args.acc || l.args.nlines == 0) return false;
    SolveArgs a = l.args;
    e = LevelEntry{};
    int rLp = 0;
    if (l.kind == 0) {
        const int w = a.P * (a.lpl == 2 ? 1 : a.kc);
        if (w > kLevelWaves || l.chunk_max > (a.lpl == 2 ? 24 : 40)) return false;
        e.body = a.lpl == 2 ? kLevelStrided2 : kLevelStrided;
        e.cmax = l.chunk_max;
        e.chunked = a.lpl == 2 ? 0 : (a.kc > 1);
        e.wpb = w;
        e.sub = kLevelWaves / w;
        e.nblocks = a.ngroups0 * a.nb1;
        e.lds_sub = a.lpl == 2 ? 2 * a.P * 128 : (int)(strided_lds_bytes(a) / sizeof(double));
    } else if ((l.kind == 2 || l.kind == 3) && reg_split(a.m, a.P, 4, rLp)) {
        // shared matrix, contiguous 16-byte-aligned lines: the register-factor
        // body with 4 rows per lane, each block a run of consecutive lines
        // (about 512 workgroups for the entry, at most 16 lines a block)
        a.C = 4;
        a.Lp = rLp;
        a.LL = a.P * rLp;
        a.LPB = 1;
        a.stage_stride = 2 * a.LL + 16;
        e.body = kLevelContigReg;
        e.cmax = 4;
        e.wpb = a.LL / 64;
        e.sub = kLevelWaves / e.wpb;
        e.lines = (int)std::max<int64_t>(1, std::min<int64_t>(16, a.nlines / (512 * (int64_t)e.sub)));
        e.nblocks = (a.nlines + e.lines - 1) / e.lines;
        e.lds_sub = (int)(contig_reg_lds_bytes(a) / sizeof(double));
    } else {
        int Lp = 1;
        while (Lp < 64 && (a.m + Lp - 1) / Lp > 8) Lp <<= 1;
        const int C = (a.m + Lp - 1) / Lp;
        const int LL = a.P * Lp;
        if (C > 8 || LL > kLevelThreads) return false;
        a.C = C;
        a.Lp = Lp;
        a.LL = LL;
        a.LPB = kLevelThreads / LL;
        e.body = kLevelContig;
        e.cmax = C <= 4 ? 4 : 8;
        e.wpb = kLevelWaves;
        e.sub = 1;
        e.nblocks = (a.nlines + a.LPB - 1) / a.LPB;
        e.lds_sub = 2 * a.P * a.LPB;
    }
    // a workgroup's LDS (one region per block it can hold) within 64 KB
    if (sizeof(double) * (size_t)e.lds_sub * (size_t)((kLevelWaves + e.wpb - 1) / e.wpb) > kLevelMaxLds) return false;
    e.a = a;
    e.method = method;
    return true;
}

// Whether every launch of `ls` has a level body (FP64 launches only).
bool level_ok(const std::vector<Launch> &ls, int method)
{
    LevelEntry e;
    for (const Launch &l : ls)
        if (l.args.nlines > 0 && !level_entry(l, method, e)) return false;
    return true;
}

// Candidate tuning values for a problem whose default launch is `base`.
std::vector<int> tune_candidates(const Problem &pb, const Launch &base)
{
    std::vector<int> c;
    const int m = (int)(pb.L.n / pb.P);
    const bool level = level_plan();
    if (base.kind == 0) {
        // chunks per partition, each with line groups in order and with
        // per-XCD contiguous ranges (+200); level launches take chunks of at
        // most 40 rows on at most 8 wavefronts
        int nk = 0;
        for (int kc = 1; kc <= 16 && nk < 4; ++kc)
            if (pick_kc(m, pb.P, kc) == kc && m / kc >= 8 &&
                (!level || (m / kc <= 40 && pb.P * kc <= kLevelWaves))) {
                c.push_back(kc);
                c.push_back(kc + 200);
                ++nk;
            }
        if (strided2_ok(pb, m) && (!level || pb.P <= kLevelWaves)) {   // two lines per lane, one wavefront per partition
            c.push_back(1001);
            c.push_back(1201);
        }
    } else if ((base.kind == 2 || base.kind == 3) && !level) {
        // (a level launch runs every contiguous solve with the plain body)
        int Lp, C;
        for (int want : {4, 8, 16})
            if (staged_split(m, Lp, C, want) && pb.P * Lp <= 1024) c.push_back(want);
        for (int want : {4, 8})
            if (reg_split(m, pb.P, want, Lp)) c.push_back(kRegTune + want);
    }
    return c;
}

}  // namespace

// One execution of `ls` (the launches of problem pb) timed on a zero-filled
// scratch buffer with pb's layout: best of seven, in ms, or -1 on failure.
static float time_on_scratch(tri_ctx ctx, const Problem &pb, std::vector<Launch> ls)
{
    const LineSet &L = pb.L;
    const int64_t span = (L.n - 1) * L.s_j + (L.nb0 - 1) * L.s_b0 + (L.nb1 - 1) * L.s_b1 + 1;
    void *scratch = nullptr;
    if (hipMalloc(&scratch, sizeof(double) * (size_t)span) != hipSuccess) return -1.f;
    for (Launch &l : ls) l.args.d = (double *)scratch + (l.args.d - L.d);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
              hipMemsetAsync(scratch, 0, sizeof(double) * (size_t)span, ctx->stream) == hipSuccess;
    // with level launches (TRI_BATCH=2) the launches are timed as the entries
    // of one level launch, the way a plan runs them
    LevelEntry *ltab = nullptr;
    int lcount = 0;
    int64_t lblocks = 0;
    size_t llds = 0;
    if (ok && level_plan() && level_ok(ls, pb.method)) {
        std::vector<LevelEntry> host;
        for (const Launch &l : ls) {
            LevelEntry e;
            if (l.args.nlines == 0 || !level_entry(l, pb.method, e)) continue;
            e.begin = lblocks;
            lblocks += (e.nblocks + e.sub - 1) / e.sub;
            llds = std::max(llds, sizeof(double) * (size_t)e.lds_sub * (size_t)((kLevelWaves + e.wpb - 1) / e.wpb));
            host.push_back(e);
        }
        lcount = (int)host.size();
        ok = lcount == 0 || (hipMalloc((void **)&ltab, sizeof(LevelEntry) * host.size()) == hipSuccess &&
                             hipMemcpy(ltab, host.data(), sizeof(LevelEntry) * host.size(),
                                       hipMemcpyHostToDevice) == hipSuccess);
    }
    auto run_all = [&]() {
        if (ltab) return launch_level(ltab, lcount, lblocks, llds, ctx->stream) == hipSuccess;
        for (const Launch &l : ls)
            if (run_launch(l, pb.method, ctx->stream) != hipSuccess) return false;
        return true;
    };
    float best = 1e30f;
    if (ok) ok = run_all();
    for (int rep = 0; ok && rep < 7; ++rep) {
        float t = 0.f;
        ok = hipEventRecord(e0, ctx->stream) == hipSuccess && run_all() &&
             hipEventRecord(e1, ctx->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&t, e0, e1) == hipSuccess;
        if (ok) best = std::min(best, t);
    }
    (void)hipStreamSynchronize(ctx->stream);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (ltab) (void)hipFree(ltab);
    (void)hipFree(scratch);
    return ok ? best : -1.f;
}

// Returns the chosen tuning value (0 = keep the heuristic launch).
static int autotune(tri_ctx ctx, const Problem &pb, const Tables &T, const Launch &base)
{
    if (env_int("TRI_AUTOTUNE", 1) == 0) return 0;
    std::vector<int> cands = tune_candidates(pb, base);
    if (cands.size() < 2) return 0;
    const std::string key = tune_key(pb, base.kind);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_cache_load();
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) return it->second;
    }
    int best = 0;
    float best_ms = 1e30f;
    for (int v : cands) {
        Launch l;
        if (plan_launch(ctx, pb, T, l, v) != TRI_OK) continue;
        const float ms = time_on_scratch(ctx, pb, {l});
        if (ms < 0.f) return 0;
        if (ms < best_ms) {
            best_ms = ms;
            best = v;
        }
    }
    if (best > 0) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_cache_store(key, best);
    }
    return best;
}

// ============================================================================
// Plans
// ============================================================================
struct tri_plan_s {
    tri_ctx ctx = nullptr;
    tri_prec prec = TRI_F64;
    int batch = 1;            // grouping of a level's launches (see kDefaultBatchMode)
    struct Item {
        Problem pb;
        Tables T;
        std::vector<Launch> launches;
        void *mem = nullptr;
        int tuned = 0;
    };
    std::vector<Item> items;
    // Execution order: launches grouped into dependency levels (a launch
    // comes after every earlier launch whose memory it overlaps); inside a
    // level, the FP64 launches run as one level launch (strided and
    // contiguous bodies side by side), or strided launches with the same
    // workgroup shape form one batched launch (see build_schedule).
    struct Step {
        int item = -1, launch = -1;                 // a single launch ...
        std::vector<std::pair<int, int>> members;   // ... or a batch of (item, launch)
        bool level = false;                         // batch run by the level kernel (table in ldev)
        LevelEntry *ldev = nullptr;
        bool refine = false;                        // batch of refinement solves
        bool exact = false;                         // ... whose chunks all have cmax rows
        bool chunked = false;
        int method = 0;
        BatchEntry *dev = nullptr;
        int count = 0, wavefronts = 0, cmax = 0;
        int64_t blocks = 0;
        size_t lds = 0;
    };
    std::vector<Step> steps;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

constexpr double kPddSafeDrop = 1e-15;   // P = 0: PDD only where the dropped entries are this small

// Problem of plan item `it` at partition count P (P = 0 is not accepted here).
tri_status item_problem(tri_ctx ctx, const tri_item &it, int P, Problem &pb)
{
    if (it.kind == TRI_ITEM_POISSON)
        return poisson_problem(ctx, (double *)it.field, it.Nx, it.Ny, it.Nz, it.a, it.c, it.lam, P, pb,
                               kPoissonFp64Kmax);
    if (it.kind >= TRI_ITEM_ADI_X && it.kind <= TRI_ITEM_ADI_Z)
        return adi_problem(ctx, it.kind - TRI_ITEM_ADI_X, (double *)it.field, it.Nx, it.Ny, it.Nz, it.a, it.b, it.c,
                           P, it.periodic, it.method, pb);
    return fail(ctx, TRI_E_ARG, "bad item kind %d", it.kind);
}

// Launches of a plan item.  Contiguous rows whose shape the refinement
// kernel does not take run the FP64 kernel under TRI_F32_REFINE.
tri_status item_launches(tri_ctx ctx, const Problem &pb, const Tables &T, tri_prec prec,
                         std::vector<Launch> &out, int want = 0)
{
    const bool contiguous = pb.L.s_j == 1 && pb.L.n > 1;
    if (prec == TRI_F32_REFINE && contiguous && build_launches(ctx, pb, T, prec, out, want) == TRI_OK) return TRI_OK;
    return build_launches(ctx, pb, T, contiguous ? TRI_F64 : prec, out, want);
}

double max_drop(const Tables &T)
{
    std::vector<double> h((size_t)T.G);
    if (hipMemcpy(h.data(), T.drop, sizeof(double) * h.size(), hipMemcpyDeviceToHost) != hipSuccess) return 1e300;
    double d = 0.0;
    for (double v : h) d = std::max(d, v);
    return d;
}

// P = 0: every partition count in {1, 2, 4, 8, 16} that divides the line is
// factored and timed on scratch memory; PDD candidates whose dropped
// reduced-system entries exceed kPddSafeDrop are skipped (P = 1 is plain
// Thomas and always exact).  Returns the fastest admissible P.
// Key of an item's partition-count choice in the tuning table (the choice
// depends on the item's kind, shape, method and precision; for PDD also on
// the coefficients, which is why a listed PDD choice is re-checked).
std::string partition_key(const tri_item &it, tri_prec prec)
{
    char buf[160];
    snprintf(buf, sizeof buf, "partitions k%d m%d per%d prec%d Nx%lld Ny%lld Nz%lld", it.kind, it.method,
             it.periodic, (int)prec, (long long)it.Nx, (long long)it.Ny, (long long)it.Nz);
    // level launches keep their own choices (timed as level entries)
    return level_plan() ? std::string(buf) + " L" : std::string(buf);
}

// The PDD admission rule for one partition count: the dropped reduced-system
// entries of the item's matrices are <= kPddSafeDrop (PPT and P = 1 always pass).
bool partitions_admissible(tri_ctx ctx, const Problem &pb)
{
    if (pb.method != TRI_PDD || pb.P == 1) return true;
    void *mem = nullptr;
    if (hipMalloc(&mem, tables_bytes(pb.G, pb.L.n, pb.P)) != hipSuccess) return false;
    Tables T = carve_tables(mem, pb.G, pb.L.n, pb.P, pb.periodic, pb.method);
    const bool ok = launch_factor(pb.src, T, ctx->status_dev, ctx->stream) == hipSuccess &&
                    hipStreamSynchronize(ctx->stream) == hipSuccess && max_drop(T) <= kPddSafeDrop;
    (void)hipFree(mem);
    return ok;
}

tri_status choose_partitions(tri_ctx ctx, const tri_item &it, tri_prec prec, int &P_out)
{
    // a choice listed in the tuning table (or the cache file) is taken as it is,
    // after the PDD admission check for these coefficients
    const std::string pkey = partition_key(it, prec);
    int listed = 0;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_cache_load();
        auto f = g_tune_cache.find(pkey);
        if (f != g_tune_cache.end()) listed = f->second;
    }
    // with level launches, a partition count whose launches have no level
    // body, or run contiguous lines with the plain body, is taken only when
    // no other is admissible
    const bool level = level_plan() && prec == TRI_F64;
    auto level_body = [&](const Problem &pb) {
        if (!level) return true;
        std::vector<Launch> ls;
        Tables T0{};
        if (item_launches(ctx, pb, T0, prec, ls) != TRI_OK) return false;
        for (const Launch &l : ls) {
            LevelEntry e;
            if (l.args.nlines > 0 && (!level_entry(l, pb.method, e) || e.body == kLevelContig)) return false;
        }
        return true;
    };
    if (listed > 0) {
        Problem pb;
        if (item_problem(ctx, it, listed, pb) == TRI_OK && partitions_admissible(ctx, pb) && level_body(pb)) {
            P_out = listed;
            return TRI_OK;
        }
    }
    int best = 0;
    float best_ms = 1e30f;
    for (int pass = 0; pass < 2 && best == 0; ++pass)
        for (int P : {1, 2, 4, 8, 16}) {
            Problem pb;
            if (item_problem(ctx, it, P, pb) != TRI_OK) continue;
            if (pass == 0 && !level_body(pb)) continue;
            void *mem = nullptr;
            if (hipMalloc(&mem, tables_bytes(pb.G, pb.L.n, pb.P)) != hipSuccess) continue;
            Tables T = carve_tables(mem, pb.G, pb.L.n, pb.P, pb.periodic, pb.method);
            std::vector<Launch> ls;
            float ms = -1.f;
            if (item_launches(ctx, pb, T, prec, ls) == TRI_OK &&
                launch_factor(pb.src, T, ctx->status_dev, ctx->stream) == hipSuccess &&
                hipStreamSynchronize(ctx->stream) == hipSuccess &&
                (pb.method != TRI_PDD || P == 1 || max_drop(T) <= kPddSafeDrop))
                ms = time_on_scratch(ctx, pb, ls);
            (void)hipFree(mem);
            if (ms >= 0.f && ms < best_ms) {
                best_ms = ms;
                best = P;
            }
        }
    if (best == 0) return fail(ctx, TRI_E_UNSUPPORTED, "no admissible partition count for item kind %d", it.kind);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_cache_store(pkey, best);
    }
    P_out = best;
    return TRI_OK;
}

struct Span {
    uintptr_t lo, hi;
};

Span launch_span(const SolveArgs &a)
{
    const int64_t span = (a.n - 1) * a.s_j + (a.nb0 - 1) * a.s_b0 + (a.nb1 - 1) * a.s_b1 + 1;
    return {(uintptr_t)a.d, (uintptr_t)(a.d + span)};
}

// Strided launches can join a batch of launches that run the same kernel
// instance: the key holds refinement (and, for it, whether every chunk has
// exactly CMAX rows), chunk instance (CMAX), method, chunking and wavefronts
// per workgroup.
bool batchable(const Launch &l) { return l.kind == 0 && l.args.nlines > 0 && l.args.lpl <= 1; }

bool refine_exact(const Launch &l) { return l.refine && l.args.Cs == l.chunk_max; }


int64_t batch_key(const Launch &l, int method)
{
    return ((((int64_t)(l.refine ? 1 : 0) * 2 + (refine_exact(l) ? 1 : 0)) * 128 + l.chunk_max) * 2 + method) *
               2 * 64 +
           (int64_t)(l.args.kc > 1 ? 64 : 0) + l.args.P * l.args.kc;
}

// Level-schedule the plan's launches and batch the strided ones (see Step).
tri_status build_schedule(tri_plan plan)
{
    tri_ctx ctx = plan->ctx;
    for (auto &st : plan->steps) {
        if (st.dev) (void)hipFree(st.dev);
        if (st.ldev) (void)hipFree(st.ldev);
    }
    plan->steps.clear();
    struct Ref {
        int item, launch, level;
        Span span;
    };
    std::vector<Ref> refs;
    int nlevels = 0;
    for (int i = 0; i < (int)plan->items.size(); ++i)
        for (int j = 0; j < (int)plan->items[(size_t)i].launches.size(); ++j) {
            const Span sp = launch_span(plan->items[(size_t)i].launches[(size_t)j].args);
            int level = 0;
            for (const Ref &r : refs)
                if (r.span.lo < sp.hi && sp.lo < r.span.hi) level = std::max(level, r.level + 1);
            refs.push_back({i, j, level, sp});
            nlevels = std::max(nlevels, level + 1);
        }
    const int mode = plan->batch;
    const bool batching = mode != 0;
    for (int lev = 0; lev < nlevels; ++lev) {
        if (mode == 2) {
            // one level launch for every launch of the level that has a body there
            std::vector<LevelEntry> host;
            tri_plan_s::Step st;
            st.level = true;
            int64_t blocks = 0;
            size_t lds = 0;
            for (const Ref &r : refs) {
                if (r.level != lev) continue;
                const auto &item = plan->items[(size_t)r.item];
                LevelEntry e;
                if (!level_entry(item.launches[(size_t)r.launch], item.pb.method, e)) continue;
                e.begin = blocks;
                blocks += (e.nblocks + e.sub - 1) / e.sub;
                lds = std::max(lds, sizeof(double) * (size_t)e.lds_sub * (size_t)((kLevelWaves + e.wpb - 1) / e.wpb));
                host.push_back(e);
                st.members.push_back({r.item, r.launch});
            }
            if (host.size() >= 2) {
                st.count = (int)host.size();
                st.blocks = blocks;
                st.lds = lds;
                const size_t bytes = sizeof(LevelEntry) * host.size();
                if (hipMalloc((void **)&st.ldev, bytes) != hipSuccess) return fail(ctx, TRI_E_NOMEM, "level table");
                plan->steps.push_back(st);
                HIP_TRY(ctx, hipMemcpy(st.ldev, host.data(), bytes, hipMemcpyHostToDevice));
            }
            const bool merged = host.size() >= 2;
            for (const Ref &r : refs) {
                if (r.level != lev) continue;
                bool in = false;
                if (merged)
                    for (const auto &mb : st.members) in = in || (mb.first == r.item && mb.second == r.launch);
                if (in) continue;
                tri_plan_s::Step one;
                one.item = r.item;
                one.launch = r.launch;
                plan->steps.push_back(one);
            }
            continue;
        }
        std::vector<Ref> cand;
        for (const Ref &r : refs) {
            if (r.level != lev) continue;
            const Launch &l = plan->items[(size_t)r.item].launches[(size_t)r.launch];
            if (batching && batchable(l)) {
                cand.push_back(r);
            } else {
                tri_plan_s::Step st;
                st.item = r.item;
                st.launch = r.launch;
                plan->steps.push_back(st);
            }
        }
        std::map<int64_t, std::vector<Ref>> groups;
        for (const Ref &r : cand) {
            const auto &item = plan->items[(size_t)r.item];
            groups[batch_key(item.launches[(size_t)r.launch], item.pb.method)].push_back(r);
        }
        for (auto &kv : groups) {
            tri_plan_s::Step st;
            if (kv.second.size() == 1) {
                st.item = kv.second[0].item;
                st.launch = kv.second[0].launch;
                plan->steps.push_back(st);
                continue;
            }
            std::vector<BatchEntry> host;
            const Launch &l0 = plan->items[(size_t)kv.second[0].item].launches[(size_t)kv.second[0].launch];
            st.refine = l0.refine;
            st.exact = refine_exact(l0);
            st.cmax = l0.chunk_max;
            st.chunked = l0.args.kc > 1;
            st.method = plan->items[(size_t)kv.second[0].item].pb.method;
            st.wavefronts = l0.args.P * l0.args.kc;
            for (const Ref &r : kv.second) {
                const auto &item = plan->items[(size_t)r.item];
                const Launch &l = item.launches[(size_t)r.launch];
                BatchEntry e{};
                e.a = l.args;
                e.R = l.R;
                e.begin = st.blocks;
                e.method = item.pb.method;
                host.push_back(e);
                st.blocks += l.args.ngroups0 * l.args.nb1;
                st.lds = std::max(st.lds, st.refine ? strided_refine_lds_bytes(l.args) : strided_lds_bytes(l.args));
                st.members.push_back({r.item, r.launch});
            }
            st.count = (int)host.size();
            const size_t bytes = sizeof(BatchEntry) * host.size();
            if (hipMalloc((void **)&st.dev, bytes) != hipSuccess) return fail(ctx, TRI_E_NOMEM, "batch table");
            plan->steps.push_back(st);
            HIP_TRY(ctx, hipMemcpy(st.dev, host.data(), bytes, hipMemcpyHostToDevice));
        }
    }
    return TRI_OK;
}

hipError_t run_step(const tri_plan_s &plan, const tri_plan_s::Step &st, hipStream_t s)
{
    if (st.members.empty()) {
        const auto &item = plan.items[(size_t)st.item];
        return run_launch(item.launches[(size_t)st.launch], item.pb.method, s);
    }
    if (st.level) return launch_level(st.ldev, st.count, st.blocks, st.lds, s);
    if (st.refine)
        return launch_strided_refine_batch(st.dev, st.count, st.blocks, st.wavefronts, st.cmax, st.method, st.exact,
                                           st.lds, s);
    return launch_strided_batch(st.dev, st.count, st.blocks, st.wavefronts, st.cmax, st.method, st.chunked, st.lds,
                                s);
}

}  // namespace

extern "C" {

tri_status tri_plan_destroy(tri_plan plan)
{
    if (!plan) return TRI_E_ARG;
    (void)hipSetDevice(plan->ctx->device);
    (void)hipStreamSynchronize(plan->ctx->stream);
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
    for (auto &it : plan->items)
        if (it.mem) (void)hipFree(it.mem);
    for (auto &st : plan->steps) {
        if (st.dev) (void)hipFree(st.dev);
        if (st.ldev) (void)hipFree(st.ldev);
    }
    delete plan;
    return TRI_OK;
}

}  // extern "C"

namespace {

// Plan creation with the grouping `mode` of its levels (see kDefaultBatchMode).
tri_status plan_create(tri_ctx ctx, const tri_item *items, int n_items, tri_prec prec, int mode, tri_plan *out)
{
    if (!ctx || !out || (n_items > 0 && !items) || n_items < 0) return TRI_E_ARG;
    *out = nullptr;
    if (prec != TRI_F64 && prec != TRI_F32_REFINE) return fail(ctx, TRI_E_ARG, "bad precision %d", (int)prec);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    tri_plan plan = new (std::nothrow) tri_plan_s;
    if (!plan) return TRI_E_NOMEM;
    plan->ctx = ctx;
    plan->prec = prec;
    plan->items.resize((size_t)n_items);
    struct LevelScope {
        explicit LevelScope(bool on) { t_level_plan = on; }
        ~LevelScope() { t_level_plan = false; }
    } level_scope(mode == 2 && n_items >= 2 && prec == TRI_F64);
    plan->batch = level_plan() ? 2 : std::min(mode, 1);
    for (int i = 0; i < n_items; ++i) {
        const tri_item &it = items[i];
        tri_plan_s::Item &pi = plan->items[(size_t)i];
        int P = it.P;
        if (it.kind < TRI_ITEM_ADI_X || it.kind > TRI_ITEM_POISSON) {
            tri_plan_destroy(plan);
            return fail(ctx, TRI_E_ARG, "item %d: bad kind %d", i, it.kind);
        }
        tri_status st = P == 0 ? choose_partitions(ctx, it, prec, P) : TRI_OK;
        if (!st) st = item_problem(ctx, it, P, pi.pb);
        if (st) {
            tri_plan_destroy(plan);
            return st;
        }
        const Problem &pb = pi.pb;
        const size_t bytes = tables_bytes(pb.G, pb.L.n, pb.P);
        if (hipMalloc(&pi.mem, bytes) != hipSuccess) {
            tri_plan_destroy(plan);
            return fail(ctx, TRI_E_NOMEM, "plan tables of %zu bytes", bytes);
        }
        pi.T = carve_tables(pi.mem, pb.G, pb.L.n, pb.P, pb.periodic, pb.method);
        pi.T.pdd_tol = prec == TRI_F32_REFINE ? 0.0 : ctx->pdd_tol;   // refinement reaches A^-1 d
        st = item_launches(ctx, pb, pi.T, prec, pi.launches);
        if (st) {
            tri_plan_destroy(plan);
            return st;
        }
        hipError_t e = launch_factor(pb.src, pi.T, ctx->status_dev, ctx->stream);
        if (e == hipSuccess && pi.launches.size() == 1 && !pi.launches[0].refine) {
            const int v = autotune(ctx, pb, pi.T, pi.launches[0]);
            if (v > 0 && item_launches(ctx, pb, pi.T, prec, pi.launches, v) != TRI_OK)
                (void)item_launches(ctx, pb, pi.T, prec, pi.launches);
            pi.tuned = v;
        }
        if (prec == TRI_F32_REFINE) {
            // the condition bound that lets a line of a well-conditioned matrix
            // be accepted after one refinement (read from the coefficients here,
            // never in a solve)
            const double kap = dominance_kappa(pb);
            for (Launch &l : pi.launches)
                if (l.refine) l.R.kappa = kap;
        }
        if (e != hipSuccess) {
            tri_plan_destroy(plan);
            return fail(ctx, TRI_E_HIP, "factor launch: %s", hipGetErrorString(e));
        }
    }
    tri_status st = build_schedule(plan);
    if (st) {
        tri_plan_destroy(plan);
        return st;
    }
    *out = plan;
    return TRI_OK;
}

}  // namespace

extern "C" {

tri_status tri_plan_create(tri_ctx ctx, const tri_item *items, int n_items, tri_prec prec,
                           tri_plan *out)
{
    return plan_create(ctx, items, n_items, prec, batch_mode(), out);
}

tri_status tri_plan_execute(tri_plan plan)
{
    if (!plan) return TRI_E_ARG;
    tri_ctx ctx = plan->ctx;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    for (const auto &st : plan->steps) HIP_TRY(ctx, run_step(*plan, st, ctx->stream));
    return TRI_OK;
}

tri_status tri_plan_capture(tri_plan plan, void **graph_exec_out)
{
    if (!plan) return TRI_E_ARG;
    tri_ctx ctx = plan->ctx;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (!plan->cap_stream) HIP_TRY(ctx, hipStreamCreateWithFlags(&plan->cap_stream, hipStreamNonBlocking));
    if (plan->exec) {
        (void)hipGraphExecDestroy(plan->exec);
        plan->exec = nullptr;
    }
    if (plan->graph) {
        (void)hipGraphDestroy(plan->graph);
        plan->graph = nullptr;
    }
    HIP_TRY(ctx, hipStreamBeginCapture(plan->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (const auto &st : plan->steps) {
        e = run_step(*plan, st, plan->cap_stream);
        if (e != hipSuccess) break;
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(plan->cap_stream, &g);
    if (e != hipSuccess) return fail(ctx, TRI_E_HIP, "capture launch: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(ctx, TRI_E_HIP, "end capture: %s", hipGetErrorString(e2));
    plan->graph = g;
    HIP_TRY(ctx, hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0));
    if (graph_exec_out) *graph_exec_out = (void *)plan->exec;
    return TRI_OK;
}

tri_status tri_plan_graph_launch(tri_plan plan)
{
    if (!plan) return TRI_E_ARG;
    if (!plan->exec) return fail(plan->ctx, TRI_E_ARG, "plan has no captured graph");
    HIP_TRY(plan->ctx, hipSetDevice(plan->ctx->device));
    HIP_TRY(plan->ctx, hipGraphLaunch(plan->exec, plan->ctx->stream));
    return TRI_OK;
}

int tri_plan_item_partitions(tri_plan plan, int i)
{
    if (!plan || i < 0 || i >= (int)plan->items.size()) return -1;
    return plan->items[(size_t)i].pb.P;
}

int tri_plan_item_describe(tri_plan plan, int i, char *buf, int len)
{
    if (!plan || i < 0 || i >= (int)plan->items.size() || !buf || len <= 0) return -1;
    const auto &it = plan->items[(size_t)i];
    std::string out;
    for (const Launch &l : it.launches) {
        static const char *const kinds[] = {"strided", "contiguous", "contiguous-staged", "contiguous-reg"};
        const char *kind = l.refine ? (l.kind == 3 ? "contiguous-refine" : "strided-refine") : kinds[l.kind];
        char tmp[200];
        snprintf(tmp, sizeof tmp, "%s%s P=%d m=%d kc=%d Cs=%d C=%d Lp=%d LPB=%d grid=%d lines=%lld", out.empty() ? "" : " + ",
                 kind, it.pb.P, l.args.m, l.args.kc, l.args.Cs, l.args.C, l.args.Lp, l.args.LPB, l.grid,
                 (long long)l.args.nlines);
        out += tmp;
    }
    out += " tuned=" + std::to_string(it.tuned);
    for (size_t b = 0; b < plan->steps.size(); ++b)
        for (const auto &m : plan->steps[b].members)
            if (m.first == i) {
                if (plan->steps[b].level)
                    out += " level=" + std::to_string(b) + "/" + std::to_string(plan->steps[b].count);
                else
                    out += " batch=" + std::to_string(b) + "/" + std::to_string(plan->steps[b].count) + "x" +
                           std::to_string(plan->steps[b].wavefronts) + "w";
            }
    return snprintf(buf, (size_t)len, "%s", out.c_str());
}

int tri_plan_launch_count(tri_plan plan)
{
    if (!plan) return -1;
    int n = 0;
    for (const auto &st : plan->steps) {
        if (!st.members.empty()) {
            ++n;
            continue;
        }
        const auto &item = plan->items[(size_t)st.item];
        n += item.launches[(size_t)st.launch].args.nlines > 0 ? 1 : 0;
    }
    return n;
}

}  // extern "C"

// ============================================================================
// Fractional-step time step (Sec. 2.2): three Runge-Kutta sub-steps, each the
// momentum right-hand side, ADI sweeps x -> y -> z of the three velocity
// components (one plan per sub-step), the velocity update, the 3-D projection
// and the pressure update.
// ============================================================================
struct tri_ns_s {
    tri_ctx ctx = nullptr;
    int64_t Nx = 0, Ny = 0, Nz = 0;
    double dx = 0.0, dz = 0.0, dt = 0.0, nu = 0.0;
    int P_poisson = 8;
    void *mem = nullptr;                  // metric, sweep coefficients and work fields, one allocation
    double *dy = nullptr, *ay = nullptr, *cy = nullptr, *lamz = nullptr, *lamx = nullptr;
    double *ycoef = nullptr;              // [Ny][NS_YCOEF] constants of the momentum right-hand side
    double *N[3] = {}, *D[3] = {};        // convection of the last sub-step; sweep right-hand sides
    double *phihat = nullptr, *phi = nullptr;
    tri_plan plans[3] = {};               // per sub-step: the x and y sweeps of du, dv, dw
    tri_plan zplans[3] = {};              // per sub-step: the z sweeps of du, dv, dw
    bool fused = false;                   // the z sweeps add their solutions to u, v, w ...
    Launch zacc[3][3];                    // ... with these launches [sub-step][component]
};

namespace {

constexpr double kRkGamma[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
constexpr double kRkZeta[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};

enum { kLapFaceX = 0, kLapCellSlipX = 1, kLapCellWallY = 2, kLapFaceY = 3, kLapPeriodic = 4 };

// Second difference along one sweep line, row t: lo_t q_{t-1} + diag_t q_t +
// up_t q_{t+1}.  kLapFaceX: u on x-faces 0..n-1 with walls at faces 0 and n
// (row 0 empty); kLapCellSlipX: cells with zero flux through both ends;
// kLapCellWallY: cells with the no-slip wall below cell 0 (mirror value -q at
// distance dy_0) and zero flux through the top; kLapFaceY: v on y-faces
// 0..n-1 with walls at faces 0 and n (row 0 empty); kLapPeriodic: uniform,
// periodic.
void ns_lap_rows(int kind, int64_t n, double h, const std::vector<double> &dy, std::vector<double> &lo,
                 std::vector<double> &diag, std::vector<double> &up)
{
    lo.assign((size_t)n, 0.0);
    diag.assign((size_t)n, 0.0);
    up.assign((size_t)n, 0.0);
    const double ih2 = 1.0 / (h * h);
    for (int64_t t = 0; t < n; ++t) {
        switch (kind) {
        case kLapFaceX:
            if (t >= 1) {
                lo[t] = ih2;
                up[t] = (t <= n - 2) ? ih2 : 0.0;
                diag[t] = -2.0 * ih2;
            }
            break;
        case kLapCellSlipX:
            lo[t] = (t >= 1) ? ih2 : 0.0;
            up[t] = (t <= n - 2) ? ih2 : 0.0;
            diag[t] = -(lo[t] + up[t]);
            break;
        case kLapCellWallY:
            lo[t] = (t >= 1) ? 1.0 / (dy[t] * (0.5 * (dy[t - 1] + dy[t]))) : 0.0;
            up[t] = (t <= n - 2) ? 1.0 / (dy[t] * (0.5 * (dy[t] + dy[t + 1]))) : 0.0;
            diag[t] = -(lo[t] + up[t]);
            if (t == 0) diag[t] -= 2.0 / (dy[0] * dy[0]);
            break;
        case kLapFaceY:
            if (t >= 1) {
                const double hj = 0.5 * (dy[t - 1] + dy[t]);
                lo[t] = 1.0 / (hj * dy[t - 1]);
                const double upf = 1.0 / (hj * dy[t]);
                diag[t] = -(lo[t] + upf);
                up[t] = (t <= n - 2) ? upf : 0.0;
            }
            break;
        default:
            lo[t] = up[t] = ih2;
            diag[t] = -2.0 * ih2;
        }
    }
}

void ns_release(tri_ns ns)
{
    for (tri_plan *set : {ns->plans, ns->zplans})
        for (int s = 0; s < 3; ++s)
            if (set[s]) {
                (void)tri_plan_destroy(set[s]);
                set[s] = nullptr;
            }
    if (ns->mem) (void)hipFree(ns->mem);
    delete ns;
}

}  // namespace

void tri::ns_ycoef_row(const double *dy, int64_t Ny, int64_t j, double *out)
{
    const double dyj = dy[j], dym = j > 0 ? dy[j - 1] : 0.0, dyp = j < Ny - 1 ? dy[j + 1] : 0.0;
    const bool ym = j >= 1, yp = j <= Ny - 2;
    const double hj = 0.5 * (dym + dyj);
    const double ifj = 1.0 / (dym + dyj), ifj1 = 1.0 / (dyj + dyp);
    out[0] = 1.0 / dyj;
    out[1] = 1.0 / hj;
    out[2] = dyj * ifj;
    out[3] = dym * ifj;
    out[4] = dyp * ifj1;
    out[5] = dyj * ifj1;
    const double ly_lo = ym ? 1.0 / (dyj * (0.5 * (dym + dyj))) : 0.0;
    const double ly_up = yp ? 1.0 / (dyj * (0.5 * (dyj + dyp))) : 0.0;
    out[6] = ly_lo;
    out[7] = -(ly_lo + ly_up) - (j == 0 ? 2.0 / (dyj * dyj) : 0.0);
    out[8] = ly_up;
    const double lv_lo = ym ? 1.0 / (hj * dym) : 0.0, lv_upf = ym ? 1.0 / (hj * dyj) : 0.0;
    out[9] = lv_lo;
    out[10] = -(lv_lo + lv_upf);
    out[11] = yp ? lv_upf : 0.0;
}

namespace {

// The accumulating form of a z sweep's launch: the strided kernel with one
// line per lane (the two-lines-per-lane kernel has no accumulating
// instance), the same partitions and factor tables.
// A strided launch as its accumulating form with one line per lane.
bool acc_one_line(Launch &l)
{
    SolveArgs &a = l.args;
    if (a.lpl == 2) {
        a.lpl = 1;
        a.kc = 1;
        a.Cs = a.m;
        a.ngroups0 = (a.nb0 + 63) / 64;
        l.chunk_max = pick_chunk(a.m);
    }
    return strided_acc_supported(TRI_PDD, l.chunk_max);
}

// The accumulating form of a z sweep's launch: two lines per lane where the
// plan chose that shape and the target's layout keeps line pairs 16-byte
// aligned (`pairs`), else one line per lane (which also serves at a step
// whose target array is not 16-byte aligned).
bool ns_acc_launch(const Launch &base, bool pairs, Launch &out)
{
    if (base.kind != 0 || base.refine) return false;
    Launch one = base;
    if (!acc_one_line(one)) return false;
    out = (pairs && base.args.lpl == 2 && strided2_acc_supported(TRI_PDD, base.chunk_max)) ? base : one;
    return true;
}

bool ns_overlap(const void *a, size_t na, const void *b, size_t nb)
{
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

}  // namespace

extern "C" {

tri_status ns_create(tri_ctx ctx, const tri_ns_config *cfg, tri_ns *out)
{
    if (!ctx || !out) return TRI_E_ARG;
    *out = nullptr;
    if (!cfg || !cfg->dy) return fail(ctx, TRI_E_ARG, "ns_create: null config or dy");
    const int64_t Nx = cfg->Nx, Ny = cfg->Ny, Nz = cfg->Nz;
    if (Nx < 2 || Ny < 2 || Nz < 2) return fail(ctx, TRI_E_SHAPE, "ns_create: grid %lld x %lld x %lld",
                                                 (long long)Nx, (long long)Ny, (long long)Nz);
    if (!(cfg->dx > 0.0) || !(cfg->dz > 0.0) || !(cfg->dt > 0.0) || !(cfg->nu >= 0.0))
        return fail(ctx, TRI_E_ARG, "ns_create: dx, dz, dt must be > 0 and nu >= 0");
    for (int64_t j = 0; j < Ny; ++j)
        if (!(cfg->dy[j] > 0.0) || !std::isfinite(cfg->dy[j]))
            return fail(ctx, TRI_E_ARG, "ns_create: dy[%lld] = %g", (long long)j, cfg->dy[j]);
    // the projection's requirements, checked here so that a step never fails on them
    FftShape S;
    if ((Nz & 1) || (Nx & 1)) return fail(ctx, TRI_E_SHAPE, "ns_create: Nx and Nz must be even");
    if (!fft_shape(Nz, S) || !dct_shape(Nx, S))
        return fail(ctx, TRI_E_UNSUPPORTED, "ns_create: Nz/2 or Nx is not 2^a 3^b 5^c within the transform limits");
    tri_status st = check_partition(ctx, Ny, cfg->P_poisson, 0);
    if (st) return st;
    const int mp = (int)(Ny / cfg->P_poisson);
    if (mp > kGeneralMaxM || (mp > 16 && cfg->P_poisson > 8))
        return fail(ctx, TRI_E_UNSUPPORTED, "ns_create: the shifted solves take at most 32 rows a partition");
    HIP_TRY(ctx, hipSetDevice(ctx->device));

    tri_ns ns = new (std::nothrow) tri_ns_s;
    if (!ns) return TRI_E_NOMEM;
    ns->ctx = ctx;
    ns->Nx = Nx;
    ns->Ny = Ny;
    ns->Nz = Nz;
    ns->dx = cfg->dx;
    ns->dz = cfg->dz;
    ns->dt = cfg->dt;
    ns->nu = cfg->nu;
    ns->P_poisson = cfg->P_poisson;
    const int64_t cells = Nx * Ny * Nz, Nk = Nz / 2 + 1;
    const int64_t nmax = std::max(Nx, std::max(Ny, Nz));
    // layout (doubles): dy ay cy [Ny each], lamz [Nk], lamx [Nx], coefficients
    // [3 sub-steps][9 sweeps][3][nmax], ycoef [Ny][NS_YCOEF], then 16-byte
    // aligned: N[3], D[3], phi [cells each], phihat [2 Nk Ny Nx]
    const int64_t head = 3 * Ny + Nk + Nx + 3 * 9 * 3 * nmax + NS_YCOEF * Ny;
    const int64_t head_al = (head + 31) / 32 * 32;
    const size_t bytes = sizeof(double) * (size_t)(head_al + 7 * cells + 2 * Nk * Ny * Nx);
    if (hipMalloc(&ns->mem, bytes) != hipSuccess) {
        ns->mem = nullptr;
        ns_release(ns);
        return fail(ctx, TRI_E_NOMEM, "ns_create: %zu bytes", bytes);
    }
    double *base = (double *)ns->mem;
    ns->dy = base;
    ns->ay = base + Ny;
    ns->cy = base + 2 * Ny;
    ns->lamz = base + 3 * Ny;
    ns->lamx = ns->lamz + Nk;
    double *coef = ns->lamx + Nx;
    ns->ycoef = coef + 3 * 9 * 3 * nmax;
    double *fields = base + head_al;
    for (int c = 0; c < 3; ++c) {
        ns->N[c] = fields + (int64_t)c * cells;
        ns->D[c] = fields + (int64_t)(3 + c) * cells;
    }
    ns->phi = fields + 6 * cells;
    ns->phihat = fields + 7 * cells;

    // metric of the projection (cell-centred Neumann second difference in y,
    // modified wavenumbers of the z Fourier and x cosine transforms)
    std::vector<double> dy(cfg->dy, cfg->dy + Ny), host((size_t)head, 0.0);
    for (int64_t j = 0; j < Ny; ++j) {
        host[(size_t)j] = dy[(size_t)j];
        if (j >= 1) host[(size_t)(Ny + j)] = 1.0 / (dy[(size_t)j] * (0.5 * (dy[(size_t)(j - 1)] + dy[(size_t)j])));
        if (j <= Ny - 2) host[(size_t)(2 * Ny + j)] = 1.0 / (dy[(size_t)j] * (0.5 * (dy[(size_t)j] + dy[(size_t)(j + 1)])));
    }
    const double pi = 3.14159265358979323846;
    for (int64_t k = 0; k < Nk; ++k) {
        const double s = std::sin(pi * (double)k / (double)Nz);
        host[(size_t)(3 * Ny + k)] = (4.0 / (cfg->dz * cfg->dz)) * s * s;
    }
    for (int64_t i = 0; i < Nx; ++i) {
        const double s = std::sin(pi * (double)i / (2.0 * (double)Nx));
        host[(size_t)(3 * Ny + Nk + i)] = (4.0 / (cfg->dx * cfg->dx)) * s * s;
    }
    // sweep coefficients (1 - beta L_d), beta = alpha_s dt nu / 2; sweeps in the
    // order du x, y, z; dv x, y, z; dw x, y, z
    static const int kind[9] = {kLapFaceX, kLapCellWallY, kLapPeriodic, kLapCellSlipX, kLapFaceY, kLapPeriodic,
                                kLapCellSlipX, kLapCellWallY, kLapPeriodic};
    std::vector<double> lo, diag, up;
    const int64_t coef_off = 3 * Ny + Nk + Nx;
    for (int s = 0; s < 3; ++s) {
        const double beta = (kRkGamma[s] + kRkZeta[s]) * cfg->dt * cfg->nu / 2.0;
        for (int q = 0; q < 9; ++q) {
            const int dir = q % 3;
            const int64_t n = dir == 0 ? Nx : (dir == 1 ? Ny : Nz);
            ns_lap_rows(kind[q], n, dir == 0 ? cfg->dx : cfg->dz, dy, lo, diag, up);
            double *row = host.data() + coef_off + ((int64_t)(s * 9 + q) * 3) * nmax;
            for (int64_t t = 0; t < n; ++t) {
                row[t] = -beta * lo[(size_t)t];
                row[nmax + t] = 1.0 - beta * diag[(size_t)t];
                row[2 * nmax + t] = -beta * up[(size_t)t];
            }
        }
    }
    for (int64_t j = 0; j < Ny; ++j)
        ns_ycoef_row(dy.data(), Ny, j, host.data() + coef_off + 3 * 9 * 3 * nmax + NS_YCOEF * j);
    if (hipMemcpy(base, host.data(), sizeof(double) * host.size(), hipMemcpyHostToDevice) != hipSuccess) {
        ns_release(ns);
        return fail(ctx, TRI_E_HIP, "ns_create: upload");
    }
    // two plans per sub-step: the x and y sweeps of the three fields (two
    // dependency levels), then their z sweeps.  Where every z sweep runs a
    // strided kernel with an accumulating instance (one line per lane), the
    // step launches those with u, v, w as targets, so that the velocity
    // update u += du is the z sweep's store.  TRI_NS_FUSE=0 keeps the separate update kernel; =1
    // makes ns_create fail with TRI_E_UNSUPPORTED where the z sweeps cannot
    // add into the velocity.
    ns->fused = true;
    for (int s = 0; s < 3; ++s) {
        tri_item xy[6], z[3];
        for (int q = 0; q < 9; ++q) {
            const int dir = q % 3, c = q / 3;
            const double *row = coef + ((int64_t)(s * 9 + q) * 3) * nmax;
            const tri_item it{dir, ns->D[c], Nx, Ny, Nz, row, row + nmax, row + 2 * nmax, nullptr,
                              cfg->P_adi[dir], dir == 2 ? 1 : 0, TRI_PDD};
            if (dir == 2) z[c] = it;
            else xy[2 * c + dir] = it;
        }
        // (per-kernel-instance batches: the three x sweeps keep the register-factor
        // kernel with 8 rows per lane, which a level launch cannot hold, and the
        // three y sweeps share one batched launch anyway)
        const int mode = std::min(batch_mode(), 1);
        st = plan_create(ctx, xy, 6, TRI_F64, mode, &ns->plans[s]);
        if (!st) st = plan_create(ctx, z, 3, TRI_F64, mode, &ns->zplans[s]);
        if (st) {
            const std::string why = ctx->last_error;
            ns_release(ns);
            return fail(ctx, st, "ns_create: sweep plan: %s", why.c_str());
        }
        for (int c = 0; c < 3; ++c) {
            const auto &item = ns->zplans[s]->items[(size_t)c];
            // line pairs of v (a_j = (Ny+1) Nx, a_b1 = Nx) and w stay aligned (Nx is
            // even); those of u (a_b1 = Nx + 1) do not
            if (item.launches.size() != 1 || !ns_acc_launch(item.launches[0], c > 0, ns->zacc[s][c]))
                ns->fused = false;
        }
    }
    const char *e = getenv("TRI_NS_FUSE");
    if (e && atoi(e) == 0) ns->fused = false;
    if (e && atoi(e) == 1 && !ns->fused) {
        ns_release(ns);
        return fail(ctx, TRI_E_UNSUPPORTED, "ns_create: a z sweep has no accumulating kernel instance");
    }
    *out = ns;
    return TRI_OK;
}

tri_status ns_step(tri_ns ns, double *u, double *v, double *w, double *p)
{
    if (!ns) return TRI_E_ARG;
    tri_ctx ctx = ns->ctx;
    const int64_t Nx = ns->Nx, Ny = ns->Ny, Nz = ns->Nz, cells = Nx * Ny * Nz;
    if (!u || !v || !w || !p) return fail(ctx, TRI_E_ARG, "ns_step: null field");
    if (misaligned(u) || misaligned(v) || misaligned(w) || misaligned(p))
        return fail(ctx, TRI_E_ARG, "ns_step: misaligned field");
    const size_t bu = sizeof(double) * (size_t)(Nz * Ny * (Nx + 1)), bv = sizeof(double) * (size_t)(Nz * (Ny + 1) * Nx);
    const size_t bc = sizeof(double) * (size_t)cells;
    if (ns_overlap(u, bu, v, bv) || ns_overlap(u, bu, w, bc) || ns_overlap(u, bu, p, bc) ||
        ns_overlap(v, bv, w, bc) || ns_overlap(v, bv, p, bc) || ns_overlap(w, bc, p, bc))
        return fail(ctx, TRI_E_ARG, "ns_step: u, v, w and p must not overlap");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    for (int s = 0; s < 3; ++s) {
        NsRhsArgs A;
        A.u = u;
        A.v = v;
        A.w = w;
        A.p = p;
        A.ycoef = ns->ycoef;
        A.Nx = Nx;
        A.Ny = Ny;
        A.Nz = Nz;
        A.idx = 1.0 / ns->dx;
        A.idz = 1.0 / ns->dz;
        A.idx2 = 1.0 / (ns->dx * ns->dx);
        A.idz2 = 1.0 / (ns->dz * ns->dz);
        A.dt = ns->dt;
        A.nu = ns->nu;
        A.gamma = kRkGamma[s];
        A.zeta = kRkZeta[s];
        A.alpha = kRkGamma[s] + kRkZeta[s];
        A.Nu = ns->N[0];
        A.Nv = ns->N[1];
        A.Nw = ns->N[2];
        A.du = ns->D[0];
        A.dv = ns->D[1];
        A.dw = ns->D[2];
        HIP_TRY(ctx, launch_ns_rhs(A, ctx->stream));
        tri_status st = tri_plan_execute(ns->plans[s]);
        if (st) return st;
        if (ns->fused) {
            // z sweeps of du, dv, dw adding into u (faces 0..Nx-1 of each row),
            // v (faces 0..Ny-1 of each plane) and w
            double *tgt[3] = {u, v, w};
            const int64_t aj[3] = {Ny * (Nx + 1), (Ny + 1) * Nx, Ny * Nx}, ab1[3] = {Nx + 1, Nx, Nx};
            for (int c = 0; c < 3; ++c) {
                Launch l = ns->zacc[s][c];
                // two lines per lane add 16-byte pairs: the target and its strides must keep them aligned
                if (l.args.lpl == 2 && ((uintptr_t)tgt[c] % 16 != 0 || aj[c] % 2 != 0 || ab1[c] % 2 != 0))
                    (void)acc_one_line(l);
                l.args.acc = tgt[c];
                l.args.a_j = aj[c];
                l.args.a_b0 = 1;
                l.args.a_b1 = ab1[c];
                HIP_TRY(ctx, run_launch(l, TRI_PDD, ctx->stream));
            }
        } else {
            st = tri_plan_execute(ns->zplans[s]);
            if (st) return st;
            HIP_TRY(ctx, launch_ns_update(u, v, w, ns->D[0], ns->D[1], ns->D[2], Nx, Ny, Nz, ctx->stream));
        }
        // the projection, whose last kernel also makes the pressure update
        // p += phi / (alpha dt)
        st = projection3d_step_p(ctx, u, v, w, ns->dx, ns->dy, ns->dz, ns->ay, ns->cy, ns->lamz, ns->lamx,
                                 ns->phihat, ns->phi, Nx, Ny, Nz, ns->P_poisson, p, 1.0 / (A.alpha * ns->dt));
        if (st) return st;
    }
    return TRI_OK;
}

tri_status ns_destroy(tri_ns ns)
{
    if (!ns) return TRI_E_ARG;
    (void)hipSetDevice(ns->ctx->device);
    (void)hipStreamSynchronize(ns->ctx->stream);
    ns_release(ns);
    return TRI_OK;
}

}  // extern "C"
