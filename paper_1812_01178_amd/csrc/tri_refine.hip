// tri_refine.hip -- FP32 elimination with FP64 residual refinement.
//
// Mixed-precision variant of the partitioned solve (not in the paper): the
// local eliminations of Eqs. (5)-(6) run in FP32 with FP32 copies of the
// factors, the reduced system (Eq. (7) / (10)) and the correction stay in
// FP64, and every sweep forms the true residual r = d - A x in FP64 from the
// original matrix rows, so the iteration converges to the exact A^{-1} d
// (the inner solver is an approximate inverse; PDD as inner solver also
// converges to A^{-1} d when its dropped entries are small).
//
//     x_0 = 0,  r_0 = d
//     repeat: delta = S32(r);  x += delta;  r = d - A x      (FP64)
//     until, on every line of the workgroup, the error estimate of a
//     linearly contracting iteration |delta_s|^2 / |delta_{s-1}| (max norms)
//     is <= tol * |x|; the plain test |delta_s| <= tol |x| would stall at
//     the FP64 noise floor of the residual on ill-conditioned lines.
//
// The FP32 solve is linear, so each line's right-hand side is scaled by a
// power of two before rounding to FP32 (exact) and the update scaled back:
// by max|d| of the line for the first solve, by the line's last max|update|
// afterwards (the next residual is A times an error of about that size).
// Lines of any magnitude stay inside FP32's range.
//
// Layout and chunking as k_strided: workgroup = P*kc wavefronts, wavefront
// (r, s) holds rows [r*m + s*Cs, +Cs) of 64 neighbouring lines; d and x stay
// in FP64 VGPRs for the whole iteration, the work vector in FP32.  Chunk
// boundary values of x (residual) and FP32 carries (elimination) go through
// LDS.  HBM traffic equals the FP64 path: read d once, write x once.
#include <hip/hip_runtime.h>

#include "tri_device.h"

namespace tri {

// max of non-negative values that keeps a NaN once one appears (fmax would
// drop it and let a failed solve look converged)
__device__ __forceinline__ double nanmax(double acc, double v) { return (v > acc || v != v) ? v : acc; }

// Binary exponent used to scale a line whose largest magnitude is v (0 for
// zero or non-finite v; clamped so that 2^(+-E) stays finite).
__device__ __forceinline__ int line_exponent(double v)
{
    if (!(v > 0.0) || !(v <= 1.7976931348623157e308)) return 0;
    return min(1000, max(-1000, ilogb(v)));
}

// EXACT: the chunk has exactly CMAX rows (no row guards).
template <int CMAX, int METHOD, bool EXACT = false>
__device__ __forceinline__ void strided_refine_solve(const SolveArgs &A, const RefineArgs &R, int64_t blk,
                                                     double *lds)
{
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int kc = A.kc, Cs = EXACT ? CMAX : A.Cs;
    const int r = w / kc, s = w - r * kc;
    const int P = A.P, m = A.m;
    const int nw = P * kc;
    double *tips = lds;                               // [2P][64]
    double *xb = tips + 2 * P * 64;                   // [nw][2][64] chunk-boundary x
    double *nrm = xb + nw * 2 * 64;                   // [nw][2][64] max|delta|, max|x|
    float *fend = (float *)(nrm + nw * 2 * 64);       // [nw][64]
    float *bbeg = fend + nw * 64;                     // [nw][64]
    float *pif = bbeg + nw * 64;                      // [nw]
    float *pib = pif + nw;                            // [nw]
    int *flag = (int *)(pib + nw);
    int *escale = flag + 4;                           // [64] per-line scale exponent
    double *ofac = (double *)(escale + 64);           // [nw][3][CMAX] true rows a, b, c
    float *ffac = (float *)(ofac + nw * 3 * CMAX);    // [nw][5][CMAX] FP32 factors

    const int64_t grp = blk % A.ngroups0;
    const int64_t b1 = blk / A.ngroups0;
    const int64_t b0 = grp * 64 + lane;
    const bool active = b0 < A.nb0;
    const int64_t n = A.n;
    const int64_t g = b1 * A.g_b1 + A.g_off;
    const int64_t row0 = (int64_t)r * m + (int64_t)s * Cs;
    // this chunk's factors and matrix rows, staged once in LDS (read back with
    // wavefront-uniform addresses inside the sweeps)
    {
        const gfloat *__restrict__ F0 = (const gfloat *)(R.F32 + g * (kNumFactors * n) + row0);
        const gdouble *__restrict__ O0 = (const gdouble *)(R.ORIG + g * (3 * n) + row0);
        for (int idx = lane; idx < kNumFactors * Cs; idx += 64) {
            const int f = idx / Cs, t = idx - f * Cs;
            ffac[(w * kNumFactors + f) * CMAX + t] = F0[f * n + t];
        }
        for (int idx = lane; idx < 3 * Cs; idx += 64) {
            const int f = idx / Cs, t = idx - f * Cs;
            ofac[(w * 3 + f) * CMAX + t] = O0[f * n + t];
        }
    }
    const double *Oa = ofac + (w * 3 + 0) * CMAX;
    const double *Oe = ofac + (w * 3 + 1) * CMAX;   // row sums a + b + c
    const double *Oc = ofac + (w * 3 + 2) * CMAX;
    const float *Fb = ffac + (w * kNumFactors + 0) * CMAX;
    const float *Fa = ffac + (w * kNumFactors + 1) * CMAX;
    const float *Fc = ffac + (w * kNumFactors + 2) * CMAX;
    const float *Fv = ffac + (w * kNumFactors + 3) * CMAX;
    const float *Fw = ffac + (w * kNumFactors + 4) * CMAX;
    __syncthreads();
    const int64_t sj = A.s_j;
    gdouble *__restrict__ p = (gdouble *)(A.d + (active ? b0 : 0) * A.s_b0 + b1 * A.s_b1 + row0 * sj);
    // neighbouring chunks in line order (wavefronts are numbered along the line)
    const int wprev = (w > 0) ? w - 1 : (A.periodic ? nw - 1 : -1);
    const int wnext = (w < nw - 1) ? w + 1 : (A.periodic ? 0 : -1);

    double dv[CMAX], xv[CMAX];
    float e[CMAX];
#pragma unroll
    for (int t = 0; t < CMAX; ++t) {
        dv[t] = 0.0;
        xv[t] = 0.0;
        e[t] = 0.0f;
    }
    if (active) {
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < Cs) dv[t] = __builtin_nontemporal_load(p + t * sj);
    }
    if (r == 0 && s == 0 && (((const gint *)A.flags)[g] & 1)) dv[0] = 0.0;   // gauge-pinned row
    // scale of the first right-hand side: the exponent of max|d| over the line
    int E;
    {
        double dm = 0.0;
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < Cs) dm = nanmax(dm, fabs(dv[t]));
        nrm[(w * 2 + 0) * 64 + lane] = dm;
        __syncthreads();
        double D0 = 0.0;
        for (int q = 0; q < nw; ++q) D0 = nanmax(D0, nrm[(q * 2 + 0) * 64 + lane]);
        E = line_exponent(D0);
    }

    const gdouble *__restrict__ it = (const gdouble *)(A.IT + ((g * P + r) * 2) * (2 * P));
    int sweep = 0;
    bool converged = false;
    double dprev = 0.0, est = 0.0;   // wavefront 0: previous update norm and error estimate of its lane's line
    for (; sweep <= R.max_sweeps; ++sweep) {
        // ---- residual r = d - A x in FP64 (true matrix rows) -------------
        const double sc = ldexp(1.0, -E);
        if (sweep == 0) {
#pragma unroll
            for (int t = 0; t < CMAX; ++t) e[t] = (float)(dv[t] * sc);
        } else {
            double xlast = 0.0;
#pragma unroll
            for (int t = 0; t < CMAX; ++t)
                if (t == Cs - 1) xlast = xv[t];
            xb[(w * 2 + 0) * 64 + lane] = xv[0];
            xb[(w * 2 + 1) * 64 + lane] = xlast;
            __syncthreads();
            double xm = (wprev >= 0) ? xb[(wprev * 2 + 1) * 64 + lane] : 0.0;
            const double xr = (wnext >= 0) ? xb[(wnext * 2 + 0) * 64 + lane] : 0.0;
#pragma unroll
            for (int t = 0; t < CMAX; ++t)
                if (t < Cs) {
                    const double xp = (t + 1 < Cs) ? xv[(t + 1 < CMAX) ? t + 1 : t] : xr;
                    // d - (a x_{t-1} + b x_t + c x_{t+1}), written without the
                    // cancellation of b x_t against a x_t + c x_t
                    const double res = dv[t] - (Oa[t] * (xm - xv[t]) + Oc[t] * (xp - xv[t]) + Oe[t] * xv[t]);
                    xm = xv[t];
                    e[t] = (float)(res * sc);
                }
        }
        // ---- FP32 partitioned elimination of A~ delta~ = r ----------------
        float tip_last;
        if (kc == 1) {
            float gp = 0.0f;
#pragma unroll
            for (int t = 0; t < CMAX; ++t)
                if (t < Cs) {
                    gp = Fb[t] * e[t] - Fa[t] * gp;
                    e[t] = gp;
                }
            tip_last = gp;
            float xn = 0.0f;
#pragma unroll
            for (int t = CMAX - 1; t >= 0; --t)
                if (t < Cs) {
                    xn = e[t] - Fc[t] * xn;
                    e[t] = xn;
                }
        } else {
            float gp = 0.0f, pf = 1.0f;
#pragma unroll
            for (int t = 0; t < CMAX; ++t)
                if (t < Cs) {
                    gp = Fb[t] * e[t] - Fa[t] * gp;
                    pf *= -Fa[t];
                }
            fend[w * 64 + lane] = gp;
            if (lane == 0) pif[w] = pf;
            __syncthreads();
            float gin = 0.0f;
            for (int s2 = 0; s2 < s; ++s2) gin = fend[(r * kc + s2) * 64 + lane] + pif[r * kc + s2] * gin;
            gp = gin;
#pragma unroll
            for (int t = 0; t < CMAX; ++t)
                if (t < Cs) {
                    gp = Fb[t] * e[t] - Fa[t] * gp;
                    e[t] = gp;
                }
            tip_last = gp;
            float xn = 0.0f, pb = 1.0f;
#pragma unroll
            for (int t = CMAX - 1; t >= 0; --t)
                if (t < Cs) {
                    xn = e[t] - Fc[t] * xn;
                    pb *= -Fc[t];
                }
            bbeg[w * 64 + lane] = xn;
            if (lane == 0) pib[w] = pb;
            __syncthreads();
            float xin = 0.0f;
            for (int s2 = kc - 1; s2 > s; --s2) xin = bbeg[(r * kc + s2) * 64 + lane] + pib[r * kc + s2] * xin;
            xn = xin;
#pragma unroll
            for (int t = CMAX - 1; t >= 0; --t)
                if (t < Cs) {
                    xn = e[t] - Fc[t] * xn;
                    e[t] = xn;
                }
        }
        // ---- reduced system and correction in FP64 ----------------------
        if (s == 0) tips[(2 * r) * 64 + lane] = (double)e[0];
        if (s == kc - 1) tips[(2 * r + 1) * 64 + lane] = (double)tip_last;
        __syncthreads();
        double yl, yr;
        interface_unknowns<METHOD>(it, r, P, A.periodic, [&](int q) { return tips[q * 64 + lane]; }, yl, yr);
        double dmax = 0.0, xmax = 0.0;
        bool nan = false;                       // (fmax drops NaNs: they are counted apart)
        const double unscale = ldexp(1.0, E);
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < Cs) {
                const double delta = ((double)e[t] - yl * (double)Fv[t] - yr * (double)Fw[t]) * unscale;
                xv[t] += delta;
                nan |= !(delta == delta) || !(xv[t] == xv[t]);
                dmax = fmax(dmax, fabs(delta));
                xmax = fmax(xmax, fabs(xv[t]));
            }
        if (nan) dmax = xmax = __builtin_nan("");
        // ---- convergence of every line of the workgroup ------------------
        nrm[(w * 2 + 0) * 64 + lane] = dmax;
        nrm[(w * 2 + 1) * 64 + lane] = xmax;
        __syncthreads();
        if (w == 0) {
            double D = 0.0, X = 0.0;
            for (int q = 0; q < nw; ++q) {
                D = nanmax(D, nrm[(q * 2 + 0) * 64 + lane]);
                X = nanmax(X, nrm[(q * 2 + 1) * 64 + lane]);
            }
            // error left after this update if the iteration contracts linearly
            const double Xs = X > 0.0 ? X : 1.0;
            const double rate = (dprev > 0.0) ? fmin(1.0, D / dprev) : (D > 0.0 ? 1.0 : 0.0);
            est = (sweep == 0) ? 1.0 : (D / Xs) * rate;
            // the contraction rate is measured between two refinement updates, so
            // a line is accepted after two refinements (or when an update alone
            // is already below the tolerance); on well-conditioned matrices the
            // first update's relative size, times the condition bound, bounds the
            // rate, and one refinement may do
            const double rel = D / Xs;
            const bool ok = !active || (sweep >= 1 && D <= R.tol * Xs) || (sweep >= 2 && est <= R.tol) ||
                            (sweep == 1 && R.kappa > 0.0 && R.kappa * rel * rel <= R.tol);
            dprev = D;
            escale[lane] = line_exponent(D);
            const bool all = __all(ok);
            if (lane == 0) *flag = all ? 1 : 0;
        }
        __syncthreads();
        converged = (*flag != 0);
        E = escale[lane];
        if (converged) break;
    }
    if (threadIdx.x == 0) {
        if (!converged) atomicOr(R.status, kStatusNotConverged);
        if (R.sweeps_used) atomicMax(R.sweeps_used, converged ? sweep : R.max_sweeps);
    }
    if (w == 0 && R.resid_bits) {
        // largest estimated remaining relative error of the workgroup's lines
        // (non-negative doubles order like their bit patterns), one atomic
        double e = active ? fabs(est) : 0.0;
        for (int off = 32; off > 0; off >>= 1) e = nanmax(e, __shfl_xor(e, off));
        if (lane == 0) atomicMax(R.resid_bits, (unsigned long long)__double_as_longlong(e));
    }
    if (active) {
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < Cs) __builtin_nontemporal_store(xv[t], p + t * sj);
    }
}

template <int CMAX, int METHOD, bool EXACT>
__global__ void __launch_bounds__(CMAX > 16 ? 512 : 1024) k_strided_refine(const SolveArgs A, const RefineArgs R)
{
    extern __shared__ double lds[];
    strided_refine_solve<CMAX, METHOD, EXACT>(A, R, blockIdx.x, lds);
}

// Ragged batch of refinement solves in one launch (see k_strided_batch):
// every entry runs with this instance's CMAX, method and P * kc.
template <int CMAX, int METHOD, bool EXACT>
__global__ void __launch_bounds__(CMAX > 16 ? 512 : 1024) k_strided_refine_batch(const BatchEntry *__restrict__ E,
                                                                                  int count)
{
    extern __shared__ double lds[];
    const int64_t b = blockIdx.x;
    int i = 0;
    while (i + 1 < count && E[i + 1].begin <= b) ++i;
    strided_refine_solve<CMAX, METHOD, EXACT>(E[i].a, E[i].R, b - E[i].begin, lds);
}

template <int CMAX, int METHOD>
static void launch_refine_batch_t(const BatchEntry *e, int count, dim3 grid, dim3 block, size_t lds, bool exact,
                                  hipStream_t s)
{
    if (exact) hipLaunchKernelGGL((k_strided_refine_batch<CMAX, METHOD, true>), grid, block, lds, s, e, count);
    else hipLaunchKernelGGL((k_strided_refine_batch<CMAX, METHOD, false>), grid, block, lds, s, e, count);
}

template <int METHOD>
static hipError_t launch_refine_batch_m(const BatchEntry *e, int count, dim3 grid, dim3 block, size_t lds,
                                        int cmax, bool exact, hipStream_t s)
{
    switch (cmax) {
    case 8: launch_refine_batch_t<8, METHOD>(e, count, grid, block, lds, exact, s); break;
    case 16: launch_refine_batch_t<16, METHOD>(e, count, grid, block, lds, exact, s); break;
    case 24: launch_refine_batch_t<24, METHOD>(e, count, grid, block, lds, exact, s); break;
    case 32: launch_refine_batch_t<32, METHOD>(e, count, grid, block, lds, exact, s); break;
    case 36: launch_refine_batch_t<36, METHOD>(e, count, grid, block, lds, exact, s); break;
    case 40: launch_refine_batch_t<40, METHOD>(e, count, grid, block, lds, exact, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_strided_refine_batch(const BatchEntry *entries, int count, int64_t blocks, int wavefronts,
                                       int cmax, int method, bool exact, size_t lds, hipStream_t s)
{
    if (blocks <= 0) return hipSuccess;
    const dim3 grid((unsigned)blocks), block(64 * wavefronts);
    return method == TRI_PDD ? launch_refine_batch_m<TRI_PDD>(entries, count, grid, block, lds, cmax, exact, s)
                             : launch_refine_batch_m<TRI_PPT>(entries, count, grid, block, lds, cmax, exact, s);
}

size_t strided_refine_lds_bytes(const SolveArgs &a)
{
    const int nw = a.P * a.kc;
    const int cmax = a.Cs <= 8 ? 8 : (a.Cs <= 16 ? 16 : (a.Cs <= 24 ? 24 : (a.Cs <= 32 ? 32 : (a.Cs == 36 ? 36 : 40))));
    return sizeof(double) * ((size_t)2 * a.P * 64 + (size_t)nw * 4 * 64) +
           sizeof(float) * ((size_t)nw * 2 * 64 + 2 * (size_t)nw) + 16 + 64 * sizeof(int) +
           sizeof(double) * (size_t)nw * 3 * cmax + sizeof(float) * (size_t)nw * kNumFactors * cmax;
}

template <int CMAX, int METHOD>
static hipError_t launch_refine_t(const SolveArgs &a, const RefineArgs &R, hipStream_t s)
{
    const int64_t blocks = a.ngroups0 * a.nb1;
    if (a.Cs == CMAX)
        hipLaunchKernelGGL((k_strided_refine<CMAX, METHOD, true>), dim3((unsigned)blocks), dim3(64 * a.P * a.kc),
                           strided_refine_lds_bytes(a), s, a, R);
    else
        hipLaunchKernelGGL((k_strided_refine<CMAX, METHOD, false>), dim3((unsigned)blocks), dim3(64 * a.P * a.kc),
                           strided_refine_lds_bytes(a), s, a, R);
    return hipGetLastError();
}

template <int METHOD>
static hipError_t launch_refine_m(const SolveArgs &a, const RefineArgs &R, int cmax, hipStream_t s)
{
    switch (cmax) {
    case 8: return launch_refine_t<8, METHOD>(a, R, s);
    case 16: return launch_refine_t<16, METHOD>(a, R, s);
    case 24: return launch_refine_t<24, METHOD>(a, R, s);
    case 32: return launch_refine_t<32, METHOD>(a, R, s);
    case 36: return launch_refine_t<36, METHOD>(a, R, s);
    case 40: return launch_refine_t<40, METHOD>(a, R, s);
    default: return hipErrorInvalidValue;
    }
}

__global__ void k_reset_counters(int *sweeps, unsigned long long *resid)
{
    if (threadIdx.x == 0) {
        *sweeps = 0;
        *resid = 0ull;
    }
}

hipError_t launch_reset_counters(int *sweeps, unsigned long long *resid, hipStream_t s)
{
    hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(64), 0, s, sweeps, resid);
    return hipGetLastError();
}

hipError_t launch_strided_refine(const SolveArgs &a, const RefineArgs &R, int method, int chunk_max, hipStream_t s)
{
    return method == TRI_PDD ? launch_refine_m<TRI_PDD>(a, R, chunk_max, s)
                             : launch_refine_m<TRI_PPT>(a, R, chunk_max, s);
}

}  // namespace tri
