// tri_general_refine.hip -- FP32 elimination with FP64 residual refinement
// for lines with their own coefficients (a, b, c per line).
//
// The iteration is the one of the other refinement kernels (not in the
// paper; the partitioned solve of Sec. 3.2 is the inner solver):
//
//     x_0 = 0,  r_0 = d
//     repeat: delta = S32(r);  x += delta;  r = d - A x      (FP64)
//
// Layout of the FP64 general kernel: workgroup = P wavefronts, wavefront r =
// partition r, lane = line.  Each lane factors its own block A~_r once, in
// FP32 (pivots, multipliers, the forward-reduced a-corner spike), and keeps
// the factors in VGPRs; every sweep forms the residual of the whole line in
// FP64 from the original coefficients (neighbouring partitions' end values
// through LDS), solves the local blocks in FP32, and the reduced system
// (PDD: one 2x2 per interface; PPT: Zbar of Eq. (10) with partial pivoting)
// and the correction in FP64.  Right-hand sides are scaled per line by a
// power of two before rounding to FP32; the stopping rule is that of the
// other refinement kernels, voted per workgroup over its lines.
#include <hip/hip_runtime.h>

#include "tri_device.h"

namespace tri {

namespace {

__device__ __forceinline__ double gmax(double acc, double v) { return (v > acc || v != v) ? v : acc; }

__device__ __forceinline__ int gexponent(double v)
{
    if (!(v > 0.0) || !(v <= 1.7976931348623157e308)) return 0;
    return min(1000, max(-1000, ilogb(v)));
}

}  // namespace

template <int CMAX, int METHOD>
__global__ void __launch_bounds__(512) k_general_refine(const GeneralArgs A, const RefineArgs R)
{
    extern __shared__ double sh[];              // [10][P][64] doubles, then 65 ints
    const int lane = threadIdx.x & 63;
    const int r = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int64_t blk = blockIdx.x;
    const int64_t grp = blk % A.ngroups0;
    const int64_t b1 = blk / A.ngroups0;
    const int64_t b0raw = grp * 64 + lane;
    const bool active = b0raw < A.nb0;
    const int64_t b0 = active ? b0raw : 0;
    const int m = A.m, P = A.P, periodic = A.periodic;
    const int64_t sj = A.s_j, csj = A.cs_j;
    double *__restrict__ p = A.d + b0 * A.s_b0 + b1 * A.s_b1 + (int64_t)r * m * sj;
    const int64_t cb = (b0 >> A.cplx) * A.cs_b0 + b1 * A.cs_b1 + (int64_t)r * m * csj;
    const double *__restrict__ ca = A.a + cb;
    const double *__restrict__ cbp = A.b + cb;
    const double *__restrict__ cc = A.c + cb;
    auto S = [&](int q, int part) -> double & { return sh[((int64_t)q * P + part) * 64 + lane]; };
    int *flag = (int *)(sh + (int64_t)10 * P * 64);
    int *escale = flag + 1;                     // [64]

    // couplings of this partition's end rows to the neighbouring partitions
    // (the corners removed from A~_r); zero at the ends of a non-periodic line
    const bool has_l = (r > 0) || periodic, has_r = (r < P - 1) || periodic;
    const double a_first = has_l ? ca[0] : 0.0;
    const double c_last = has_r ? cc[(int64_t)(m - 1) * csj] : 0.0;
    const int Lp = (r > 0) ? r - 1 : P - 1, Rp = (r < P - 1) ? r + 1 : 0;

    double dv[CMAX], xv[CMAX];
    float fa[CMAX], fbeta[CMAX], fcp[CMAX], fgv[CMAX], e[CMAX];
#pragma unroll
    for (int t = 0; t < CMAX; ++t) {
        dv[t] = 0.0;
        xv[t] = 0.0;
    }
    if (active) {
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < m) dv[t] = p[t * sj];
    }
    // FP32 factors of A~_r and the forward-reduced a-corner spike
    // (an FP32 pivot that vanishes or overflows shows as non-convergence;
    // zero pivots of the FP64 matrix are the FP64 path's to report)
    float cpp = 0.0f, gvp = 0.0f, beta_last = 0.0f;
#pragma unroll
    for (int t = 0; t < CMAX; ++t) {
        fa[t] = 0.0f;
        fbeta[t] = 0.0f;
        fcp[t] = 0.0f;
        fgv[t] = 0.0f;
        if (t < m) {
            const float aa = (t == 0) ? 0.0f : (float)ca[t * csj];
            const float ccv = (t == m - 1) ? 0.0f : (float)cc[t * csj];
            const float den = (float)cbp[t * csj] - aa * cpp;
            const float beta = 1.0f / den;
            fa[t] = aa;
            fbeta[t] = beta;
            gvp = (t == 0) ? (float)a_first * beta : -(aa * beta) * gvp;
            fgv[t] = gvp;
            cpp = ccv * beta;
            fcp[t] = cpp;
            beta_last = beta;
        }
    }
    // spike tips of A~_r^{-1} (v: a-corner, w: c-corner), FP64 from the FP32 factors
    double vn = 0.0, cprod = 1.0;
#pragma unroll
    for (int t = CMAX - 1; t >= 0; --t)
        if (t < m) {
            vn = (double)fgv[t] - (double)fcp[t] * vn;
            if (t < m - 1) cprod *= -(double)fcp[t];
        }
    const double v0 = vn, vm = (double)gvp;
    const double wm = (double)beta_last * c_last, w0 = wm * cprod;
    S(2, r) = v0;
    S(3, r) = vm;
    S(4, r) = w0;
    S(5, r) = wm;
    // scale of the first right-hand side: the exponent of max|d| over the line
    {
        double dm = 0.0;
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < m) dm = gmax(dm, fabs(dv[t]));
        S(8, r) = dm;
    }
    __syncthreads();
    int E;
    {
        double D0 = 0.0;
        for (int q = 0; q < P; ++q) D0 = gmax(D0, S(8, q));
        E = gexponent(D0);
    }

    int sweep = 0;
    bool converged = false;
    double dprev = 0.0, est = 0.0;
    for (; sweep <= R.max_sweeps; ++sweep) {
        const double sc = ldexp(1.0, -E);
        if (sweep == 0) {
#pragma unroll
            for (int t = 0; t < CMAX; ++t) e[t] = (float)(dv[t] * sc);
        } else {
            // r = d - A x from the original coefficients, in FP64, as
            // d - a (x_{j-1} - x_j) - c (x_{j+1} - x_j) - (a + b + c) x_j with the
            // row sum rounded once
            double xlast = 0.0;
#pragma unroll
            for (int t = 0; t < CMAX; ++t)
                if (t == m - 1) xlast = xv[t];
            S(6, r) = xv[0];
            S(7, r) = xlast;
            __syncthreads();
            double xm = has_l ? S(7, Lp) : 0.0;
            const double xr = has_r ? S(6, Rp) : 0.0;
#pragma unroll
            for (int t = 0; t < CMAX; ++t)
                if (t < m) {
                    const double aJ = (t == 0) ? a_first : ca[t * csj];
                    const double cJ = (t == m - 1) ? c_last : cc[t * csj];
                    const double xp = (t + 1 < m) ? xv[(t + 1 < CMAX) ? t + 1 : t] : xr;
                    const double s1 = aJ + cJ, bb = s1 - aJ;
                    const double t1 = (aJ - (s1 - bb)) + (cJ - bb);
                    const double eJ = (cbp[t * csj] + s1) + t1;
                    const double res = dv[t] - (aJ * (xm - xv[t]) + cJ * (xp - xv[t]) + eJ * xv[t]);
                    xm = xv[t];
                    e[t] = (float)(res * sc);
                }
        }
        // FP32 solve of A~_r delta~ = r
        float gx = 0.0f;
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < m) {
                gx = (e[t] - fa[t] * gx) * fbeta[t];
                e[t] = gx;
            }
        const float xl = gx;
        float xn = 0.0f;
#pragma unroll
        for (int t = CMAX - 1; t >= 0; --t)
            if (t < m) {
                xn = e[t] - fcp[t] * xn;
                e[t] = xn;
            }
        S(0, r) = (double)e[0];
        S(1, r) = (double)xl;
        __syncthreads();
        // reduced system (FP64)
        double yl = 0.0, yr = 0.0;
        const double xf = (double)e[0];
        if (METHOD == TRI_PDD) {
            if (has_l) yl = (S(1, Lp) - S(5, Lp) * xf) / (1.0 - S(5, Lp) * v0);
            if (has_r) yr = (S(0, Rp) - S(2, Rp) * (double)xl) / (1.0 - wm * S(2, Rp));
        } else {
            const int NI = periodic ? P : P - 1, K = 2 * NI;
            double rhs[kGenKMax];
            bool ok = true;
            if (!periodic) {
                double dl[kGenKMax], dd[kGenKMax], du[kGenKMax];
                for (int i = 1; i <= NI; ++i) {
                    const int Li = i - 1, Ri = i;
                    const int u1 = 2 * i - 2, u2 = 2 * i - 1;
                    if (u1 > 0) dl[u1 - 1] = S(3, Li);
                    dd[u1] = S(5, Li);
                    du[u1] = 1.0;
                    dl[u1] = 1.0;
                    dd[u2] = S(2, Ri);
                    if (u2 < K - 1) du[u2] = S(4, Ri);
                    rhs[u1] = S(1, Li);
                    rhs[u2] = S(0, Ri);
                }
                if (K > 0) ok = gtsv_pivot(K, dl, dd, du, rhs);
            } else {
                double Zm[kGenKDense * kGenKDense];
                for (int t = 0; t < K * kGenKDense; ++t) Zm[t] = 0.0;
                for (int i = 1; i <= NI; ++i) {
                    const int Li = i - 1, Ri = i % P;
                    const int u1 = 2 * i - 2, u2 = 2 * i - 1;
                    const int il = (Li >= 1) ? Li : P, ir = Ri + 1;
                    Zm[u1 * kGenKDense + (u1 ^ 1)] += 1.0;
                    Zm[u1 * kGenKDense + (u2 ^ 1)] += S(5, Li);
                    Zm[u1 * kGenKDense + ((2 * il - 2) ^ 1)] += S(3, Li);
                    Zm[u2 * kGenKDense + (u2 ^ 1)] += 1.0;
                    Zm[u2 * kGenKDense + (u1 ^ 1)] += S(2, Ri);
                    Zm[u2 * kGenKDense + ((2 * ir - 1) ^ 1)] += S(4, Ri);
                    rhs[u1] = S(1, Li);
                    rhs[u2] = S(0, Ri);
                }
                ok = dense_gepp(K, Zm, rhs);
            }
            if (!ok && active) atomicOr(R.status, kStatusZeroPivot);
            if (has_l) yl = rhs[2 * ((r >= 1) ? r : P) - 1];
            if (has_r) yr = rhs[2 * r];
        }
        // correction delta = x~ - (y_l v + y_r w), v and w back-substituted
        // with the same multipliers, then undo the scale
        const double unscale = ldexp(1.0, E);
        double dmax = 0.0, xmax = 0.0, dn = 0.0;
#pragma unroll
        for (int t = CMAX - 1; t >= 0; --t)
            if (t < m) {
                const double gd = yl * (double)fgv[t] + ((t == m - 1) ? yr * wm : 0.0);
                dn = gd - (double)fcp[t] * dn;
                const double delta = ((double)e[t] - dn) * unscale;
                xv[t] += delta;
                dmax = gmax(dmax, fabs(delta));
                xmax = gmax(xmax, fabs(xv[t]));
            }
        // convergence of every line of the workgroup
        S(8, r) = dmax;
        S(9, r) = xmax;
        __syncthreads();
        if (r == 0) {
            double D = 0.0, X = 0.0;
            for (int q = 0; q < P; ++q) {
                D = gmax(D, S(8, q));
                X = gmax(X, S(9, q));
            }
            const double Xs = X > 0.0 ? X : 1.0;
            const double rate = (dprev > 0.0) ? fmin(1.0, D / dprev) : (D > 0.0 ? 1.0 : 0.0);
            est = (sweep == 0) ? 1.0 : (D / Xs) * rate;
            const bool ok = !active || (sweep >= 1 && D <= R.tol * Xs) || (sweep >= 2 && est <= R.tol);
            dprev = D;
            escale[lane] = gexponent(D);
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
    if (r == 0 && R.resid_bits) {
        double ev = active ? fabs(est) : 0.0;
        for (int off = 32; off > 0; off >>= 1) ev = gmax(ev, __shfl_xor(ev, off));
        if (lane == 0) atomicMax(R.resid_bits, (unsigned long long)__double_as_longlong(ev));
    }
    if (active) {
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < m) p[t * sj] = xv[t];
    }
}

size_t general_refine_lds_bytes(int P) { return sizeof(double) * 10 * (size_t)P * 64 + sizeof(int) * 65; }

template <int CMAX, int METHOD>
static hipError_t launch_general_refine_t(const GeneralArgs &a, const RefineArgs &R, hipStream_t s)
{
    const int64_t blocks = a.ngroups0 * a.nb1;
    hipLaunchKernelGGL((k_general_refine<CMAX, METHOD>), dim3((unsigned)blocks), dim3(64 * a.P),
                       general_refine_lds_bytes(a.P), s, a, R);
    return hipGetLastError();
}

hipError_t launch_general_refine(const GeneralArgs &a, const RefineArgs &R, int method, hipStream_t s)
{
    if (a.m <= 8)
        return method == TRI_PDD ? launch_general_refine_t<8, TRI_PDD>(a, R, s)
                                 : launch_general_refine_t<8, TRI_PPT>(a, R, s);
    if (a.m <= 16)
        return method == TRI_PDD ? launch_general_refine_t<16, TRI_PDD>(a, R, s)
                                 : launch_general_refine_t<16, TRI_PPT>(a, R, s);
    return hipErrorInvalidValue;
}

}  // namespace tri
