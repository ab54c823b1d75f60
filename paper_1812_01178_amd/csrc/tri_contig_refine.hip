// tri_contig_refine.hip -- FP32 elimination with FP64 residual refinement for
// lines whose rows are contiguous (the x sweep), one shared matrix.
//
// The iteration is the one of the strided refinement kernel (not in the
// paper; the partitioned solve of Sec. 3.2 is the inner solver):
//
//     x_0 = 0,  r_0 = d
//     repeat: delta = S32(r);  x += delta;  r = d - A x      (FP64)
//
// with the local eliminations of Eqs. (5)-(6) in FP32, the reduced system
// (Eq. (7) / (10)) and the correction in FP64, the residual from the true
// rows (a, a+b+c, c) in FP64, each line's right-hand side scaled by a power
// of two before rounding to FP32, and the same stopping rule (the error
// estimate |delta_s|^2 / |delta_{s-1}| of a linearly contracting iteration,
// max norms over the line, after at least two refinements, or one update
// already below the tolerance).
//
// Mapping as the FP64 register-factor kernel: one line per workgroup, thread
// (r, k) owns rows [r*m + k*C, +C) of partition r and keeps the FP32 factors
// and the FP64 true rows of those rows in VGPRs; the FP32 recurrences run as
// zero-carry pass + Kogge-Stone scan of the chunk maps + exact pass.  The
// line is the workgroup, so the convergence vote is a workgroup reduction.
// HBM traffic equals the FP64 path: d is read once, x written once.
#include <hip/hip_runtime.h>

#include "tri_device.h"

namespace tri {

namespace {

__device__ __forceinline__ double rmax(double acc, double v) { return (v > acc || v != v) ? v : acc; }

__device__ __forceinline__ int scale_exponent(double v)
{
    if (!(v > 0.0) || !(v <= 1.7976931348623157e308)) return 0;
    return min(1000, max(-1000, ilogb(v)));
}

// workgroup-wide max of two values (NaN-propagating); every thread returns
// the same result.  red: [2][16] doubles of LDS.
__device__ __forceinline__ void block_max2(double &a, double &b, double *red)
{
    for (int off = 32; off > 0; off >>= 1) {
        a = rmax(a, __shfl_xor(a, off));
        b = rmax(b, __shfl_xor(b, off));
    }
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w] = a;
        red[16 + w] = b;
    }
    __syncthreads();
    a = 0.0;
    b = 0.0;
    for (int q = 0; q < nw; ++q) {
        a = rmax(a, red[q]);
        b = rmax(b, red[16 + q]);
    }
}

}  // namespace

template <int C, int METHOD>
__global__ void __launch_bounds__(512) k_contig_refine(const SolveArgs A, const RefineArgs R)
{
    extern __shared__ double lds[];
    constexpr int Q = C / 2;
    constexpr int kSteps = 6;
    const int tid = threadIdx.x;
    const int LL = A.LL, Lp = A.Lp, P = A.P, S = A.stage_stride;
    const int r = tid / Lp;
    const int k = tid - r * Lp;
    const int64_t n = A.n;
    double *stage = lds;                  // [Q][S]
    double *tips = stage + Q * S;         // [2P]
    double *itl = tips + 2 * P;           // [P][2][2P]
    double *xb = itl + 4 * P * P;         // [2][LL] first / last x of every thread
    double *red = xb + 2 * LL;            // [2][16] per-wavefront maxima

    const double *__restrict__ IT = A.IT + A.g_off * (int64_t)(P * 4 * P);
    for (int i = tid; i < P * 4 * P; i += LL) itl[i] = IT[i];

    // this thread's rows: FP32 factors, FP64 true rows, FP32 scan multipliers
    const int64_t J0 = (int64_t)r * A.m + (int64_t)k * C;
    const float *__restrict__ F = R.F32 + A.g_off * (kNumFactors * n) + J0;
    const double *__restrict__ O = R.ORIG + A.g_off * (3 * n) + J0;
    float fb[C], fa[C], fc[C], fv[C], fw[C];
    double oa[C], oe[C], oc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        fb[c] = F[c];
        fa[c] = F[n + c];
        fc[c] = F[2 * n + c];
        fv[c] = F[3 * n + c];
        fw[c] = F[4 * n + c];
        oa[c] = O[c];
        oe[c] = O[n + c];
        oc[c] = O[2 * n + c];
    }
    float psk[kSteps], ssk[kSteps];
    {
        float Ps = 1.0f, Ss = 1.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            Ps *= -fa[c];
            Ss *= -fc[c];
        }
#pragma unroll
        for (int si = 0; si < kSteps; ++si) {
            const int s = 1 << si;
            psk[si] = Ps;
            ssk[si] = Ss;
            if (s < Lp) {
                const float Po = __shfl_up(Ps, s, Lp);
                const float So = __shfl_down(Ss, s, Lp);
                if (k >= s) Ps *= Po;
                if (k + s < Lp) Ss *= So;
            }
        }
    }
    int soff[Q];
#pragma unroll
    for (int it = 0; it < Q; ++it) {
        const int v = it * LL + tid;
        soff[it] = (v % Q) * S + 2 * (v / Q);
    }
    const bool pinned = (A.flags[A.g_off] & 1) && r == 0 && k == 0;
    const double *__restrict__ it_rows = itl + r * 2 * (2 * P);
    auto line_ptr = [&](int64_t L) -> double * {
        if (A.lines_linear) return A.d + L * A.s_b0;
        const int64_t b0 = L % A.nb0, b1 = L / A.nb0;
        return A.d + b0 * A.s_b0 + b1 * A.s_b1;
    };
    // neighbours of this thread's first and last rows along the line
    const int tprev = tid > 0 ? tid - 1 : (A.periodic ? LL - 1 : -1);
    const int tnext = tid < LL - 1 ? tid + 1 : (A.periodic ? 0 : -1);

    for (int64_t L = blockIdx.x; L < A.nlines; L += gridDim.x) {
        // d of this thread's rows, through the coalesced staging planes
        v2d *line = (v2d *)line_ptr(L);
        __syncthreads();   // staging free (previous line stored; first pass: rows above)
#pragma unroll
        for (int it = 0; it < Q; ++it) *(v2d *)(stage + soff[it]) = __builtin_nontemporal_load(line + it * LL + tid);
        __syncthreads();
        double dv[C], xv[C];
        float e[C];
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            const v2d t = *(const v2d *)(stage + p * S + 2 * tid);
            dv[2 * p] = t.x;
            dv[2 * p + 1] = t.y;
        }
        if (pinned) dv[0] = 0.0;
        int E;
        {
            double dm = 0.0, unused = 0.0;
#pragma unroll
            for (int c = 0; c < C; ++c) dm = rmax(dm, fabs(dv[c]));
            block_max2(dm, unused, red);
            E = scale_exponent(dm);
        }
#pragma unroll
        for (int c = 0; c < C; ++c) xv[c] = 0.0;

        int sweep = 0;
        bool converged = false;
        double dprev = 0.0, est = 0.0;
        for (; sweep <= R.max_sweeps; ++sweep) {
            const double sc = ldexp(1.0, -E);
            if (sweep == 0) {
#pragma unroll
                for (int c = 0; c < C; ++c) e[c] = (float)(dv[c] * sc);
            } else {
                // r = d - A x in FP64 from the true rows; the neighbours of
                // the thread's end rows come from the adjacent threads
                xb[tid] = xv[0];
                xb[LL + tid] = xv[C - 1];
                __syncthreads();
                double xm = tprev >= 0 ? xb[LL + tprev] : 0.0;
                const double xr = tnext >= 0 ? xb[tnext] : 0.0;
#pragma unroll
                for (int c = 0; c < C; ++c) {
                    const double xp = c + 1 < C ? xv[c + 1 < C ? c + 1 : c] : xr;
                    const double res = dv[c] - (oa[c] * (xm - xv[c]) + oc[c] * (xp - xv[c]) + oe[c] * xv[c]);
                    xm = xv[c];
                    e[c] = (float)(res * sc);
                }
            }
            // FP32 elimination of A~ delta~ = r: forward, scanned over the partition's lanes
            float gp = 0.0f;
#pragma unroll
            for (int c = 0; c < C; ++c) gp = fb[c] * e[c] - fa[c] * gp;
            float Fs = gp;
#pragma unroll
            for (int si = 0; si < kSteps; ++si) {
                const int s = 1 << si;
                if (s < Lp) {
                    const float Fo = __shfl_up(Fs, s, Lp);
                    if (k >= s) Fs += psk[si] * Fo;
                }
            }
            float gin = __shfl_up(Fs, 1, Lp);
            if (k == 0) gin = 0.0f;
            gp = gin;
#pragma unroll
            for (int c = 0; c < C; ++c) {
                gp = fb[c] * e[c] - fa[c] * gp;
                e[c] = gp;
            }
            const float tip_last = gp;
            // backward
            float xn = 0.0f;
#pragma unroll
            for (int c = C - 1; c >= 0; --c) xn = e[c] - fc[c] * xn;
            float Bs = xn;
#pragma unroll
            for (int si = 0; si < kSteps; ++si) {
                const int s = 1 << si;
                if (s < Lp) {
                    const float Bo = __shfl_down(Bs, s, Lp);
                    if (k + s < Lp) Bs += ssk[si] * Bo;
                }
            }
            float xin = __shfl_down(Bs, 1, Lp);
            if (k == Lp - 1) xin = 0.0f;
            xn = xin;
#pragma unroll
            for (int c = C - 1; c >= 0; --c) {
                xn = e[c] - fc[c] * xn;
                e[c] = xn;
            }
            // reduced system and correction in FP64
            if (k == 0) tips[2 * r] = (double)e[0];
            if (k == Lp - 1) tips[2 * r + 1] = (double)tip_last;
            __syncthreads();
            double yl, yr;
            interface_unknowns<METHOD>(it_rows, r, P, A.periodic, [&](int q) { return tips[q]; }, yl, yr);
            const double unscale = ldexp(1.0, E);
            double dmax = 0.0, xmax = 0.0;
            bool nan = false;                   // (fmax drops NaNs: they are counted apart)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double delta = ((double)e[c] - yl * (double)fv[c] - yr * (double)fw[c]) * unscale;
                xv[c] += delta;
                nan |= !(delta == delta) || !(xv[c] == xv[c]);
                dmax = fmax(dmax, fabs(delta));
                xmax = fmax(xmax, fabs(xv[c]));
            }
            if (nan) dmax = xmax = __builtin_nan("");
            // convergence of the line (the workgroup): every thread takes the
            // same decision from the same reduced values
            block_max2(dmax, xmax, red);
            const double Xs = xmax > 0.0 ? xmax : 1.0;
            const double rate = (dprev > 0.0) ? fmin(1.0, dmax / dprev) : (dmax > 0.0 ? 1.0 : 0.0);
            est = (sweep == 0) ? 1.0 : (dmax / Xs) * rate;
            const double rel = dmax / Xs;
            const bool ok = (sweep >= 1 && dmax <= R.tol * Xs) || (sweep >= 2 && est <= R.tol) ||
                            (sweep == 1 && R.kappa > 0.0 && R.kappa * rel * rel <= R.tol);
            dprev = dmax;
            E = scale_exponent(dmax);
            if (ok) {
                converged = true;
                break;
            }
        }
        if (tid == 0) {
            if (!converged) atomicOr(R.status, kStatusNotConverged);
            if (R.sweeps_used) atomicMax(R.sweeps_used, converged ? sweep : R.max_sweeps);
            if (R.resid_bits) atomicMax(R.resid_bits, (unsigned long long)__double_as_longlong(fabs(est)));
        }
        // x of this line back through the staging planes
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            v2d t;
            t.x = xv[2 * p];
            t.y = xv[2 * p + 1];
            *(v2d *)(stage + p * S + 2 * tid) = t;
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < Q; ++it) __builtin_nontemporal_store(*(const v2d *)(stage + soff[it]), line + it * LL + tid);
    }
}

size_t contig_refine_lds_bytes(const SolveArgs &a)
{
    return sizeof(double) * ((size_t)(a.C / 2) * a.stage_stride + 2 * (size_t)a.P + 4 * (size_t)a.P * a.P +
                             2 * (size_t)a.LL + 32);
}

template <int C, int METHOD>
static hipError_t launch_contig_refine_t(const SolveArgs &a, const RefineArgs &R, int grid, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>(std::max(grid, 1), a.nlines);
    hipLaunchKernelGGL((k_contig_refine<C, METHOD>), dim3((unsigned)blocks), dim3(a.LL), contig_refine_lds_bytes(a),
                       s, a, R);
    return hipGetLastError();
}

template <int C, int METHOD>
static int contig_refine_grid_t(const SolveArgs &a)
{
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(&k_contig_refine<C, METHOD>), a.LL, contig_refine_lds_bytes(a)) !=
        hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return std::max(1, per_cu) * cus;
}

int contig_refine_grid(const SolveArgs &a, int method)
{
    const bool pdd = method == TRI_PDD;
    if (a.C == 4) return pdd ? contig_refine_grid_t<4, TRI_PDD>(a) : contig_refine_grid_t<4, TRI_PPT>(a);
    if (a.C == 8) return pdd ? contig_refine_grid_t<8, TRI_PDD>(a) : contig_refine_grid_t<8, TRI_PPT>(a);
    return 0;
}

hipError_t launch_contig_refine(const SolveArgs &a, const RefineArgs &R, int method, int grid, hipStream_t s)
{
    if (a.C == 4)
        return method == TRI_PDD ? launch_contig_refine_t<4, TRI_PDD>(a, R, grid, s)
                                 : launch_contig_refine_t<4, TRI_PPT>(a, R, grid, s);
    if (a.C == 8)
        return method == TRI_PDD ? launch_contig_refine_t<8, TRI_PDD>(a, R, grid, s)
                                 : launch_contig_refine_t<8, TRI_PPT>(a, R, grid, s);
    return hipErrorInvalidValue;
}

}  // namespace tri
