// tri_contig_reg.hip -- contiguous-row partitioned solve with the shared
// matrix's factors held in registers.
//
// Same algebra as the other contiguous kernels (Sec. 3.2: local solves of
// Eqs. (5)-(6) by Thomas elimination, reduced system of Eq. (7) or (10),
// correction of Eq. (8) / (11)); only the mapping onto the machine differs:
//
//  * one line per workgroup: thread (r, k) owns rows [r*m + k*C, +C) of
//    partition r, so its factors (beta, alpha, cp and the spikes v, w of
//    those rows, 5*C doubles) are the same for every line and stay in VGPRs
//    for the whole persistent loop -- no factor traffic at all per line;
//  * the reduced-system rows of the matrix are copied to LDS once;
//  * a line moves HBM -> LDS -> VGPRs and back with coalesced 16-byte
//    nontemporal accesses through a double-buffered staging area, so a line
//    costs three workgroup barriers;
//  * the next line's loads are issued before the current line is solved;
//  * workgroups are small (one line) and several are resident per CU, so one
//    workgroup's barrier and memory waits overlap the others' work.
//
// Requirements (checked by the host): contiguous rows (s_j = 1), one shared
// matrix, C in {4, 8}, Lp = m / C a power of two <= 64, P * Lp a multiple
// of 64 and <= 512, n even and every line 16-byte aligned.
#include <hip/hip_runtime.h>

#include "tri_device.h"

namespace tri {

template <int C, int METHOD>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(C == 8 ? 2 : 4)))
k_contig_reg(const SolveArgs A)
{
    extern __shared__ double lds[];
    constexpr int Q = C / 2;          // 16-byte pairs per thread per line
    constexpr int kSteps = 6;         // Kogge-Stone steps for up to 64 lanes per partition
    const int tid = threadIdx.x;
    const int LL = A.LL, Lp = A.Lp, P = A.P, S = A.stage_stride;
    const int r = tid / Lp;
    const int k = tid - r * Lp;
    const int64_t n = A.n;
    double *stage = lds;                        // [2][Q][S]
    double *tips = lds + 2 * Q * S;             // [2P]
    double *itl = tips + 2 * P;                 // [P][2][2P]

    const double *__restrict__ IT = A.IT + A.g_off * (int64_t)(P * 4 * P);
    for (int i = tid; i < P * 4 * P; i += LL) itl[i] = IT[i];

    // this thread's rows of the factor table
    const double *__restrict__ F = A.F + A.g_off * (kNumFactors * n);
    const int64_t J0 = (int64_t)r * A.m + (int64_t)k * C;
    double fb[C], fa[C], fc[C], fv[C], fw[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        fb[c] = F[J0 + c];
        fa[c] = F[n + J0 + c];
        fc[c] = F[2 * n + J0 + c];
        fv[c] = F[3 * n + J0 + c];
        fw[c] = F[4 * n + J0 + c];
    }
    // multipliers of the partner's carry at each scan step: the product of
    // the chunk maps' slopes (-alpha forward, -cp backward) of the lanes
    // between this lane and the partner
    double psk[kSteps], ssk[kSteps];
    {
        double Ps = 1.0, Ss = 1.0;
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
                const double Po = __shfl_up(Ps, s, Lp);
                const double So = __shfl_down(Ss, s, Lp);
                if (k >= s) Ps *= Po;
                if (k + s < Lp) Ss *= So;
            }
        }
    }
    // coalesced copy slots: pair v = it*LL + tid of the line holds rows
    // 2v, 2v+1, i.e. pair (v % Q) of owner thread v / Q
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

    const int64_t nlines = A.nlines;
    // The next line is loaded into VGPRs while this one is solved and is
    // written to the other staging buffer just before this line's stores are
    // issued, so the wait for those loads never includes the stores.
    int buf = 0;
    if ((int64_t)blockIdx.x < nlines) {
        const v2d *src = (const v2d *)line_ptr(blockIdx.x);
#pragma unroll
        for (int it = 0; it < Q; ++it) *(v2d *)(stage + soff[it]) = __builtin_nontemporal_load(src + it * LL + tid);
    }
    for (int64_t L = blockIdx.x; L < nlines; L += gridDim.x) {
        double *st = stage + buf * (Q * S);
        __syncthreads();   // line L staged (first pass: also the reduced-system rows)
        double x[C];
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            const v2d t = *(const v2d *)(st + p * S + 2 * tid);
            x[2 * p] = t.x;
            x[2 * p + 1] = t.y;
        }
        if (pinned) x[0] = 0.0;
        const int64_t Ln = L + gridDim.x;
        const bool more = Ln < nlines;
        v2d pre[Q];
        if (more) {
            const v2d *src = (const v2d *)line_ptr(Ln);
#pragma unroll
            for (int it = 0; it < Q; ++it) pre[it] = __builtin_nontemporal_load(src + it * LL + tid);
        }

        // forward elimination of this thread's rows with a zero carry; the
        // chunk map g_out = G + M * g_in is then scanned across the lanes of
        // the partition (M = product of -alpha), giving each lane its carry
        double gp = 0.0;
#pragma unroll
        for (int c = 0; c < C; ++c) gp = fb[c] * x[c] - fa[c] * gp;
        double Fs = gp;
#pragma unroll
        for (int si = 0; si < kSteps; ++si) {
            const int s = 1 << si;
            if (s < Lp) {
                const double Fo = __shfl_up(Fs, s, Lp);
                if (k >= s) Fs += psk[si] * Fo;
            }
        }
        double gin = __shfl_up(Fs, 1, Lp);
        if (k == 0) gin = 0.0;
        gp = gin;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            gp = fb[c] * x[c] - fa[c] * gp;
            x[c] = gp;
        }
        const double tip_last = gp;

        // back substitution, scanned the same way from the partition's end
        double xn = 0.0;
#pragma unroll
        for (int c = C - 1; c >= 0; --c) xn = x[c] - fc[c] * xn;
        double Bs = xn;
#pragma unroll
        for (int si = 0; si < kSteps; ++si) {
            const int s = 1 << si;
            if (s < Lp) {
                const double Bo = __shfl_down(Bs, s, Lp);
                if (k + s < Lp) Bs += ssk[si] * Bo;
            }
        }
        double xin = __shfl_down(Bs, 1, Lp);
        if (k == Lp - 1) xin = 0.0;
        xn = xin;
#pragma unroll
        for (int c = C - 1; c >= 0; --c) {
            xn = x[c] - fc[c] * xn;
            x[c] = xn;
        }

        // reduced system: tips of every partition, then this partition's
        // interface unknowns and the correction x = x~ - y_l v - y_r w
        if (k == 0) tips[2 * r] = x[0];
        if (k == Lp - 1) tips[2 * r + 1] = tip_last;
        __syncthreads();   // tips complete
        double yl, yr;
        interface_unknowns<METHOD>(it_rows, r, P, A.periodic, [&](int q) { return tips[q]; }, yl, yr);
#pragma unroll
        for (int p = 0; p < Q; ++p) {
            v2d t;
            t.x = x[2 * p] - yl * fv[2 * p] - yr * fw[2 * p];
            t.y = x[2 * p + 1] - yl * fv[2 * p + 1] - yr * fw[2 * p + 1];
            *(v2d *)(st + p * S + 2 * tid) = t;
        }
        __syncthreads();   // solution staged
        v2d out[Q];
#pragma unroll
        for (int it = 0; it < Q; ++it) out[it] = *(const v2d *)(st + soff[it]);
        buf ^= 1;
        if (more) {
            double *sn = stage + buf * (Q * S);
#pragma unroll
            for (int it = 0; it < Q; ++it) *(v2d *)(sn + soff[it]) = pre[it];
        }
        v2d *dst = (v2d *)line_ptr(L);
#pragma unroll
        for (int it = 0; it < Q; ++it) __builtin_nontemporal_store(out[it], dst + it * LL + tid);
    }
}

size_t contig_reg_lds_bytes(const SolveArgs &a)
{
    return sizeof(double) * ((size_t)2 * (a.C / 2) * a.stage_stride + 2 * (size_t)a.P + 4 * (size_t)a.P * a.P);
}

template <int C, int METHOD>
static hipError_t launch_contig_reg_t(const SolveArgs &a, int grid, hipStream_t s)
{
    const int64_t blocks = std::min<int64_t>(std::max(grid, 1), a.nlines);
    hipLaunchKernelGGL((k_contig_reg<C, METHOD>), dim3((unsigned)blocks), dim3(a.LL), contig_reg_lds_bytes(a), s, a);
    return hipGetLastError();
}

template <int C, int METHOD>
static int contig_reg_grid_t(const SolveArgs &a)
{
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(&k_contig_reg<C, METHOD>),
                                                     a.LL, contig_reg_lds_bytes(a)) != hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return std::max(1, per_cu) * cus;
}

int contig_reg_grid(const SolveArgs &a, int method)
{
    const bool pdd = method == TRI_PDD;
    if (a.C == 4) return pdd ? contig_reg_grid_t<4, TRI_PDD>(a) : contig_reg_grid_t<4, TRI_PPT>(a);
    if (a.C == 8) return pdd ? contig_reg_grid_t<8, TRI_PDD>(a) : contig_reg_grid_t<8, TRI_PPT>(a);
    return 0;
}

hipError_t launch_contig_reg(const SolveArgs &a, int method, int grid, hipStream_t s)
{
    if (a.C == 4)
        return method == TRI_PDD ? launch_contig_reg_t<4, TRI_PDD>(a, grid, s)
                                 : launch_contig_reg_t<4, TRI_PPT>(a, grid, s);
    if (a.C == 8)
        return method == TRI_PDD ? launch_contig_reg_t<8, TRI_PDD>(a, grid, s)
                                 : launch_contig_reg_t<8, TRI_PPT>(a, grid, s);
    return hipErrorInvalidValue;
}

}  // namespace tri
