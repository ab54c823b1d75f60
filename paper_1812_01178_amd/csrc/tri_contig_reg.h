// tri_contig_reg.h -- the register-factor contiguous solve as a device
// function (tri_contig_reg.hip runs it as a persistent kernel, the level
// kernel in tri_kernels.hip runs it per block of a ragged batch).
//
// Same algebra as the other contiguous kernels (Sec. 3.2: local solves of
// Eqs. (5)-(6) by Thomas elimination, reduced system of Eq. (7) or (10),
// correction of Eq. (8) / (11)); only the mapping onto the machine differs:
//
//  * one line per block of LL = P * Lp threads: thread (r, k) owns rows
//    [r*m + k*C, +C) of partition r, so its factors (beta, alpha, cp and the
//    spikes v, w of those rows, 5*C doubles) are the same for every line and
//    stay in VGPRs for all the lines the block solves -- no factor traffic
//    per line;
//  * the reduced-system rows of the matrix are copied to LDS once;
//  * a line moves HBM -> LDS -> VGPRs and back with coalesced 16-byte
//    nontemporal accesses through a double-buffered staging area, so a line
//    costs three barriers;
//  * the next line's loads are issued before the current line is solved.
//
// Requirements (checked by the host): contiguous rows (s_j = 1), one shared
// matrix, C in {4, 8}, Lp = m / C a power of two <= 64, P * Lp a multiple
// of 64 and <= 512, n even and every line 16-byte aligned.
#pragma once

#include "tri_device.h"

namespace tri {

// The solve of lines L0, L0 + step, ... by LL = P * Lp threads (tid < LL)
// with `lds` holding contig_reg_lds_bytes of this block.  RUN = false: every
// such line below A.nlines (a persistent grid); RUN = true: `iters` lines,
// those at or past A.nlines ghosts (no field access, the same barriers), so
// that blocks sharing a workgroup meet the same barriers.
template <int C, int METHOD, bool RUN = false>
__device__ __forceinline__ void contig_reg_solve(const SolveArgs &A, int64_t L0, int64_t step, int64_t iters,
                                                 int tid, double *lds)
{
    constexpr int Q = C / 2;          // 16-byte pairs per thread per line
    constexpr int kSteps = 6;         // Kogge-Stone steps for up to 64 lanes per partition
    const int LL = A.LL, Lp = A.Lp, P = A.P, S = A.stage_stride;
    const int r = tid / Lp;
    const int k = tid - r * Lp;
    const int64_t n = A.n;
    double *stage = lds;                        // [2][Q][S]
    double *tips = lds + 2 * Q * S;             // [2P]
    double *itl = tips + 2 * P;                 // [P][2][2P]

    const gdouble *__restrict__ IT = (const gdouble *)(A.IT + A.g_off * (int64_t)(P * 4 * P));
    for (int i = tid; i < P * 4 * P; i += LL) itl[i] = IT[i];

    // this thread's rows of the factor table
    const gdouble *__restrict__ F = (const gdouble *)(A.F + A.g_off * (kNumFactors * n));
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
    const bool pinned = (((const gint *)A.flags)[A.g_off] & 1) && r == 0 && k == 0;
    const double *__restrict__ it_rows = itl + r * 2 * (2 * P);
    auto line_ptr = [&](int64_t L) -> gv2d * {
        if (A.lines_linear) return (gv2d *)(A.d + L * A.s_b0);
        const int64_t b0 = L % A.nb0, b1 = L / A.nb0;
        return (gv2d *)(A.d + b0 * A.s_b0 + b1 * A.s_b1);
    };

    const int64_t nlines = A.nlines;
    // The next line is loaded into VGPRs while this one is solved and is
    // written to the other staging buffer just before this line's stores are
    // issued, so the wait for those loads never includes the stores.
    const int64_t Lend = RUN ? L0 + iters * step : nlines;          // loop bound
    const int64_t Lreal = RUN ? (Lend < nlines ? Lend : nlines) : nlines;   // lines with data
    int buf = 0;
    if (L0 < Lreal) {
        const gv2d *src = line_ptr(L0);
#pragma unroll
        for (int it = 0; it < Q; ++it) *(v2d *)(stage + soff[it]) = __builtin_nontemporal_load(src + it * LL + tid);
    }
    for (int64_t L = L0; L < Lend; L += step) {
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
        const int64_t Ln = L + step;
        const bool more = Ln < Lreal;
        v2d pre[Q];
        if (more) {
            const gv2d *src = line_ptr(Ln);
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
        if (!RUN || L < nlines) {
            gv2d *dst = line_ptr(L);
#pragma unroll
            for (int it = 0; it < Q; ++it) __builtin_nontemporal_store(out[it], dst + it * LL + tid);
        }
    }
}


}  // namespace tri
