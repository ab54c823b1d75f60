// tri_kernels.hip -- gfx950 kernels of libtri (FP64 path).
//
// Partitioned tridiagonal solves of Ha, Park & You (arXiv:1812.01178),
// Sec. 3.2: every line of n rows is split into P partitions; each partition
// solves its block A~_r (Eqs. (5), (6)); the partitions exchange the first
// and last entries of x~ ("tips"); the reduced system (PDD: 2x2 blocks of
// Eq. (7); PPT: Zbar of Eq. (10)) gives the interface unknowns; the
// correction x = x~ - Y y (Eqs. (8), (11)) is fused into the store.
//
// The paper runs one partition per GPU and exchanges tips with MPI; here the
// partitions of a line live in one workgroup and exchange tips through LDS.
// The path is HBM-bound (about 1 flop per byte), so the kernels are built
// around coalesced loads and stores and on-chip residency of each partition
// between its elimination and its correction; no matrix-core work.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tri_contig_reg.h"
#include "tri_device.h"

namespace tri {

// ===========================================================================
// Factor kernel: one workgroup per shared matrix g, one thread per partition.
// Writes the Thomas factors and spikes of every partition block (Eqs. (5),
// (6) are linear in the right-hand side, so everything except d is done
// once per matrix) and the reduced-system rows of every partition.
// ===========================================================================
struct MatView {
    MatSrc S;
    int64_t g;
    bool pin;
    __device__ double A(int64_t J) const { return S.a[J * S.cs_j + g * S.cs_g]; }
    __device__ double Cc(int64_t J) const {
        if (pin && J == 0) return 0.0;
        return S.c[J * S.cs_j + g * S.cs_g];
    }
    __device__ double B(int64_t J) const {
        if (S.lam) {
            if (pin && J == 0) return 1.0;
            return -(S.a[J * S.cs_j + g * S.cs_g] + S.c[J * S.cs_j + g * S.cs_g]) - S.lam[g];
        }
        return S.b[J * S.cs_j + g * S.cs_g];
    }
};

// Small dense LU with partial pivoting, K <= 2*kPMax, row-major in LDS.
constexpr int kKMax = 2 * kPMax;

__global__ __launch_bounds__(64) void k_factor(MatSrc S, Tables T, int *status)
{
    __shared__ double Z[kKMax * kKMax];
    __shared__ double Zi[kKMax * kKMax];
    __shared__ int piv[kKMax];
    __shared__ int bad_lu;

    const int64_t g = blockIdx.x;
    const int P = T.P;
    const int64_t n = T.n;
    const int m = (int)(n / P);
    const int periodic = T.periodic;
    MatView M{S, g, S.lam != nullptr && S.lam[g] == 0.0};
    double *F = T.F + g * kNumFactors * n;
    double *Fb = F, *Fa = F + n, *Fc = F + 2 * n, *Fv = F + 3 * n, *Fw = F + 4 * n;
    const int tid = threadIdx.x;

    if (tid == 0) {
        T.flags[g] = M.pin ? 1 : 0;
        bad_lu = 0;
    }
    if (tid < P) {
        const int r = tid;
        const int64_t o = (int64_t)r * m;
        bool bad = false;
        double cpp = 0.0;
        for (int t = 0; t < m; ++t) {
            const int64_t J = o + t;
            const double aa = (t == 0) ? 0.0 : M.A(J);        // corner removed
            const double cc = (t == m - 1) ? 0.0 : M.Cc(J);    // corner removed
            const double den = M.B(J) - aa * cpp;
            if (!(den != 0.0) || !isfinite(den)) bad = true;
            const double beta = 1.0 / den;
            Fb[J] = beta;
            Fa[J] = aa * beta;
            cpp = cc * beta;
            Fc[J] = cpp;
        }
        // spike v^(r) = A~_r^{-1} (a_{rm} e_0): only partitions with a left coupling
        const double a_first = (r >= 1 || periodic) ? M.A(o) : 0.0;
        double gv = 0.0;
        for (int t = 0; t < m; ++t) {
            const int64_t J = o + t;
            gv = (t == 0) ? Fb[J] * a_first : -Fa[J] * gv;
            Fv[J] = gv;
        }
        double vn = 0.0;
        for (int t = m - 1; t >= 0; --t) {
            const int64_t J = o + t;
            vn = Fv[J] - Fc[J] * vn;
            Fv[J] = vn;
        }
        // spike w^(r) = A~_r^{-1} (c_{rm+m-1} e_{m-1}): only with a right coupling
        const double c_last = (r <= P - 2 || periodic) ? M.Cc(o + m - 1) : 0.0;
        double wn = Fb[o + m - 1] * c_last;
        Fw[o + m - 1] = wn;
        for (int t = m - 2; t >= 0; --t) {
            const int64_t J = o + t;
            wn = -Fc[J] * wn;
            Fw[J] = wn;
        }
        if (bad) atomicOr(status, kStatusZeroPivot);
        // FP32 copy of the factors and the true rows for the refinement residual
        float *F32 = T.F32 + g * kNumFactors * n;
        double *O = T.ORIG + g * 3 * n;
        for (int t = 0; t < m; ++t) {
            const int64_t J = o + t;
            for (int f = 0; f < kNumFactors; ++f) F32[f * n + J] = (float)F[f * n + J];
            const double aJ = (J == 0 && !periodic) ? 0.0 : M.A(J);
            const double cJ = (J == n - 1 && !periodic) ? 0.0 : M.Cc(J);
            // row sum a + b + c to full FP64 accuracy (error-free a + c, then b)
            const double s1 = aJ + cJ;
            const double bb = s1 - aJ;
            const double t1 = (aJ - (s1 - bb)) + (cJ - bb);
            O[J] = aJ;
            O[n + J] = (M.B(J) + s1) + t1;
            O[2 * n + J] = cJ;
        }
    }
    // zero this matrix's reduced-system rows
    const int rowlen = 2 * P;
    double *IT = T.IT + g * (int64_t)P * 2 * rowlen;
    for (int i = tid; i < P * 2 * rowlen; i += blockDim.x) IT[i] = 0.0;
    __syncthreads();

    const int NI = periodic ? P : P - 1;
    const int K = 2 * NI;
    auto vfirst = [&](int q) { return Fv[(int64_t)q * m]; };
    auto vlast = [&](int q) { return Fv[(int64_t)q * m + m - 1]; };
    auto wfirst = [&](int q) { return Fw[(int64_t)q * m]; };
    auto wlast = [&](int q) { return Fw[(int64_t)q * m + m - 1]; };

    if (tid == 0) {
        // entries PDD drops from Z: v_m^(L) and w_1^(R) of every interface
        double dmax = 0.0;
        for (int i = 1; i <= NI; ++i) {
            const int L = i - 1, R = i % P;
            if (L >= 1 || periodic) dmax = fmax(dmax, fabs(vlast(L)));
            if (R <= P - 2 || periodic) dmax = fmax(dmax, fabs(wfirst(R)));
        }
        T.drop[g] = dmax;
        if (T.method == TRI_PDD && T.pdd_tol > 0.0 && dmax > T.pdd_tol) atomicOr(status, kStatusPddUnsafe);
    }

    if (T.method == TRI_PDD) {
        // 2x2 block of interface i: [[1, w_m^(L)], [v_1^(R), 1]] (y_{2i-1}, y_{2i})
        //   = (x~_m^(L), x~_1^(R)); inverse of a 2x2 matrix (Algorithm 1, step 5).
        if (tid < NI) {
            const int i = tid + 1, L = i - 1, R = i % P;
            const double w = wlast(L), v = vfirst(R);
            const double det = 1.0 - w * v;
            if (!(det != 0.0)) atomicOr(status, kStatusZeroPivot);
            const double inv = 1.0 / det;
            // y_{2i-1}: left unknown of partition R
            double *rowR = IT + ((int64_t)R * 2 + 0) * rowlen;
            rowR[2 * L + 1] += inv;
            rowR[2 * R] += -w * inv;
            // y_{2i}: right unknown of partition L
            double *rowL = IT + ((int64_t)L * 2 + 1) * rowlen;
            rowL[2 * R] += inv;
            rowL[2 * L + 1] += -v * inv;
        }
        return;
    }

    // PPT: Zbar = Z P (Eq. (10)), factor with partial pivoting, invert.
    if (K == 0) return;
    if (tid == 0) {
        for (int t = 0; t < K * K; ++t) Z[t] = 0.0;
        for (int i = 1; i <= NI; ++i) {
            const int L = i - 1, R = i % P;
            const int u1 = 2 * i - 2, u2 = 2 * i - 1;
            // row of y_{2i-1}; columns already swapped in pairs (Zbar = Z P)
            Z[u1 * K + (u1 ^ 1)] += 1.0;
            Z[u1 * K + (u2 ^ 1)] += wlast(L);
            if (L >= 1 || periodic) {
                const int il = (L >= 1) ? L : P;
                Z[u1 * K + ((2 * il - 2) ^ 1)] += vlast(L);
            }
            Z[u2 * K + (u2 ^ 1)] += 1.0;
            Z[u2 * K + (u1 ^ 1)] += vfirst(R);
            if (R <= P - 2 || periodic) {
                const int ir = R + 1;
                Z[u2 * K + ((2 * ir - 1) ^ 1)] += wfirst(R);
            }
        }
        for (int k = 0; k < K; ++k) {
            int p = k;
            double best = fabs(Z[k * K + k]);
            for (int i = k + 1; i < K; ++i)
                if (fabs(Z[i * K + k]) > best) { best = fabs(Z[i * K + k]); p = i; }
            piv[k] = p;
            if (best == 0.0) { bad_lu = 1; break; }
            if (p != k)
                for (int t = 0; t < K; ++t) { double s = Z[k * K + t]; Z[k * K + t] = Z[p * K + t]; Z[p * K + t] = s; }
            for (int i = k + 1; i < K; ++i) {
                const double l = Z[i * K + k] / Z[k * K + k];
                Z[i * K + k] = l;
                for (int t = k + 1; t < K; ++t) Z[i * K + t] -= l * Z[k * K + t];
            }
        }
        if (bad_lu) atomicOr(status, kStatusZeroPivot);
    }
    __syncthreads();
    if (bad_lu) return;
    if (tid < K) {
        // column tid of Zbar^{-1}
        double col[kKMax];
        for (int i = 0; i < K; ++i) col[i] = (i == tid) ? 1.0 : 0.0;
        // rows were interchanged whole (multipliers included), so the stored L
        // belongs to the fully permuted matrix: permute first, then substitute
        for (int k = 0; k < K; ++k) {
            const int p = piv[k];
            if (p != k) { double s = col[k]; col[k] = col[p]; col[p] = s; }
        }
        for (int k = 0; k < K; ++k)
            for (int i = k + 1; i < K; ++i) col[i] -= Z[i * K + k] * col[k];
        for (int k = K - 1; k >= 0; --k) {
            double s = col[k];
            for (int t = k + 1; t < K; ++t) s -= Z[k * K + t] * col[t];
            col[k] = s / Z[k * K + k];
        }
        for (int i = 0; i < K; ++i) Zi[i * K + tid] = col[i];
    }
    __syncthreads();
    if (tid < P) {
        const int r = tid;
        // E^T x~ entry u in terms of the tip vector T: u = 2i-2 -> last of L(i),
        // u = 2i-1 -> first of R(i).
        auto tipidx = [&](int u) {
            const int i = u / 2 + 1;
            return (u & 1) ? 2 * (i % P) : 2 * (i - 1) + 1;
        };
        if (r >= 1 || periodic) {
            const int il = (r >= 1) ? r : P;
            const int row = 2 * il - 1;              // y_{2il-1} = ybar_{2il}
            double *dst = IT + ((int64_t)r * 2 + 0) * rowlen;
            for (int u = 0; u < K; ++u) dst[tipidx(u)] += Zi[row * K + u];
        }
        if (r <= P - 2 || periodic) {
            const int row = 2 * r;                   // y_{2r+2} = ybar_{2r+1}
            double *dst = IT + ((int64_t)r * 2 + 1) * rowlen;
            for (int u = 0; u < K; ++u) dst[tipidx(u)] += Zi[row * K + u];
        }
    }
}

hipError_t launch_factor(const MatSrc &src, const Tables &T, int *status, hipStream_t s)
{
    if (T.G <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_factor, dim3((unsigned)T.G), dim3(64), 0, s, src, T, status);
    return hipGetLastError();
}

// ===========================================================================
// Strided-direction solve (rows j at stride s_j, lines side by side).
// Workgroup = P*kc wavefronts; wavefront w = r*kc + s holds chunk s (Cs =
// m/kc consecutive rows) of partition r for 64 neighbouring lines (lane =
// line).  Every row access of a wavefront is one coalesced 512-byte segment,
// every factor is wavefront-uniform (scalar loads), and the chunk's values
// stay in VGPRs from load to store.  With kc > 1 the partition's forward and
// backward Thomas recurrences are carried across its chunks through LDS
// (zero-carry pass, combine the chunk maps, exact pass), which is the same
// elimination as one wavefront per partition with a smaller VGPR footprint.
// ===========================================================================
// Workgroup blk -> (line group grp, outer index b1).  Order 0: line groups
// fastest; 1: outer index fastest; 2: as 0, but workgroups that run on one
// XCD (dispatched round-robin over the 8 XCDs) take a contiguous range.
__device__ __forceinline__ void strided_block(const SolveArgs &A, int64_t blk, int64_t &grp, int64_t &b1)
{
    int64_t b = blk;
    if (A.blk_map == 2) {
        const int64_t nb = A.ngroups0 * A.nb1, per = nb / 8, rem = nb % 8, xcd = blk % 8, idx = blk / 8;
        b = xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
    }
    if (A.blk_map == 1) {
        b1 = b % A.nb1;
        grp = b / A.nb1;
    } else {
        grp = b % A.ngroups0;
        b1 = b / A.ngroups0;
    }
}

// tid: the thread's index in the block (64 * P * kc threads).  A ghost block
// (a level launch's padding) runs the same barriers and LDS traffic with every
// lane inactive: it reads and writes no field memory.
template <int CMAX, int METHOD, bool CHUNKED, bool ACC = false>
__device__ __forceinline__ void strided_solve(const SolveArgs &A, int64_t blk, double *lds, int tid,
                                              bool ghost = false)
{
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int kc = A.kc, Cs = A.Cs;
    const int r = w / kc, s = w - r * kc;
    const int P = A.P, m = A.m;
    const int nw = P * kc;
    double *tips = lds;                          // [2P][64]
    double *fend = lds + 2 * P * 64;             // [nw][64] forward chunk ends
    double *bbeg = fend + nw * 64;               // [nw][64] backward chunk starts
    double *pif = bbeg + nw * 64;                // [nw] forward chunk multipliers
    double *pib = pif + nw;                      // [nw] backward chunk multipliers

    int64_t grp, b1;
    strided_block(A, blk, grp, b1);
    const int64_t b0 = grp * 64 + lane;
    const bool active = !ghost && b0 < A.nb0;
    const int64_t n = A.n;
    const int64_t g = b1 * A.g_b1 + A.g_off;
    const int64_t row0 = (int64_t)r * m + (int64_t)s * Cs;
    const cdouble *__restrict__ F = (const cdouble *)(A.F + g * (kNumFactors * n) + row0);
    const cdouble *__restrict__ Fb = F;
    const cdouble *__restrict__ Fa = F + n;
    const cdouble *__restrict__ Fc = F + 2 * n;
    const cdouble *__restrict__ Fv = F + 3 * n;
    const cdouble *__restrict__ Fw = F + 4 * n;
    const int64_t sj = A.s_j;
    gdouble *__restrict__ p = (gdouble *)(A.d + (active ? b0 : 0) * A.s_b0 + b1 * A.s_b1 + row0 * sj);

    double x[CMAX];
#pragma unroll
    for (int t = 0; t < CMAX; ++t) x[t] = 0.0;
    if (active) {
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < Cs) x[t] = __builtin_nontemporal_load(p + t * sj);
    }
    if (r == 0 && s == 0 && (((const cint *)A.flags)[g] & 1)) x[0] = 0.0;   // gauge-pinned row

    // Eq. (5): A~_r x~ = d with the precomputed pivots
    double tip_last;
    if (!CHUNKED) {
        double gp = 0.0;
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < Cs) {
                gp = Fb[t] * x[t] - Fa[t] * gp;
                x[t] = gp;
            }
        tip_last = gp;
        double xn = 0.0;
#pragma unroll
        for (int t = CMAX - 1; t >= 0; --t)
            if (t < Cs) {
                xn = x[t] - Fc[t] * xn;
                x[t] = xn;
            }
    } else {
        // forward: zero-carry pass, then the carry entering this chunk
        double gp = 0.0, pf = 1.0;
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < Cs) {
                gp = Fb[t] * x[t] - Fa[t] * gp;
                pf *= -Fa[t];
            }
        fend[w * 64 + lane] = gp;
        if (lane == 0) pif[w] = pf;
        __syncthreads();
        double gin = 0.0;
        for (int s2 = 0; s2 < s; ++s2) gin = fend[(r * kc + s2) * 64 + lane] + pif[r * kc + s2] * gin;
        gp = gin;
        const cdouble *__restrict__ Fb2 = Fb + A.zero;   // reissue, do not keep pass-1 loads live
        const cdouble *__restrict__ Fa2 = Fa + A.zero;
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < Cs) {
                gp = Fb2[t] * x[t] - Fa2[t] * gp;
                x[t] = gp;
            }
        tip_last = gp;
        // backward: zero-carry pass, then the carry entering from the right
        double xn = 0.0, pb = 1.0;
#pragma unroll
        for (int t = CMAX - 1; t >= 0; --t)
            if (t < Cs) {
                xn = x[t] - Fc[t] * xn;
                pb *= -Fc[t];
            }
        bbeg[w * 64 + lane] = xn;
        if (lane == 0) pib[w] = pb;
        __syncthreads();
        double xin = 0.0;
        for (int s2 = kc - 1; s2 > s; --s2) xin = bbeg[(r * kc + s2) * 64 + lane] + pib[r * kc + s2] * xin;
        xn = xin;
        const cdouble *__restrict__ Fc2 = Fc + A.zero;
#pragma unroll
        for (int t = CMAX - 1; t >= 0; --t)
            if (t < Cs) {
                xn = x[t] - Fc2[t] * xn;
                x[t] = xn;
            }
    }

    // exchange the tips of the P partitions (the paper's SENDRECV / ALLGATHER)
    if (s == 0) tips[(2 * r) * 64 + lane] = x[0];
    if (s == kc - 1) tips[(2 * r + 1) * 64 + lane] = tip_last;
    __syncthreads();

    const cdouble *__restrict__ it = (const cdouble *)(A.IT + ((g * P + r) * 2) * (2 * P));
    double yl, yr;
    interface_unknowns<METHOD>(it, r, P, A.periodic,
                               [&](int q) { return tips[q * 64 + lane]; }, yl, yr);

    // Eq. (8) / (11): x = x~ - y_left v^(r) - y_right w^(r).  Every row is
    // corrected before the first store, so the spike values are read with
    // scalar loads (a load after a store to the field could not be).
#pragma unroll
    for (int t = 0; t < CMAX; ++t)
        if (t < Cs) x[t] = x[t] - yl * Fv[t] - yr * Fw[t];
    if (active && ACC) {
        // add the solution to the accumulation target (its own layout)
        const int64_t aj = A.a_j;
        gdouble *__restrict__ q = (gdouble *)(A.acc + b0 * A.a_b0 + b1 * A.a_b1 + row0 * aj);
        double z[CMAX];
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < Cs) z[t] = __builtin_nontemporal_load(q + t * aj);
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < Cs) __builtin_nontemporal_store(z[t] + x[t], q + t * aj);
    } else if (active) {
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < Cs) __builtin_nontemporal_store(x[t], p + t * sj);
    }
}

template <int CMAX, int METHOD, bool CHUNKED, bool ACC = false>
__global__ void __launch_bounds__(CMAX > 40 ? 512 : 1024) k_strided(const SolveArgs A)
{
    extern __shared__ double lds[];
    strided_solve<CMAX, METHOD, CHUNKED, ACC>(A, blockIdx.x, lds, (int)threadIdx.x);
}

// ===========================================================================
// Strided solve with two neighbouring lines per lane: every row access of a
// wavefront is one 1-KB segment of 16-byte lane accesses (the strided
// kernel's 512-B segments of 8-byte accesses move less per request when rows
// are far apart, as in the spanwise direction), and each lane runs the two
// lines' recurrences side by side on the same wavefront-uniform factors.
// One wavefront per partition (kc = 1), rows kept in VGPRs load -> store.
// ===========================================================================
// ACC: the solutions are added to A.acc in its own layout (a_b0 = 1, pairs
// 16-byte aligned) instead of being stored over d, a few rows at a time so
// that the added rows need few registers.
template <int CMAX, int METHOD, bool ACC = false>
__device__ __forceinline__ void strided2_solve(const SolveArgs &A, int64_t blk, double *lds, int tid,
                                               bool ghost = false)
{
    const int lane = tid & 63;
    const int r = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int P = A.P, m = A.m;
    double *tips = lds;                                     // [2P][128]
    int64_t grp, b1;
    strided_block(A, blk, grp, b1);
    const int64_t b0 = grp * 128 + 2 * lane;
    const bool act0 = !ghost && b0 < A.nb0, act1 = !ghost && b0 + 1 < A.nb0;
    const int64_t n = A.n;
    const int64_t g = b1 * A.g_b1 + A.g_off;
    const int64_t row0 = (int64_t)r * m;
    const cdouble *__restrict__ F = (const cdouble *)(A.F + g * (kNumFactors * n) + row0);
    const cdouble *__restrict__ Fb = F;
    const cdouble *__restrict__ Fa = F + n;
    const cdouble *__restrict__ Fc = F + 2 * n;
    const cdouble *__restrict__ Fv = F + 3 * n;
    const cdouble *__restrict__ Fw = F + 4 * n;
    const int64_t sj = A.s_j;
    gdouble *__restrict__ p = (gdouble *)(A.d + (act0 ? b0 : 0) + b1 * A.s_b1 + row0 * sj);

    double x0[CMAX], x1[CMAX];
#pragma unroll
    for (int t = 0; t < CMAX; ++t) {
        x0[t] = 0.0;
        x1[t] = 0.0;
        if (t < m) {
            if (act1) {
                const v2d v = __builtin_nontemporal_load((const __attribute__((address_space(1))) v2d *)(p + t * sj));
                x0[t] = v.x;
                x1[t] = v.y;
            } else if (act0) {
                x0[t] = __builtin_nontemporal_load(p + t * sj);
            }
        }
    }
    if (r == 0 && (((const cint *)A.flags)[g] & 1)) {
        x0[0] = 0.0;
        x1[0] = 0.0;
    }
    // Eq. (5) for both lines with the shared pivots
    double g0 = 0.0, g1 = 0.0;
#pragma unroll
    for (int t = 0; t < CMAX; ++t)
        if (t < m) {
            g0 = Fb[t] * x0[t] - Fa[t] * g0;
            g1 = Fb[t] * x1[t] - Fa[t] * g1;
            x0[t] = g0;
            x1[t] = g1;
        }
    const double l0 = g0, l1 = g1;
    double n0 = 0.0, n1 = 0.0;
#pragma unroll
    for (int t = CMAX - 1; t >= 0; --t)
        if (t < m) {
            n0 = x0[t] - Fc[t] * n0;
            n1 = x1[t] - Fc[t] * n1;
            x0[t] = n0;
            x1[t] = n1;
        }
    tips[(2 * r) * 128 + 2 * lane] = x0[0];
    tips[(2 * r) * 128 + 2 * lane + 1] = x1[0];
    tips[(2 * r + 1) * 128 + 2 * lane] = l0;
    tips[(2 * r + 1) * 128 + 2 * lane + 1] = l1;
    __syncthreads();
    const cdouble *__restrict__ it = (const cdouble *)(A.IT + ((g * P + r) * 2) * (2 * P));
    double yl0, yr0, yl1, yr1;
    interface_unknowns<METHOD>(it, r, P, A.periodic, [&](int q) { return tips[q * 128 + 2 * lane]; }, yl0, yr0);
    interface_unknowns<METHOD>(it, r, P, A.periodic, [&](int q) { return tips[q * 128 + 2 * lane + 1]; }, yl1, yr1);
    // Eq. (8) / (11), every row corrected before the first store
#pragma unroll
    for (int t = 0; t < CMAX; ++t)
        if (t < m) {
            x0[t] = x0[t] - yl0 * Fv[t] - yr0 * Fw[t];
            x1[t] = x1[t] - yl1 * Fv[t] - yr1 * Fw[t];
        }
    if (ACC) {
        constexpr int B = 6;
        const int64_t aj = A.a_j;
        gdouble *__restrict__ q = (gdouble *)(A.acc + (act0 ? b0 : 0) + b1 * A.a_b1 + row0 * aj);
#pragma unroll
        for (int t0 = 0; t0 < CMAX; t0 += B) {
            v2d z[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int t = t0 + u;
                z[u] = v2d{0.0, 0.0};
                if (t < CMAX && t < m) {
                    if (act1) z[u] = __builtin_nontemporal_load((const gv2d *)(q + t * aj));
                    else if (act0) z[u].x = __builtin_nontemporal_load(q + t * aj);
                }
            }
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int t = t0 + u;
                if (t < CMAX && t < m) {
                    if (act1) {
                        v2d v;
                        v.x = z[u].x + x0[t];
                        v.y = z[u].y + x1[t];
                        __builtin_nontemporal_store(v, (gv2d *)(q + t * aj));
                    } else if (act0) {
                        __builtin_nontemporal_store(z[u].x + x0[t], q + t * aj);
                    }
                }
            }
        }
        return;
    }
#pragma unroll
    for (int t = 0; t < CMAX; ++t)
        if (t < m) {
            if (act1) {
                v2d v;
                v.x = x0[t];
                v.y = x1[t];
                __builtin_nontemporal_store(v, (__attribute__((address_space(1))) v2d *)(p + t * sj));
            } else if (act0) {
                __builtin_nontemporal_store(x0[t], p + t * sj);
            }
        }
}

template <int CMAX, int METHOD, bool ACC = false>
__global__ void __launch_bounds__(1024) k_strided2(const SolveArgs A)
{
    extern __shared__ double lds[];
    strided2_solve<CMAX, METHOD, ACC>(A, blockIdx.x, lds, (int)threadIdx.x);
}

bool strided2_acc_supported(int method, int chunk_max) { return method == TRI_PDD && chunk_max == 24; }

hipError_t launch_strided2(const SolveArgs &a, int method, int chunk_max, hipStream_t s)
{
    const int64_t blocks = a.ngroups0 * a.nb1;
    const size_t lds = sizeof(double) * 2 * (size_t)a.P * 128;
    const dim3 grid((unsigned)blocks), block(64 * a.P);
    const bool pdd = method == TRI_PDD;
    if (a.acc) {
        // accumulating instances: PDD, 24 rows (the spanwise lines at P = 16)
        if (!strided2_acc_supported(method, chunk_max)) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_strided2<24, TRI_PDD, true>), grid, block, lds, s, a);
        return hipGetLastError();
    }
    switch (chunk_max) {
    case 8:
        if (pdd) hipLaunchKernelGGL((k_strided2<8, TRI_PDD>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_strided2<8, TRI_PPT>), grid, block, lds, s, a);
        break;
    case 16:
        if (pdd) hipLaunchKernelGGL((k_strided2<16, TRI_PDD>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_strided2<16, TRI_PPT>), grid, block, lds, s, a);
        break;
    case 24:
        if (pdd) hipLaunchKernelGGL((k_strided2<24, TRI_PDD>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_strided2<24, TRI_PPT>), grid, block, lds, s, a);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// ===========================================================================
// Ragged batch of strided solves in one launch.  Each entry of the device
// table is a complete strided problem (its own line length, strides,
// partition count, factor tables); workgroup b runs block b - begin of the
// entry whose block range holds b.  A batch only joins problems that the
// single-problem launch would run with this very instance (same CMAX,
// method, chunking and P * kc), so batching never changes a problem's
// arithmetic or launch shape.  The entries must not overlap in memory.
// ===========================================================================
template <int CMAX, int METHOD, bool CHUNKED>
__global__ void __launch_bounds__(CMAX > 40 ? 512 : 1024) k_strided_batch(const BatchEntry *__restrict__ E, int count)
{
    extern __shared__ double lds[];
    const int64_t b = blockIdx.x;
    int i = 0;
    while (i + 1 < count && E[i + 1].begin <= b) ++i;
    strided_solve<CMAX, METHOD, CHUNKED>(E[i].a, b - E[i].begin, lds, (int)threadIdx.x);
}

template <int CMAX, int METHOD>
static void launch_batch_t(const BatchEntry *e, int count, dim3 grid, dim3 block, size_t lds, bool chunked,
                           hipStream_t s)
{
    if (chunked) hipLaunchKernelGGL((k_strided_batch<CMAX, METHOD, true>), grid, block, lds, s, e, count);
    else hipLaunchKernelGGL((k_strided_batch<CMAX, METHOD, false>), grid, block, lds, s, e, count);
}

template <int METHOD>
static hipError_t launch_batch_m(const BatchEntry *e, int count, dim3 grid, dim3 block, size_t lds, int cmax,
                                 bool chunked, hipStream_t s)
{
    switch (cmax) {
    case 8: launch_batch_t<8, METHOD>(e, count, grid, block, lds, chunked, s); break;
    case 16: launch_batch_t<16, METHOD>(e, count, grid, block, lds, chunked, s); break;
    case 24: launch_batch_t<24, METHOD>(e, count, grid, block, lds, chunked, s); break;
    case 32: launch_batch_t<32, METHOD>(e, count, grid, block, lds, chunked, s); break;
    case 40: launch_batch_t<40, METHOD>(e, count, grid, block, lds, chunked, s); break;
    case 48: launch_batch_t<48, METHOD>(e, count, grid, block, lds, chunked, s); break;
    case 56: launch_batch_t<56, METHOD>(e, count, grid, block, lds, chunked, s); break;
    case 64: launch_batch_t<64, METHOD>(e, count, grid, block, lds, chunked, s); break;
    case 72: launch_batch_t<72, METHOD>(e, count, grid, block, lds, chunked, s); break;
    case 80: launch_batch_t<80, METHOD>(e, count, grid, block, lds, chunked, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_strided_batch(const BatchEntry *entries, int count, int64_t blocks, int wavefronts, int cmax,
                                int method, bool chunked, size_t lds, hipStream_t s)
{
    if (blocks <= 0) return hipSuccess;
    const dim3 grid((unsigned)blocks), block(64 * wavefronts);
    return method == TRI_PDD ? launch_batch_m<TRI_PDD>(entries, count, grid, block, lds, cmax, chunked, s)
                             : launch_batch_m<TRI_PPT>(entries, count, grid, block, lds, cmax, chunked, s);
}

size_t strided_lds_bytes(const SolveArgs &a)
{
    const int nw = a.P * a.kc;
    return sizeof(double) * ((size_t)(2 * a.P + 2 * nw) * 64 + 2 * nw);
}

template <int CMAX, int METHOD>
static hipError_t launch_strided_t(const SolveArgs &a, hipStream_t s)
{
    const int64_t blocks = a.ngroups0 * a.nb1;
    if (a.kc > 1)
        hipLaunchKernelGGL((k_strided<CMAX, METHOD, true>), dim3((unsigned)blocks), dim3(64 * a.P * a.kc),
                           strided_lds_bytes(a), s, a);
    else
        hipLaunchKernelGGL((k_strided<CMAX, METHOD, false>), dim3((unsigned)blocks), dim3(64 * a.P),
                           strided_lds_bytes(a), s, a);
    return hipGetLastError();
}

template <int METHOD>
static hipError_t launch_strided_m(const SolveArgs &a, int cmax, hipStream_t s)
{
    switch (cmax) {
    case 8: return launch_strided_t<8, METHOD>(a, s);
    case 16: return launch_strided_t<16, METHOD>(a, s);
    case 24: return launch_strided_t<24, METHOD>(a, s);
    case 32: return launch_strided_t<32, METHOD>(a, s);
    case 40: return launch_strided_t<40, METHOD>(a, s);
    case 48: return launch_strided_t<48, METHOD>(a, s);
    case 56: return launch_strided_t<56, METHOD>(a, s);
    case 64: return launch_strided_t<64, METHOD>(a, s);
    case 72: return launch_strided_t<72, METHOD>(a, s);
    case 80: return launch_strided_t<80, METHOD>(a, s);
    default: return hipErrorInvalidValue;
    }
}

// Accumulating instances (PDD, one line per lane, at most 24 rows a chunk):
// x is added to a.acc in its own layout instead of being stored over a.d.
// (With two lines per lane the added rows would not fit in registers.)
template <int CMAX>
static hipError_t launch_strided_acc_t(const SolveArgs &a, hipStream_t s)
{
    const int64_t blocks = a.ngroups0 * a.nb1;
    if (a.kc > 1)
        hipLaunchKernelGGL((k_strided<CMAX, TRI_PDD, true, true>), dim3((unsigned)blocks), dim3(64 * a.P * a.kc),
                           strided_lds_bytes(a), s, a);
    else
        hipLaunchKernelGGL((k_strided<CMAX, TRI_PDD, false, true>), dim3((unsigned)blocks), dim3(64 * a.P),
                           strided_lds_bytes(a), s, a);
    return hipGetLastError();
}

bool strided_acc_supported(int method, int chunk_max)
{
    return method == TRI_PDD && (chunk_max == 8 || chunk_max == 16 || chunk_max == 24);
}

hipError_t launch_strided(const SolveArgs &a, int method, int chunk_max, hipStream_t s)
{
    if (a.acc) {
        if (!strided_acc_supported(method, chunk_max)) return hipErrorInvalidValue;
        switch (chunk_max) {
        case 8: return launch_strided_acc_t<8>(a, s);
        case 16: return launch_strided_acc_t<16>(a, s);
        default: return launch_strided_acc_t<24>(a, s);
        }
    }
    return method == TRI_PDD ? launch_strided_m<TRI_PDD>(a, chunk_max, s)
                             : launch_strided_m<TRI_PPT>(a, chunk_max, s);
}

// ===========================================================================
// Contiguous-direction solve (rows contiguous, s_j = 1).
// A partition of m rows is spread over Lp lanes (Lp a power of two dividing
// 64) of C consecutive rows each.  The forward and backward Thomas sweeps of
// the partition are affine first-order recurrences, so each lane runs its C
// rows with a zero carry, the carries are combined by a segmented
// Kogge-Stone scan over the Lp lanes with cross-lane shuffles, and each lane
// re-runs its rows with the true carry.  The result is the partition's
// Thomas solution; the tips go through LDS to the other partitions.
// ===========================================================================
template <int CMAX, int METHOD>
__device__ __forceinline__ void contig_solve(const SolveArgs &A, int64_t blk, double *lds, int tid)
{
    // lds: [LPB][2P] tips
    const int LL = A.LL, Lp = A.Lp, C = A.C, m = A.m, P = A.P;
    const int li = tid / LL;
    const int lt = tid - li * LL;
    const int r = lt / Lp;
    const int k = lt - r * Lp;
    const bool inblk = li < A.LPB;
    const int64_t L = blk * A.LPB + li;
    const bool active = inblk && L < A.nlines;
    const int64_t b0 = active ? L % A.nb0 : 0;
    const int64_t b1 = active ? L / A.nb0 : 0;
    const int64_t g = b1 * A.g_b1 + A.g_off;
    const int64_t n = A.n;
    const int row0 = k * C;
    const int64_t J0 = (int64_t)(inblk ? r : 0) * m + row0;
    const double *__restrict__ F = A.F + g * (kNumFactors * n) + J0;
    double *__restrict__ p = A.d + b0 * A.s_b0 + b1 * A.s_b1 + J0;

    double x[CMAX], fb[CMAX], fa[CMAX], fc[CMAX];
#pragma unroll
    for (int t = 0; t < CMAX; ++t) {
        const bool valid = inblk && (t < C) && (row0 + t < m);
        x[t] = (valid && active) ? p[t] : 0.0;
        fb[t] = valid ? F[t] : 0.0;
        fa[t] = valid ? F[n + t] : 0.0;
        fc[t] = valid ? F[2 * n + t] : 0.0;
    }
    if (active && r == 0 && k == 0 && (A.flags[g] & 1)) x[0] = 0.0;

    // forward sweep, zero carry: chunk map g_out = Fs + Ps * g_in
    double gp = 0.0, ps = 1.0;
#pragma unroll
    for (int t = 0; t < CMAX; ++t)
        if (t < C) {
            gp = fb[t] * x[t] - fa[t] * gp;
            ps *= -fa[t];
        }
    double Fs = gp, Ps = ps;
    for (int s = 1; s < Lp; s <<= 1) {
        const double Fo = __shfl_up(Fs, s, Lp);
        const double Po = __shfl_up(Ps, s, Lp);
        if (k >= s) {
            Fs = Fs + Ps * Fo;
            Ps = Ps * Po;
        }
    }
    double gin = __shfl_up(Fs, 1, Lp);
    if (k == 0) gin = 0.0;
    gp = gin;
#pragma unroll
    for (int t = 0; t < CMAX; ++t)
        if (t < C) {
            gp = fb[t] * x[t] - fa[t] * gp;
            x[t] = gp;
        }
    const int kl = (m - 1) / C, tl = (m - 1) - kl * C;
    double tip_last = 0.0;
#pragma unroll
    for (int t = 0; t < CMAX; ++t)
        if (t == tl) tip_last = x[t];

    // backward sweep, zero carry: chunk map x_first = Bs + Ss * x_after
    double xn = 0.0, ss = 1.0;
#pragma unroll
    for (int t = CMAX - 1; t >= 0; --t)
        if (t < C) {
            xn = x[t] - fc[t] * xn;
            ss *= -fc[t];
        }
    double Bs = xn, Ss = ss;
    for (int s = 1; s < Lp; s <<= 1) {
        const double Bo = __shfl_down(Bs, s, Lp);
        const double So = __shfl_down(Ss, s, Lp);
        if (k + s < Lp) {
            Bs = Bs + Ss * Bo;
            Ss = Ss * So;
        }
    }
    double xin = __shfl_down(Bs, 1, Lp);
    if (k == Lp - 1) xin = 0.0;
    xn = xin;
#pragma unroll
    for (int t = CMAX - 1; t >= 0; --t)
        if (t < C) {
            xn = x[t] - fc[t] * xn;
            x[t] = xn;
        }

    double *tips = lds + (inblk ? li : 0) * 2 * P;
    if (inblk && k == 0) tips[2 * r] = x[0];
    if (inblk && k == kl) tips[2 * r + 1] = tip_last;
    __syncthreads();

    const double *__restrict__ it = A.IT + ((g * P + r) * 2) * (2 * P);
    double yl = 0.0, yr = 0.0;
    if (inblk)
        interface_unknowns<METHOD>(it, r, P, A.periodic, [&](int q) { return tips[q]; }, yl, yr);

    if (active) {
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < C && row0 + t < m) p[t] = x[t] - yl * F[3 * n + t] - yr * F[4 * n + t];
    }
}

template <int CMAX, int METHOD>
__global__ void __launch_bounds__(CMAX > 8 ? 256 : 1024) k_contig(const SolveArgs A)
{
    extern __shared__ double lds[];
    contig_solve<CMAX, METHOD>(A, blockIdx.x, lds, (int)threadIdx.x);
}

template <int CMAX, int METHOD>
static hipError_t launch_contig_t(const SolveArgs &a, hipStream_t s)
{
    const int64_t blocks = (a.nlines + a.LPB - 1) / a.LPB;
    int threads = a.LPB * a.LL;
    threads = ((threads + 63) / 64) * 64;
    const size_t lds = sizeof(double) * 2 * a.P * a.LPB;
    hipLaunchKernelGGL((k_contig<CMAX, METHOD>), dim3((unsigned)blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_contig(const SolveArgs &a, int method, hipStream_t s)
{
    if (a.C <= 4)
        return method == TRI_PDD ? launch_contig_t<4, TRI_PDD>(a, s) : launch_contig_t<4, TRI_PPT>(a, s);
    if (a.C <= 8)
        return method == TRI_PDD ? launch_contig_t<8, TRI_PDD>(a, s) : launch_contig_t<8, TRI_PPT>(a, s);
    if (a.C <= 16)
        return method == TRI_PDD ? launch_contig_t<16, TRI_PDD>(a, s) : launch_contig_t<16, TRI_PPT>(a, s);
    return hipErrorInvalidValue;
}

// ===========================================================================
// A dependency level in one launch: the strided solves (one or two lines per
// lane, any partition count and chunking of at most 8 wavefronts, chunks of
// at most 40 rows) and the contiguous solves (the register-factor body with
// 4 rows per lane, a run of consecutive lines per block; else the plain body
// with at most 8 rows per lane) of a ragged batch run side by side in
// 512-lane workgroups, at most 128 VGPRs (two workgroups a CU).  Each workgroup holds blocks of one entry only --
// 8 / wpb of them, each with its own LDS region -- so every wavefront of the
// workgroup takes the same branch and meets the same barriers; blocks past
// the entry's end (and the waves left over when wpb does not divide 8) run
// as ghosts.  The arithmetic of every line is that of the entry's own kernel.
// ===========================================================================
template <int METHOD>
__device__ __forceinline__ void level_strided(const LevelEntry &e, int64_t blk, double *l, int tid, bool ghost)
{
    if (e.chunked) {
        switch (e.cmax) {
        case 8: strided_solve<8, METHOD, true>(e.a, blk, l, tid, ghost); break;
        case 16: strided_solve<16, METHOD, true>(e.a, blk, l, tid, ghost); break;
        case 24: strided_solve<24, METHOD, true>(e.a, blk, l, tid, ghost); break;
        case 32: strided_solve<32, METHOD, true>(e.a, blk, l, tid, ghost); break;
        default: strided_solve<40, METHOD, true>(e.a, blk, l, tid, ghost); break;
        }
    } else {
        switch (e.cmax) {
        case 8: strided_solve<8, METHOD, false>(e.a, blk, l, tid, ghost); break;
        case 16: strided_solve<16, METHOD, false>(e.a, blk, l, tid, ghost); break;
        case 24: strided_solve<24, METHOD, false>(e.a, blk, l, tid, ghost); break;
        case 32: strided_solve<32, METHOD, false>(e.a, blk, l, tid, ghost); break;
        default: strided_solve<40, METHOD, false>(e.a, blk, l, tid, ghost); break;
        }
    }
}

template <int METHOD>
__device__ __forceinline__ void level_body(const LevelEntry &e, int64_t blk, double *l, int tid, bool ghost)
{
    if (e.body == kLevelStrided) {
        level_strided<METHOD>(e, blk, l, tid, ghost);
    } else if (e.body == kLevelStrided2) {
        switch (e.cmax) {
        case 8: strided2_solve<8, METHOD>(e.a, blk, l, tid, ghost); break;
        case 16: strided2_solve<16, METHOD>(e.a, blk, l, tid, ghost); break;
        default: strided2_solve<24, METHOD>(e.a, blk, l, tid, ghost); break;
        }
    } else if (e.body == kLevelContigReg) {
        contig_reg_solve<4, METHOD, true>(e.a, ghost ? e.a.nlines : blk * e.lines, 1, e.lines, tid, l);
    } else {
        if (e.cmax <= 4) contig_solve<4, METHOD>(e.a, blk, l, tid);
        else contig_solve<8, METHOD>(e.a, blk, l, tid);
    }
}

__global__ void __launch_bounds__(kLevelThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_level(const LevelEntry *__restrict__ E, int count)
{
    extern __shared__ double lds[];
    const int64_t wg = blockIdx.x;
    int i = 0;
    while (i + 1 < count && E[i + 1].begin <= wg) ++i;
    const LevelEntry &e = E[i];
    const int nt = 64 * e.wpb;
    const int sb = __builtin_amdgcn_readfirstlane((int)threadIdx.x / nt);   // block within the workgroup
    const int tid = (int)threadIdx.x - sb * nt;
    int64_t blk = (wg - e.begin) * e.sub + sb;
    const bool ghost = sb >= e.sub || blk >= e.nblocks;
    if (ghost) blk = 0;
    double *l = lds + (int64_t)sb * e.lds_sub;
    if (e.method == TRI_PDD) level_body<TRI_PDD>(e, blk, l, tid, ghost);
    else level_body<TRI_PPT>(e, blk, l, tid, ghost);
}

hipError_t launch_level(const LevelEntry *entries, int count, int64_t blocks, size_t lds, hipStream_t s)
{
    if (blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_level, dim3((unsigned)blocks), dim3(kLevelThreads), lds, s, entries, count);
    return hipGetLastError();
}

// ===========================================================================
// Persistent contiguous-direction solve with LDS staging (one shared matrix).
// Same algebra as k_contig, rearranged for bandwidth:
//  * one large workgroup per CU loops over groups of LPB lines; the factors
//    and spikes of the (single, shared) matrix sit in LDS once, per lane
//    position in a line ([lane][factor][row], odd stride against bank
//    conflicts, compile-time offsets), read by every line of the group, and
//    the line-independent multipliers of the carry scans are formed once;
//  * lines move between HBM and LDS with coalesced 16-byte accesses (each
//    wavefront instruction covers 1 KB of a line); a lane then reads its C
//    consecutive rows from padded staging planes (conflict-free);
//  * the next group's loads are issued into VGPRs before the current group
//    is solved, so HBM always has a group in flight per workgroup.
// Requires m % C == 0, C even, n even and 16-byte aligned lines.
// ===========================================================================
template <int CMAX, int METHOD>
__global__ void __launch_bounds__(1024) k_contig_staged(const SolveArgs A)
{
    extern __shared__ double lds[];
    constexpr int QMAX = CMAX / 2;
    const int tid = threadIdx.x;
    const int NTH = blockDim.x;
    const int LL = A.LL, Lp = A.Lp, C = A.C, m = A.m, P = A.P, LPB = A.LPB;
    const int S = A.stage_stride;
    const int NQ = C / 2;
    const int NT = LPB * LL;
    constexpr int FS = 5 * CMAX + 1;             // per-lane factor stride (odd)
    double *stage = lds;                         // [NQ][S]
    double *fac = lds + (size_t)NQ * S;          // [LL][5][CMAX] (+1 pad)
    double *tips = fac + (size_t)FS * LL;        // [LPB][2P]
    const int li = tid / LL;
    const int lt = tid - li * LL;
    const int r = lt / Lp;
    const int k = lt - r * Lp;
    const bool inblk = li < LPB;
    const int64_t n = A.n;
    const int UPL = (int)(n / 2);

    // the shared matrix's factors and spikes, once per workgroup
    for (int idx = tid; idx < 5 * C * LL; idx += NTH) {
        const int l2 = idx / (5 * C), rem = idx - l2 * (5 * C);
        const int f = rem / C, c = rem - f * C;
        const int r2 = l2 / Lp, k2 = l2 - r2 * Lp;
        fac[l2 * FS + f * CMAX + c] = A.F[f * n + (int64_t)r2 * m + (int64_t)k2 * C + c];
    }
    // multipliers of the partner's carry at each Kogge-Stone step
    constexpr int kSteps = 6;
    double psk[kSteps], ssk[kSteps];
    {
        const int64_t J0 = (int64_t)(inblk ? r : 0) * m + (int64_t)k * C;
        double Ps = 1.0, Ss = 1.0;
#pragma unroll
        for (int c = 0; c < CMAX; ++c)
            if (c < C && inblk) {
                Ps *= -A.F[n + J0 + c];
                Ss *= -A.F[2 * n + J0 + c];
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
    // this thread's share of the coalesced line <-> LDS copies
    int soff[QMAX], srow[QMAX], sline[QMAX];
#pragma unroll
    for (int it = 0; it < QMAX; ++it) {
        const int g = tid + it * NTH;
        soff[it] = -1;
        srow[it] = 0;
        sline[it] = 0;
        if (it < NQ && g < NT * NQ) {
            const int l2 = g / UPL, w = g - l2 * UPL;
            const int row = 2 * w;
            const int r2 = row / m, rr = row - r2 * m;
            const int k2 = rr / C, c2 = rr - k2 * C;
            const int owner = l2 * LL + r2 * Lp + k2;
            soff[it] = (c2 / 2) * S + owner * 2;
            srow[it] = row;
            sline[it] = l2;
        }
    }
    auto line_ptr = [&](int64_t L) -> double * {
        if (A.lines_linear) return A.d + L * A.s_b0;
        const int64_t b0 = L % A.nb0, b1 = L / A.nb0;
        return A.d + b0 * A.s_b0 + b1 * A.s_b1;
    };
    const double *__restrict__ it_rows = A.IT + ((int64_t)r * 2) * (2 * P);
    const bool pinned = (A.flags[0] & 1) && r == 0 && k == 0;
    double *mytips = tips + (inblk ? li : 0) * 2 * P;
    const int64_t ngrp = (A.nlines + LPB - 1) / LPB;

    v2d pre[QMAX];
    auto prefetch = [&](int64_t grp) {
#pragma unroll
        for (int it = 0; it < QMAX; ++it)
            if (soff[it] >= 0 && grp * LPB + sline[it] < A.nlines)
                pre[it] = __builtin_nontemporal_load((const v2d *)(line_ptr(grp * LPB + sline[it]) + srow[it]));
    };
    if (blockIdx.x < ngrp) prefetch(blockIdx.x);
    __syncthreads();   // factor table complete

    for (int64_t grp = blockIdx.x; grp < ngrp; grp += gridDim.x) {
        const int64_t Lbase = grp * LPB;
#pragma unroll
        for (int it = 0; it < QMAX; ++it)
            if (soff[it] >= 0 && Lbase + sline[it] < A.nlines) *(v2d *)(stage + soff[it]) = pre[it];
        __syncthreads();
        if (grp + gridDim.x < ngrp) prefetch(grp + gridDim.x);

        double x[CMAX];
#pragma unroll
        for (int c = 0; c < CMAX; ++c)
            x[c] = (c < C && inblk) ? stage[(c >> 1) * S + tid * 2 + (c & 1)] : 0.0;
        if (pinned) x[0] = 0.0;
        const double *myfac = fac + lt * FS;
        auto F = [&](int f, int c) { return myfac[f * CMAX + c]; };

        // forward sweep: zero-carry pass, carry scan, exact pass
        double gp = 0.0;
#pragma unroll
        for (int c = 0; c < CMAX; ++c)
            if (c < C) gp = F(0, c) * x[c] - F(1, c) * gp;
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
        for (int c = 0; c < CMAX; ++c)
            if (c < C) {
                gp = F(0, c) * x[c] - F(1, c) * gp;
                x[c] = gp;
            }
        const double tip_last = gp;

        // backward sweep
        double xn = 0.0;
#pragma unroll
        for (int c = CMAX - 1; c >= 0; --c)
            if (c < C) xn = x[c] - F(2, c) * xn;
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
        for (int c = CMAX - 1; c >= 0; --c)
            if (c < C) {
                xn = x[c] - F(2, c) * xn;
                x[c] = xn;
            }

        if (inblk && k == 0) mytips[2 * r] = x[0];
        if (inblk && k == Lp - 1) mytips[2 * r + 1] = tip_last;
        __syncthreads();
        double yl = 0.0, yr = 0.0;
        if (inblk)
            interface_unknowns<METHOD>(it_rows, r, P, A.periodic, [&](int q) { return mytips[q]; }, yl, yr);
        if (inblk) {
#pragma unroll
            for (int c = 0; c < CMAX; ++c)
                if (c < C) stage[(c >> 1) * S + tid * 2 + (c & 1)] = x[c] - yl * F(3, c) - yr * F(4, c);
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < QMAX; ++it)
            if (soff[it] >= 0 && Lbase + sline[it] < A.nlines)
                __builtin_nontemporal_store(*(const v2d *)(stage + soff[it]),
                                            (v2d *)(line_ptr(Lbase + sline[it]) + srow[it]));
        __syncthreads();
    }
}

size_t contig_staged_lds_bytes(const SolveArgs &a)
{
    const int cmax = a.C <= 4 ? 4 : (a.C <= 8 ? 8 : 16);
    return sizeof(double) * ((size_t)(a.C / 2) * a.stage_stride + (size_t)(5 * cmax + 1) * a.LL +
                             (size_t)a.LPB * 2 * a.P);
}

template <int CMAX, int METHOD>
static hipError_t launch_contig_staged_t(const SolveArgs &a, int grid, hipStream_t s)
{
    int threads = a.LPB * a.LL;
    threads = ((threads + 63) / 64) * 64;
    const size_t lds = contig_staged_lds_bytes(a);
    const int64_t ngrp = (a.nlines + a.LPB - 1) / a.LPB;
    const int64_t blocks = std::min<int64_t>(std::max(grid, 1), ngrp);
    hipLaunchKernelGGL((k_contig_staged<CMAX, METHOD>), dim3((unsigned)blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <int CMAX, int METHOD>
static int staged_grid_t(const SolveArgs &a)
{
    int threads = ((a.LPB * a.LL + 63) / 64) * 64;
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(&k_contig_staged<CMAX, METHOD>), threads,
            contig_staged_lds_bytes(a)) != hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return std::max(1, per_cu) * cus;
}

int contig_staged_grid(const SolveArgs &a, int method)
{
    const bool pdd = method == TRI_PDD;
    if (a.C <= 4) return pdd ? staged_grid_t<4, TRI_PDD>(a) : staged_grid_t<4, TRI_PPT>(a);
    if (a.C <= 8) return pdd ? staged_grid_t<8, TRI_PDD>(a) : staged_grid_t<8, TRI_PPT>(a);
    return pdd ? staged_grid_t<16, TRI_PDD>(a) : staged_grid_t<16, TRI_PPT>(a);
}

hipError_t launch_contig_staged(const SolveArgs &a, int method, int grid, hipStream_t s)
{
    if (a.C <= 4)
        return method == TRI_PDD ? launch_contig_staged_t<4, TRI_PDD>(a, grid, s)
                                 : launch_contig_staged_t<4, TRI_PPT>(a, grid, s);
    if (a.C <= 8)
        return method == TRI_PDD ? launch_contig_staged_t<8, TRI_PDD>(a, grid, s)
                                 : launch_contig_staged_t<8, TRI_PPT>(a, grid, s);
    if (a.C <= 16)
        return method == TRI_PDD ? launch_contig_staged_t<16, TRI_PDD>(a, grid, s)
                                 : launch_contig_staged_t<16, TRI_PPT>(a, grid, s);
    return hipErrorInvalidValue;
}

// ===========================================================================
// General kernel: coefficients per line.  Same layout as the strided kernel
// (wavefront = partition, lane = line); every lane factors its own block,
// carrying the right-hand side and the a-corner spike through one forward
// elimination (the paper batches Eq. (6) with Eq. (5) the same way), and
// keeps x~, the forward-reduced spike and the pivots in VGPRs.  SHIFT: the
// shifted Poisson systems of GeneralArgs (coefficients formed on the fly from
// the shared ay, cy and the line's shift, never stored).
// ===========================================================================
template <int CMAX, int METHOD, bool SHIFT, int MAXT>
__global__ void __launch_bounds__(MAXT) k_general(const GeneralArgs A)
{
    // LW lines a workgroup: 64 (a wavefront per partition), or 32 for the
    // shifted systems (half a wavefront per partition), whose blocks fill up
    // to 252 VGPRs: two such workgroups share a CU, so one loads while the
    // other computes
    constexpr int LW = (SHIFT && MAXT == 512) ? 32 : 64;
    extern __shared__ double sh[];              // [6][P][LW]
    const int lane = threadIdx.x & (LW - 1);
    const int r = LW == 64 ? __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) : (int)(threadIdx.x / LW);
    const int64_t blk = blockIdx.x;
    const int64_t grp = blk % A.ngroups0;
    const int64_t b1 = blk / A.ngroups0;
    const int64_t b0raw = grp * LW + lane;
    const bool active = b0raw < A.nb0;
    const int64_t b0 = active ? b0raw : 0;
    const int m = A.m, P = A.P, periodic = A.periodic;
    const int64_t sj = A.s_j, csj = A.cs_j;
    double *__restrict__ p = A.d + b0 * A.s_b0 + b1 * A.s_b1 + (int64_t)r * m * sj;
    const int64_t cb = (b0 >> A.cplx) * A.cs_b0 + b1 * A.cs_b1 + (int64_t)r * m * csj;
    const double *__restrict__ ca = A.a + cb;
    const double *__restrict__ cbp = A.b + cb;
    const double *__restrict__ cc = A.c + cb;

    // row t of the block: (a_t, b_t, c_t)
    const double sigma = SHIFT ? A.lamz[b1] + A.lamx[b0 >> A.cplx] : 0.0;
    const bool pin = SHIFT && sigma == 0.0 && r == 0;     // global row 0 becomes x_0 = 0
    auto row_c = [&](int t) { return (pin && t == 0) ? 0.0 : cc[t * csj]; };
    auto row_b = [&](int t) {
        if (!SHIFT) return cbp[t * csj];
        return (pin && t == 0) ? 1.0 : -(ca[t * csj] + cc[t * csj]) - sigma;
    };

    double x[CMAX], gv[CMAX], cp[CMAX];
#pragma unroll
    for (int t = 0; t < CMAX; ++t) { x[t] = 0.0; gv[t] = 0.0; cp[t] = 0.0; }
    if (active) {
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < m) x[t] = p[t * sj];
    }
    if (pin) x[0] = 0.0;
    const double a_first = (r >= 1 || periodic) ? ca[0] : 0.0;
    const double c_last = (r <= P - 2 || periodic) ? row_c(m - 1) : 0.0;

    // Block elimination with diagonal pivoting (the local solver the PPT
    // paragraph of Sec. 3.2 names): at row t the pivot is the 1x1 entry d_t, or
    // the 2x2 block of rows t, t+1 when |d_t| sigma < kappa |a_{t+1} c_t|
    // (Bunch-Kaufman test as used for tridiagonal systems, sigma the largest
    // neighbouring entry, kappa = (sqrt 5 - 1)/2).  Every row ends as
    // x_t = p_t - q_t x_{t+link}: link 1, or 2 for the first row of a 2x2
    // block (bit t of `two`).  p for the right-hand side (x) and for the
    // a-corner spike (gv), q in cp.  Diagonally dominant rows always take the
    // 1x1 pivot (plain Thomas); the shifted Poisson rows are, so SHIFT
    // compiles the test out, and so does PDD (meant for dominant rows: on
    // others its truncation is inaccurate whatever the pivots).
    constexpr bool PIVOT = !SHIFT && METHOD == TRI_PPT;
    constexpr double kKappa = 0.61803398874989484820;
    uint64_t two = 0;
    double pq = 0.0, px = 0.0, pv = 0.0;       // q, p of the row before (link 1 to this row)
    double wl1 = 0.0, wl2 = 0.0;               // p of the c-corner spike at rows m-1, m-2
    bool bad = false, pend = false;
    double xl = 0.0, vm = 0.0, wm = 0.0, xf = 0.0, v0 = 0.0, w0 = 0.0;
    if constexpr (!PIVOT) {
        // 1x1 pivots only (plain Thomas), w from the product of the multipliers
        double cpp = 0.0, gx = 0.0, gvp = 0.0, beta_last = 0.0;
#pragma unroll
        for (int t = 0; t < CMAX; ++t)
            if (t < m) {
                const double aa = (t == 0) ? 0.0 : ca[t * csj];
                const double ccv = (t == m - 1) ? 0.0 : row_c(t);
                const double den = row_b(t) - aa * cpp;
                bad |= !(den != 0.0);
                // the shifted rows' pivots are far from the range ends: the
                // reciprocal estimate and two Newton steps (each r += r(1 - den r)
                // doubles the correct bits) replace the longer IEEE division
                double beta;
                if constexpr (SHIFT) {
                    beta = __builtin_amdgcn_rcp(den);
                    beta = fma(beta, fma(-den, beta, 1.0), beta);
                    beta = fma(beta, fma(-den, beta, 1.0), beta);
                } else {
                    beta = 1.0 / den;
                }
                gx = (x[t] - aa * gx) * beta;
                x[t] = gx;
                gvp = (t == 0) ? a_first * beta : -(aa * beta) * gvp;
                gv[t] = gvp;
                cpp = ccv * beta;
                cp[t] = cpp;
                beta_last = beta;
            }
        if (bad && active) atomicOr(A.status, kStatusZeroPivot);
        xl = gx, vm = gvp;
        double xn = 0.0, vn = 0.0, cprod = 1.0;
#pragma unroll
        for (int t = CMAX - 1; t >= 0; --t)
            if (t < m) {
                xn = x[t] - cp[t] * xn;
                x[t] = xn;
                vn = gv[t] - cp[t] * vn;
                if (t < m - 1) cprod *= -cp[t];
            }
        xf = x[0], v0 = vn;
        wm = beta_last * c_last, w0 = wm * cprod;
        wl1 = wm;
    } else {
#pragma unroll
    for (int t = 0; t < CMAX; ++t) {
        if (t >= m) continue;
        if (pend) {                            // second row of a 2x2 block, done with its first
            pend = false;
            continue;
        }
        const double at = (t == 0) ? 0.0 : ca[t * csj];
        const double ct = (t == m - 1) ? 0.0 : row_c(t);
        const double d = row_b(t) - at * pq;
        const double rx = x[t] - at * px;
        const double rv = ((t == 0) ? a_first : 0.0) - at * pv;
        bool use2 = false;
        double a1 = 0.0, b1 = 0.0, c1 = 0.0;
        if (PIVOT && t + 1 < CMAX && t + 1 < m) {
            a1 = ca[(t + 1) * csj];
            b1 = row_b(t + 1);
            c1 = (t + 1 == m - 1) ? 0.0 : row_c(t + 1);
            const double a2 = (t + 2 < m) ? ca[(t + 2) * csj] : 0.0;
            const double sg = fmax(fmax(fmax(fabs(ct), fabs(a1)), fmax(fabs(b1), fabs(c1))), fabs(a2));
            use2 = fabs(d) * sg < kKappa * fabs(a1 * ct);
        }
        if (!use2) {
            bad |= !(d != 0.0);
            const double beta = 1.0 / d;
            x[t] = rx * beta;
            gv[t] = rv * beta;
            cp[t] = ct * beta;
            pq = cp[t];
            px = x[t];
            pv = gv[t];
            if (t == m - 1) wl1 = c_last * beta;
        } else if (t + 1 < CMAX) {
            const double det = d * b1 - ct * a1;
            bad |= !(det != 0.0);
            const double idet = 1.0 / det;
            const double r1 = x[t + 1];        // row t+1's own right-hand side (the spike's is 0)
            x[t] = (b1 * rx - ct * r1) * idet;
            gv[t] = (b1 * rv) * idet;
            cp[t] = -(ct * c1) * idet;         // x_t couples to x_{t+2}
            x[t + 1] = (d * r1 - a1 * rx) * idet;
            gv[t + 1] = -(a1 * rv) * idet;
            cp[t + 1] = (d * c1) * idet;
            two |= 1ull << t;
            pq = cp[t + 1];
            px = x[t + 1];
            pv = gv[t + 1];
            if (t + 1 == m - 1) {
                wl2 = -(ct * c_last) * idet;
                wl1 = (d * c_last) * idet;
            }
            pend = true;
        }
    }
    if (bad && active) atomicOr(A.status, kStatusZeroPivot);
    if (A.piv && active) {
        unsigned char *pk = A.piv + (b1 * A.nb0 + b0) * A.n + (int64_t)r * m;
        for (int t = 0; t < m; ++t)
            pk[t] = ((two >> t) & 1) ? 2 : ((t > 0 && ((two >> (t - 1)) & 1)) ? 0 : 1);
    }
    // back substitution of x~, v (a-corner spike) and w (c-corner spike),
    // keeping the values of the two rows below
    double x1 = 0.0, x2 = 0.0, v1 = 0.0, v2 = 0.0, w1 = 0.0, w2 = 0.0;
#pragma unroll
    for (int t = CMAX - 1; t >= 0; --t)
        if (t < m) {
            const bool l2 = (two >> t) & 1;
            const double xt = x[t] - cp[t] * (l2 ? x2 : x1);
            const double vt = gv[t] - cp[t] * (l2 ? v2 : v1);
            const double pw = (t == m - 1) ? wl1 : ((t == m - 2) ? wl2 : 0.0);
            const double wt = pw - cp[t] * (l2 ? w2 : w1);
            x[t] = xt;
            x2 = x1, x1 = xt;
            v2 = v1, v1 = vt;
            w2 = w1, w1 = wt;
            if (t == m - 1) xl = xt, vm = vt, wm = wt;
        }
    xf = x1, v0 = v1, w0 = w1;
    }

    auto S = [&](int q, int part) -> double & { return sh[((int64_t)q * P + part) * LW + lane]; };
    S(0, r) = xf; S(1, r) = xl; S(2, r) = v0; S(3, r) = vm; S(4, r) = w0; S(5, r) = wm;
    __syncthreads();

    double yl = 0.0, yr = 0.0;
    const bool has_l = (r > 0) || periodic, has_r = (r < P - 1) || periodic;
    if (METHOD == TRI_PDD && A.pdd_tol > 0.0 && active) {
        // the entries PDD drops that this partition holds: v at its last row
        // (left side of the next interface), w at its first row (right side)
        const double d = fmax(has_l && has_r ? fabs(vm) : 0.0, has_l && has_r ? fabs(w0) : 0.0);
        if (d > A.pdd_tol) atomicOr(A.status, kStatusPddUnsafe);
    }
    if (METHOD == TRI_PDD) {
        if (has_l) {
            const int L = (r > 0) ? r - 1 : P - 1;
            const double det = 1.0 - S(5, L) * v0;
            yl = (S(1, L) - S(5, L) * xf) / det;
        }
        if (has_r) {
            const int R = (r < P - 1) ? r + 1 : 0;
            const double det = 1.0 - wm * S(2, R);
            yr = (S(0, R) - S(2, R) * xl) / det;
        }
    } else if constexpr (SHIFT && MAXT == 512) {
        // Shifted rows are diagonally dominant and never periodic, so the
        // reduced system needs no pivoting: it is solved by block cyclic
        // reduction over the P partitions, all wavefronts at once.  Partition
        // r's unknowns X_r = (x at its first row, x at its last row) satisfy
        //   X_r + L_r X_{r-1} + U_r X_{r+1} = (x~ first, x~ last),
        // L_r = [[0, v_1], [0, v_m]] on the left neighbour's last row and
        // U_r = [[w_1, 0], [w_m, 0]] on the right neighbour's first row (the
        // same equations as the rows of Z in Eq. (7), grouped by partition).
        // A step at distance h eliminates X_{r-h} and X_{r+h} with rows r-h and
        // r+h and rescales the row to a unit diagonal block; after the steps
        // h = 1, 2, 4, .. < P each row stands alone.  Dominance (|v| + |w| <= 1
        // row by row) carries through the steps.  Rows cross between
        // wavefronts through LDS (10 values a row, over the tips, which no
        // one reads on this path).  The rows stay in LDS between steps, since
        // the registers hold what the correction needs; a step reads this row
        // and the neighbours' blocks as it uses them and writes the new row
        // after a barrier.
        auto Q = [&](int q, int part) -> double & { return sh[((int64_t)q * P + part) * LW + lane]; };
        bool ok = true;
        Q(0, r) = 0.0; Q(1, r) = v0; Q(2, r) = 0.0; Q(3, r) = vm;      // L_r
        Q(4, r) = w0; Q(5, r) = 0.0; Q(6, r) = wm; Q(7, r) = 0.0;      // U_r
        Q(8, r) = xf; Q(9, r) = xl;                                    // right-hand side
        for (int h = 1; h < P; h *= 2) {
            __syncthreads();
            double d00 = 1.0, d01 = 0.0, d10 = 0.0, d11 = 1.0;
            double e0 = Q(8, r), e1 = Q(9, r);
            double n0 = 0.0, n1 = 0.0, n2 = 0.0, n3 = 0.0;       // -L_r L_{r-h}
            double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;       // -U_r U_{r+h}
            if (r - h >= 0) {
                const double l00 = Q(0, r), l01 = Q(1, r), l10 = Q(2, r), l11 = Q(3, r);
                const int q = r - h;
                const double t0 = Q(4, q), t1 = Q(5, q), t2 = Q(6, q), t3 = Q(7, q);
                d00 -= l00 * t0 + l01 * t2; d01 -= l00 * t1 + l01 * t3;
                d10 -= l10 * t0 + l11 * t2; d11 -= l10 * t1 + l11 * t3;
                const double s0 = Q(8, q), s1 = Q(9, q);
                e0 -= l00 * s0 + l01 * s1; e1 -= l10 * s0 + l11 * s1;
                const double k0 = Q(0, q), k1 = Q(1, q), k2 = Q(2, q), k3 = Q(3, q);
                n0 = -(l00 * k0 + l01 * k2); n1 = -(l00 * k1 + l01 * k3);
                n2 = -(l10 * k0 + l11 * k2); n3 = -(l10 * k1 + l11 * k3);
            }
            if (r + h < P) {
                const double u00 = Q(4, r), u01 = Q(5, r), u10 = Q(6, r), u11 = Q(7, r);
                const int q = r + h;
                const double t0 = Q(0, q), t1 = Q(1, q), t2 = Q(2, q), t3 = Q(3, q);
                d00 -= u00 * t0 + u01 * t2; d01 -= u00 * t1 + u01 * t3;
                d10 -= u10 * t0 + u11 * t2; d11 -= u10 * t1 + u11 * t3;
                const double s0 = Q(8, q), s1 = Q(9, q);
                e0 -= u00 * s0 + u01 * s1; e1 -= u10 * s0 + u11 * s1;
                const double k0 = Q(4, q), k1 = Q(5, q), k2 = Q(6, q), k3 = Q(7, q);
                m0 = -(u00 * k0 + u01 * k2); m1 = -(u00 * k1 + u01 * k3);
                m2 = -(u10 * k0 + u11 * k2); m3 = -(u10 * k1 + u11 * k3);
            }
            const double det = d00 * d11 - d01 * d10;
            if (det == 0.0) ok = false;
            const double id = 1.0 / det;
            const double i00 = d11 * id, i01 = -d01 * id, i10 = -d10 * id, i11 = d00 * id;
            __syncthreads();                  // every partition has read step h's rows
            Q(0, r) = i00 * n0 + i01 * n2; Q(1, r) = i00 * n1 + i01 * n3;
            Q(2, r) = i10 * n0 + i11 * n2; Q(3, r) = i10 * n1 + i11 * n3;
            Q(4, r) = i00 * m0 + i01 * m2; Q(5, r) = i00 * m1 + i01 * m3;
            Q(6, r) = i10 * m0 + i11 * m2; Q(7, r) = i10 * m1 + i11 * m3;
            Q(8, r) = i00 * e0 + i01 * e1; Q(9, r) = i10 * e0 + i11 * e1;
        }
        // X_r is now row r's right-hand side: y are the left neighbour's last
        // row and the right neighbour's first row
        __syncthreads();
        if (has_l) yl = Q(9, r - 1);
        if (has_r) yr = Q(8, r + 1);
        if (!ok && active) atomicOr(A.status, kStatusZeroPivot);
    } else {
        // Zbar (Eq. (10)) of this lane's line: row 2i-1 = [v_m^(L), w_m^(L), 1],
        // row 2i = [1, v_1^(R), w_1^(R)] around the diagonal; cyclic if periodic.
        const int NI = periodic ? P : P - 1, K = 2 * NI;
        bool ok = true;
        if (SHIFT || !periodic) {             // (shifted systems are never periodic)
            // the band of every lane's Zbar in LDS (after the tips), solved by
            // wavefront 0 alone; the other partitions read their y after the barrier
            double *Z = sh + (size_t)6 * P * LW;
            auto B = [&](int q, int k) -> double & { return Z[((size_t)q * K + k) * LW + lane]; };
            if (r == 0 && K > 0) {
                for (int i = 1; i <= NI; ++i) {
                    const int Li = i - 1, Ri = i;
                    const int u1 = 2 * i - 2, u2 = 2 * i - 1;
                    if (u1 > 0) B(0, u1 - 1) = S(3, Li);   // dl: v_m^(L) (zero for L = 0)
                    B(1, u1) = S(5, Li);                    // dd: w_m^(L)
                    B(2, u1) = 1.0;                         // du
                    B(0, u1) = 1.0;                         // dl
                    B(1, u2) = S(2, Ri);                    // dd: v_1^(R)
                    if (u2 < K - 1) B(2, u2) = S(4, Ri);    // du: w_1^(R)
                    B(4, u1) = S(1, Li);                    // rhs
                    B(4, u2) = S(0, Ri);
                }
                ok = gtsv_pivot_strided(K, &B(0, 0), &B(1, 0), &B(2, 0), &B(3, 0), &B(4, 0), LW);
            }
            __syncthreads();
            if (has_l) yl = B(4, 2 * r - 1);   // r >= 1 here (not periodic)
            if (has_r) yr = B(4, 2 * r);
        } else {
            double rhs[kGenKDense];
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
            if (has_l) {
                const int il = (r >= 1) ? r : P;
                yl = rhs[2 * il - 1];
            }
            if (has_r) yr = rhs[2 * r];
        }
        if (!ok && active) atomicOr(A.status, kStatusZeroPivot);
    }

    // x = x~ - (y_left v + y_right w), with v + w reduced by the same pivots
    if (active && !PIVOT) {
        double dn = 0.0;
#pragma unroll
        for (int t = CMAX - 1; t >= 0; --t)
            if (t < m) {
                const double gd = yl * gv[t] + ((t == m - 1) ? yr * wm : 0.0);
                dn = gd - cp[t] * dn;
                p[t * sj] = x[t] - dn;
            }
    } else if (active) {
        double d1 = 0.0, d2 = 0.0;
#pragma unroll
        for (int t = CMAX - 1; t >= 0; --t)
            if (t < m) {
                const bool l2 = (two >> t) & 1;
                const double pw = (t == m - 1) ? wl1 : ((t == m - 2) ? wl2 : 0.0);
                const double dn = (yl * gv[t] + yr * pw) - cp[t] * (l2 ? d2 : d1);
                d2 = d1, d1 = dn;
                p[t * sj] = x[t] - dn;
            }
    }
}

size_t general_lds_bytes(int P, int periodic, bool shift)
{
    if (shift) return sizeof(double) * (size_t)10 * P * 32;   // block cyclic reduction rows
    const int K = periodic ? 0 : 2 * (P - 1);   // LDS band of the non-periodic reduced systems
    return sizeof(double) * ((size_t)6 * P + 5 * K) * 64;
}

template <int CMAX, int METHOD>
static hipError_t launch_general_t(const GeneralArgs &a, hipStream_t s)
{
    const int64_t blocks = a.ngroups0 * a.nb1;
    const size_t lds = general_lds_bytes(a.P, METHOD == TRI_PPT ? a.periodic : 1, METHOD == TRI_PPT && a.lamz);
    // 64 lines and P > 8 partitions need 1024-lane workgroups (at most 128
    // VGPRs a lane); fewer run with the 512-lane bound and twice the registers
    // (more than 16 rows per partition come with at most 8 partitions).  The
    // shifted systems run 32 lines a workgroup, so up to 16 partitions fit 512.
    if constexpr (CMAX <= 16) {
        if (a.P > 8 && !a.lamz) {
            hipLaunchKernelGGL((k_general<CMAX, METHOD, false, 1024>), dim3((unsigned)blocks), dim3(64 * a.P), lds, s, a);
            return hipGetLastError();
        }
    }
    if (a.P > (a.lamz ? 16 : 8)) return hipErrorInvalidValue;
    if (a.lamz) {
        // 32 lines a workgroup (the kernel's LW for these instances)
        GeneralArgs h = a;
        h.ngroups0 = (a.nb0 + 31) / 32;
        const size_t lds32 = METHOD == TRI_PPT ? lds : sizeof(double) * (size_t)6 * a.P * 32;
        hipLaunchKernelGGL((k_general<CMAX, METHOD, true, 512>), dim3((unsigned)(h.ngroups0 * h.nb1)), dim3(32 * a.P),
                           lds32, s, h);
    } else {
        hipLaunchKernelGGL((k_general<CMAX, METHOD, false, 512>), dim3((unsigned)blocks), dim3(64 * a.P), lds, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_general(const GeneralArgs &a, int method, hipStream_t s)
{
    if (a.m <= 8)
        return method == TRI_PDD ? launch_general_t<8, TRI_PDD>(a, s) : launch_general_t<8, TRI_PPT>(a, s);
    if (a.m <= 16)
        return method == TRI_PDD ? launch_general_t<16, TRI_PDD>(a, s) : launch_general_t<16, TRI_PPT>(a, s);
    if (a.m <= 32)
        return method == TRI_PDD ? launch_general_t<32, TRI_PDD>(a, s) : launch_general_t<32, TRI_PPT>(a, s);
    return hipErrorInvalidValue;
}

}  // namespace tri
