// tri_device.h -- device helpers shared by the libtri kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "tri_internal.h"

namespace tri {

typedef double v2d __attribute__((ext_vector_type(2)));   // 16-byte vector access

// Global-address-space views of table and field pointers.  The solve bodies
// load through these, so the compiler emits global (and, for uniform
// addresses, scalar) loads even where the pointer was read from memory, as
// in the batched launches, rather than flat ones.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) int gint;
typedef __attribute__((address_space(1))) v2d gv2d;
// Constant-address-space views of the factor tables, which no kernel writes
// while it reads them: wavefront-uniform loads through these are scalar loads
// whatever else the kernel stores (the level kernel, with many bodies in one
// function, is too large for the compiler to prove that by itself).
typedef __attribute__((address_space(4))) double cdouble;
typedef __attribute__((address_space(4))) int cint;

// ===========================================================================
// Reduced-system evaluation shared by the solve kernels: the left and right
// interface unknowns of partition r from the tips of its line.
// tip(q): q = 2*partition (first row) or 2*partition + 1 (last row).
// ===========================================================================
template <int METHOD, typename ItPtr, typename TipFn>
__device__ __forceinline__ void interface_unknowns(ItPtr it, int r, int P, int periodic, TipFn tip, double &yl,
                                                   double &yr)
{
    yl = 0.0;
    yr = 0.0;
    const bool has_l = (r > 0) || periodic;
    const bool has_r = (r < P - 1) || periodic;
    const int rowlen = 2 * P;
    if (METHOD == TRI_PDD) {
        if (has_l) {
            const int L = (r > 0) ? r - 1 : P - 1;
            yl = it[2 * L + 1] * tip(2 * L + 1) + it[2 * r] * tip(2 * r);
        }
        if (has_r) {
            const int R = (r < P - 1) ? r + 1 : 0;
            yr = it[rowlen + 2 * R] * tip(2 * R) + it[rowlen + 2 * r + 1] * tip(2 * r + 1);
        }
    } else {
        const int q0 = periodic ? 0 : 1;
        const int q1 = periodic ? rowlen : rowlen - 1;
        if (has_l)
            for (int q = q0; q < q1; ++q) yl += it[q] * tip(q);
        if (has_r)
            for (int q = q0; q < q1; ++q) yr += it[rowlen + q] * tip(q);
    }
}

// ===========================================================================
// Reduced systems of per-line coefficients (general kernels): one per lane.
// ===========================================================================
constexpr int kGenKMax = 2 * kPMax;        // banded reduced system (non-periodic)
constexpr int kGenKDense = 8;              // dense reduced system (periodic, P <= 4)

// Tridiagonal Gaussian elimination with partial pivoting (row interchanges
// between neighbours, one extra superdiagonal of fill), K <= kGenKMax.
// dl[k]: entry (k+1, k), dd[k]: (k, k), du[k]: (k, k+1).  rhs -> solution.
__device__ inline bool gtsv_pivot(int K, double *dl, double *dd, double *du, double *rhs)
{
    double du2[kGenKMax];
    for (int k = 0; k < K - 1; ++k) {
        if (fabs(dd[k]) >= fabs(dl[k])) {
            if (dd[k] == 0.0) return false;
            const double l = dl[k] / dd[k];
            dd[k + 1] -= l * du[k];
            rhs[k + 1] -= l * rhs[k];
            du2[k] = 0.0;
        } else {
            const double l = dd[k] / dl[k];
            const double old_ddk1 = dd[k + 1];
            dd[k] = dl[k];
            dd[k + 1] = du[k] - l * old_ddk1;
            du[k] = old_ddk1;
            if (k < K - 2) {
                du2[k] = du[k + 1];
                du[k + 1] = -l * du2[k];
            } else {
                du2[k] = 0.0;
            }
            const double rk = rhs[k];
            rhs[k] = rhs[k + 1];
            rhs[k + 1] = rk - l * rhs[k];
        }
    }
    if (dd[K - 1] == 0.0) return false;
    rhs[K - 1] /= dd[K - 1];
    if (K >= 2) rhs[K - 2] = (rhs[K - 2] - du[K - 2] * rhs[K - 1]) / dd[K - 2];
    for (int k = K - 3; k >= 0; --k)
        rhs[k] = (rhs[k] - du[k] * rhs[k + 1] - du2[k] * rhs[k + 2]) / dd[k];
    return true;
}

// The same elimination on arrays with element k at x[k * st] (a lane's
// column of LDS arrays): dl, dd, du, du2 (fill, scratch), rhs -> solution.
__device__ inline bool gtsv_pivot_strided(int K, double *dl, double *dd, double *du, double *du2, double *rhs,
                                          int st)
{
    for (int k = 0; k < K - 1; ++k) {
        const double dlk = dl[k * st], ddk = dd[k * st], duk = du[k * st];
        if (fabs(ddk) >= fabs(dlk)) {
            if (ddk == 0.0) return false;
            const double l = dlk / ddk;
            dd[(k + 1) * st] -= l * duk;
            rhs[(k + 1) * st] -= l * rhs[k * st];
            du2[k * st] = 0.0;
        } else {
            const double l = ddk / dlk;
            const double old_ddk1 = dd[(k + 1) * st];
            dd[k * st] = dlk;
            dd[(k + 1) * st] = duk - l * old_ddk1;
            du[k * st] = old_ddk1;
            if (k < K - 2) {
                const double f = du[(k + 1) * st];
                du2[k * st] = f;
                du[(k + 1) * st] = -l * f;
            } else {
                du2[k * st] = 0.0;
            }
            const double rk = rhs[k * st];
            rhs[k * st] = rhs[(k + 1) * st];
            rhs[(k + 1) * st] = rk - l * rhs[k * st];
        }
    }
    if (dd[(K - 1) * st] == 0.0) return false;
    rhs[(K - 1) * st] /= dd[(K - 1) * st];
    if (K >= 2) rhs[(K - 2) * st] = (rhs[(K - 2) * st] - du[(K - 2) * st] * rhs[(K - 1) * st]) / dd[(K - 2) * st];
    for (int k = K - 3; k >= 0; --k)
        rhs[k * st] = (rhs[k * st] - du[k * st] * rhs[(k + 1) * st] - du2[k * st] * rhs[(k + 2) * st]) / dd[k * st];
    return true;
}

// Dense Gaussian elimination with partial pivoting, K <= kGenKDense.
__device__ inline bool dense_gepp(int K, double *M, double *rhs)
{
    for (int k = 0; k < K; ++k) {
        int p = k;
        double best = fabs(M[k * kGenKDense + k]);
        for (int i = k + 1; i < K; ++i)
            if (fabs(M[i * kGenKDense + k]) > best) { best = fabs(M[i * kGenKDense + k]); p = i; }
        if (best == 0.0) return false;
        if (p != k) {
            for (int t = k; t < K; ++t) {
                const double s = M[k * kGenKDense + t];
                M[k * kGenKDense + t] = M[p * kGenKDense + t];
                M[p * kGenKDense + t] = s;
            }
            const double s = rhs[k]; rhs[k] = rhs[p]; rhs[p] = s;
        }
        for (int i = k + 1; i < K; ++i) {
            const double l = M[i * kGenKDense + k] / M[k * kGenKDense + k];
            for (int t = k + 1; t < K; ++t) M[i * kGenKDense + t] -= l * M[k * kGenKDense + t];
            rhs[i] -= l * rhs[k];
        }
    }
    for (int k = K - 1; k >= 0; --k) {
        double s = rhs[k];
        for (int t = k + 1; t < K; ++t) s -= M[k * kGenKDense + t] * rhs[t];
        rhs[k] = s / M[k * kGenKDense + k];
    }
    return true;
}

}  // namespace tri
