// tri_ns.hip -- the explicit parts of the fractional-step time step (Sec. 2.2):
// convection and viscous terms of the momentum right-hand side, the velocity
// update after the ADI sweeps and the pressure update after the projection.
//
// Staggered grid (Sec. 2.1): Nx x Ny x Nz cells, uniform dx and dz, cell widths
// dy_j in y.  u[Nz][Ny][Nx+1] on x-faces (faces 0 and Nx are walls, held 0),
// v[Nz][Ny+1][Nx] on y-faces (face 0 the no-slip wall, face Ny the top, held
// 0), w[Nz][Ny][Nx] on z-faces (periodic), p[Nz][Ny][Nx] at cells.  Tangential
// components: no-slip at y = 0 (mirror value -q at distance dy_0),
// stress-free top (zero flux), slip walls at both x-ends (zero flux).
//
// Sub-step s of the Runge-Kutta scheme (coefficients gamma_s, zeta_s,
// alpha_s) forms, for every velocity unknown q,
//     N_q = -d(q u_j)/dx_j   (second-order central, divergence form)
//     R_q = dt (gamma_s N_q + zeta_s N_q,prev + alpha_s (nu L q - G_q p))
// (N_q,prev is not read when zeta_s = 0, the first sub-step) and stores R_q
// into the increment arrays du, dv, dw ([Nz][Ny][Nx]: x-faces
// 0..Nx-1 of u, y-faces 0..Ny-1 of v, every z-face of w; the wall faces 0 get
// R = 0) and N_q over N_q,prev.  Interpolations to a face: the mean of the two
// neighbours on the uniform directions, the distance-weighted mean on the
// stretched y mesh, (dy_j q_{j-1} + dy_{j-1} q_j) / (dy_{j-1} + dy_j).
// One thread per column (i, j) marches in z and computes the three unknowns
// of every cell of the column; the kernel is bound by HBM.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "tri_ns.h"

namespace tri {

namespace {

// The stencil of one cell (i, j) in one z-plane: every value of u, v, w, p at
// that plane the three unknowns of the cell need (_xm/_xp: i -/+ 1, _ym/_yp:
// j -/+ 1; values outside the grid read as 0 and are never used).
struct Plane {
    double u_xm, u0, u_xp, u_ym, u_yp, u_ymxp;
    double v_xm, v0, v_xp, v_ypxm, v_yp, v_ym;
    double w_xm, w0, w_xp, w_ym, w_yp;
    double p0, p_xm, p_ym;
};

struct NsColumn {
    const double *u, *v, *w, *p;
    int64_t Nx, Ny;
    int64_t i, j;
    // the plane-k stencil of cell (i, j)
    __device__ __forceinline__ void load(int64_t k, Plane &q) const
    {
        const double *U = u + (k * Ny + j) * (Nx + 1) + i;       // u[k][j][i]
        const double *V = v + (k * (Ny + 1) + j) * Nx + i;      // v[k][j][i]
        const double *Wp = w + (k * Ny + j) * Nx + i;
        const double *Pp = p + (k * Ny + j) * Nx + i;
        const bool xm = i >= 1, xp = i <= Nx - 2, ym = j >= 1, yp = j <= Ny - 2;
        const int64_t su = Nx + 1, sv = Nx;
        q.u_xm = xm ? U[-1] : 0.0;
        q.u0 = U[0];
        q.u_xp = U[1];                                            // face i + 1 <= Nx exists
        q.u_ym = ym ? U[-su] : 0.0;
        q.u_yp = yp ? U[su] : 0.0;
        q.u_ymxp = ym ? U[1 - su] : 0.0;
        q.v_xm = xm ? V[-1] : 0.0;
        q.v0 = V[0];
        q.v_xp = xp ? V[1] : 0.0;
        q.v_ypxm = xm ? V[sv - 1] : 0.0;                          // face j + 1 <= Ny exists
        q.v_yp = V[sv];
        q.v_ym = ym ? V[-sv] : 0.0;
        q.w_xm = xm ? Wp[-1] : 0.0;
        q.w0 = Wp[0];
        q.w_xp = xp ? Wp[1] : 0.0;
        q.w_ym = ym ? Wp[-sv] : 0.0;
        q.w_yp = yp ? Wp[sv] : 0.0;
        q.p0 = Pp[0];
        q.p_xm = xm ? Pp[-1] : 0.0;
        q.p_ym = ym ? Pp[-sv] : 0.0;
    }
};


// One thread per column (i, j), marching in z over the planes of its segment
// (blockIdx.z; the segments split the periodic z range evenly) with the
// stencils of planes k - 1 (the values still needed), k (C) and k + 1 (Nn,
// loaded while plane k is computed) in registers: every plane of u, v, w, p
// is read once per column and segment (the x- and y-neighbours of a row come
// from the same cache lines as the neighbouring columns'), and no address is
// recomputed from (i, j, k) inside the march.
__global__ void __launch_bounds__(256) k_ns_rhs(const NsRhsArgs A)
{
    const int64_t Nx = A.Nx, Ny = A.Ny, Nz = A.Nz;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j = blockIdx.y;
    if (i >= Nx) return;
    const NsColumn G{A.u, A.v, A.w, A.p, Nx, Ny, i, j};
    const double cg = A.gamma, cz = A.zeta, ca = A.alpha, nu = A.nu, dt = A.dt;
    const double idx = A.idx, idz = A.idz, idx2 = A.idx2, idz2 = A.idz2;
    const bool xm = i >= 1, xp = i <= Nx - 2, ym = j >= 1, yp = j <= Ny - 2;
    // this row's constants of the y mesh (uniform: scalar loads), so that the
    // march multiplies where the definitions divide
    const double *__restrict__ yc = A.ycoef + j * NS_YCOEF;
    const double idyj = yc[0], ihj = yc[1], fm = yc[2], fp = yc[3], gm = yc[4], gp = yc[5];
    const double ly_lo = yc[6], ly_dg = yc[7], ly_up = yc[8], lv_lo = yc[9], lv_dg = yc[10], lv_up = yc[11];
    auto face_j = [&](double qm, double q) { return fm * qm + fp * q; };      // q at y-face j
    auto face_j1 = [&](double q, double qp) { return gm * q + gp * qp; };     // q at y-face j+1
    auto lap_y_cell = [&](double qm, double q, double qp) { return ly_lo * qm + ly_dg * q + ly_up * qp; };
    // x second difference of a cell-centred component (slip walls at both ends)
    const double lx_lo = xm ? idx2 : 0.0, lx_up = xp ? idx2 : 0.0, lx_dg = -(lx_lo + lx_up);
    auto lap_x_cell = [&](double qm, double q, double qp) { return lx_lo * qm + lx_dg * q + lx_up * qp; };
    auto lap_z = [&](double qm, double q, double qp) { return idz2 * qm + (-2.0 * idz2) * q + idz2 * qp; };

    // planes k0 .. k1-1 of this segment; plane k0 - 1 (periodic) values still
    // needed: u, u_xp, v, v_yp, w, p
    const int64_t k0 = Nz * blockIdx.z / gridDim.z, k1 = Nz * (blockIdx.z + 1) / gridDim.z;
    Plane C, Nn;
    double b_u0, b_uxp, b_v0, b_vyp, b_w0, b_p0;
    G.load(k0 > 0 ? k0 - 1 : Nz - 1, C);
    b_u0 = C.u0, b_uxp = C.u_xp, b_v0 = C.v0, b_vyp = C.v_yp, b_w0 = C.w0, b_p0 = C.p0;
    G.load(k0, C);
    const int64_t plane = Ny * Nx;
    int64_t o = (k0 * Ny + j) * Nx + i;
    for (int64_t k = k0; k < k1; ++k, o += plane) {
        G.load(k + 1 < Nz ? k + 1 : 0, Nn);
        // the previous convection terms are read once and the outputs written
        // once (non-temporal); u, v, w, p are shared with the neighbour columns
        const double Nu_prev = cz != 0.0 ? __builtin_nontemporal_load(A.Nu + o) : 0.0;
        const double Nv_prev = cz != 0.0 ? __builtin_nontemporal_load(A.Nv + o) : 0.0;
        const double Nw_prev = cz != 0.0 ? __builtin_nontemporal_load(A.Nw + o) : 0.0;
        // ---------------- u at x-face i (interior faces 1..Nx-1) ----------------
        {
            double R = 0.0, Nq = 0.0;
            if (xm) {
                const double u0 = C.u0, uxm = C.u_xm, uxp = C.u_xp;
                const double ucp = 0.5 * (u0 + uxp), ucm = 0.5 * (uxm + u0);
                const double duu = (ucp * ucp - ucm * ucm) * idx;
                // flux u v through the y-faces j (bottom) and j+1 (top) of the cell
                const double uym = C.u_ym, uyp = C.u_yp;
                const double Fb = ym ? face_j(uym, u0) * (0.5 * (C.v_xm + C.v0)) : 0.0;
                const double Ft = yp ? face_j1(u0, uyp) * (0.5 * (C.v_ypxm + C.v_yp)) : 0.0;
                const double duv = (Ft - Fb) * idyj;
                // flux u w through the z-faces k and k+1
                const double uzm = b_u0, uzp = Nn.u0;
                const double Gk = (0.5 * (uzm + u0)) * (0.5 * (C.w_xm + C.w0));
                const double Gk1 = (0.5 * (u0 + uzp)) * (0.5 * (Nn.w_xm + Nn.w0));
                const double duw = (Gk1 - Gk) * idz;
                Nq = -(duu + duv + duw);
                // u_Nx (the far wall) is 0, so the x row needs no special case
                const double Lq = (idx2 * uxm + (-2.0 * idx2) * u0 + idx2 * (xp ? uxp : 0.0)) +
                                  lap_y_cell(uym, u0, uyp) + lap_z(uzm, u0, uzp);
                const double Gp = (C.p0 - C.p_xm) * idx;
                R = dt * (cg * Nq + cz * Nu_prev + ca * (nu * Lq - Gp));
            }
            __builtin_nontemporal_store(Nq, A.Nu + o);
            __builtin_nontemporal_store(R, A.du + o);
        }
        // ---------------- v at y-face j (interior faces 1..Ny-1) ----------------
        {
            double R = 0.0, Nq = 0.0;
            if (ym) {
                const double v0 = C.v0, vxm = C.v_xm, vxp = C.v_xp;
                // flux v u through the x-faces i and i+1 (u = 0 on the x-walls)
                const double Hl = xm ? (0.5 * (vxm + v0)) * face_j(C.u_ym, C.u0) : 0.0;
                const double Hr = xp ? (0.5 * (v0 + vxp)) * face_j(C.u_ymxp, C.u_xp) : 0.0;
                const double dvu = (Hr - Hl) * idx;
                const double vym = C.v_ym, vyp = C.v_yp;
                const double vcp = 0.5 * (v0 + vyp), vcm = 0.5 * (vym + v0);
                const double dvv = (vcp * vcp - vcm * vcm) * ihj;
                // flux v w through the z-faces k and k+1
                const double vzm = b_v0, vzp = Nn.v0;
                const double Gk = (0.5 * (vzm + v0)) * face_j(C.w_ym, C.w0);
                const double Gk1 = (0.5 * (v0 + vzp)) * face_j(Nn.w_ym, Nn.w0);
                const double dvw = (Gk1 - Gk) * idz;
                Nq = -(dvu + dvv + dvw);
                const double Ly = lv_lo * vym + lv_dg * v0 + lv_up * vyp;
                const double Lq = lap_x_cell(vxm, v0, vxp) + Ly + lap_z(vzm, v0, vzp);
                const double Gp = (C.p0 - C.p_ym) * ihj;
                R = dt * (cg * Nq + cz * Nv_prev + ca * (nu * Lq - Gp));
            }
            __builtin_nontemporal_store(Nq, A.Nv + o);
            __builtin_nontemporal_store(R, A.dv + o);
        }
        // ---------------- w at z-face k ----------------------------------------
        {
            const double w0 = C.w0, wxm = C.w_xm, wxp = C.w_xp;
            // flux w u through the x-faces i and i+1 (u = 0 on the x-walls)
            const double Hl = xm ? (0.5 * (wxm + w0)) * (0.5 * (b_u0 + C.u0)) : 0.0;
            const double Hr = xp ? (0.5 * (w0 + wxp)) * (0.5 * (b_uxp + C.u_xp)) : 0.0;
            const double dwu = (Hr - Hl) * idx;
            // flux w v through the y-faces j and j+1 (v = 0 on the y-walls)
            const double wym = C.w_ym, wyp = C.w_yp;
            const double Fb = ym ? face_j(wym, w0) * (0.5 * (b_v0 + C.v0)) : 0.0;
            const double Ft = yp ? face_j1(w0, wyp) * (0.5 * (b_vyp + C.v_yp)) : 0.0;
            const double dwv = (Ft - Fb) * idyj;
            const double wzm = b_w0, wzp = Nn.w0;
            const double wcp = 0.5 * (w0 + wzp), wcm = 0.5 * (wzm + w0);
            const double dww = (wcp * wcp - wcm * wcm) * idz;
            const double Nq = -(dwu + dwv + dww);
            const double Lq = lap_x_cell(wxm, w0, wxp) + lap_y_cell(wym, w0, wyp) + lap_z(wzm, w0, wzp);
            const double Gp = (C.p0 - b_p0) * idz;
            const double R = dt * (cg * Nq + cz * Nw_prev + ca * (nu * Lq - Gp));
            __builtin_nontemporal_store(Nq, A.Nw + o);
            __builtin_nontemporal_store(R, A.dw + o);
        }
        b_u0 = C.u0, b_uxp = C.u_xp, b_v0 = C.v0, b_vyp = C.v_yp, b_w0 = C.w0, b_p0 = C.p0;
        C = Nn;
    }
}

// u* = u + du (x-faces 0..Nx-1), v* = v + dv (y-faces 0..Ny-1), w* = w + dw;
// the far wall faces (u at Nx, v at Ny) are not touched
__global__ void __launch_bounds__(256) k_ns_update(double *u, double *v, double *w, const double *du,
                                                   const double *dv, const double *dw, int64_t Nx, int64_t Ny)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j = blockIdx.y, k = blockIdx.z;
    if (i >= Nx) return;
    const int64_t o = (k * Ny + j) * Nx + i;
    u[(k * Ny + j) * (Nx + 1) + i] += du[o];
    v[(k * (Ny + 1) + j) * Nx + i] += dv[o];
    w[o] += dw[o];
}

// p += phi * scale (scale = 1/(alpha_s dt))
__global__ void __launch_bounds__(256) k_ns_pressure(double *p, const double *phi, double scale, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < n) p[t] += phi[t] * scale;
}

}  // namespace

hipError_t launch_ns_rhs(const NsRhsArgs &A, hipStream_t s)
{
    // z segments of about 48 planes (at most 8): enough workgroups that the
    // last round of a launch is a small part of it, few enough that the
    // plane each segment re-reads below its first is a small part of the reads
    const int64_t nseg = std::max<int64_t>(1, std::min<int64_t>(8, A.Nz / 48));
    const dim3 grid((unsigned)((A.Nx + 255) / 256), (unsigned)A.Ny, (unsigned)nseg);
    hipLaunchKernelGGL(k_ns_rhs, grid, dim3(256), 0, s, A);
    return hipGetLastError();
}

hipError_t launch_ns_update(double *u, double *v, double *w, const double *du, const double *dv, const double *dw,
                            int64_t Nx, int64_t Ny, int64_t Nz, hipStream_t s)
{
    const dim3 grid((unsigned)((Nx + 255) / 256), (unsigned)Ny, (unsigned)Nz);
    hipLaunchKernelGGL(k_ns_update, grid, dim3(256), 0, s, u, v, w, du, dv, dw, Nx, Ny);
    return hipGetLastError();
}

hipError_t launch_ns_pressure(double *p, const double *phi, double scale, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ns_pressure, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, phi, scale, n);
    return hipGetLastError();
}

}  // namespace tri
