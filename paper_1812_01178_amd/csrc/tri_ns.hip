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
// One thread per cell (i, j, k) computes the three unknowns of that index;
// every array is HBM-resident and read through the caches (stencil reuse of
// neighbouring rows), so the kernel is bound by HBM.
#include <hip/hip_runtime.h>

#include "tri_internal.h"

namespace tri {

namespace {

struct NsView {
    const double *u, *v, *w, *p;
    const double *dy;
    int64_t Nx, Ny, Nz;
    __device__ __forceinline__ double U(int64_t k, int64_t j, int64_t i) const { return u[(k * Ny + j) * (Nx + 1) + i]; }
    __device__ __forceinline__ double V(int64_t k, int64_t j, int64_t i) const { return v[(k * (Ny + 1) + j) * Nx + i]; }
    __device__ __forceinline__ double W(int64_t k, int64_t j, int64_t i) const { return w[(k * Ny + j) * Nx + i]; }
    __device__ __forceinline__ double Pc(int64_t k, int64_t j, int64_t i) const { return p[(k * Ny + j) * Nx + i]; }
};

// cell-centred quantity q(j) interpolated to the interior y-face j (1..Ny-1)
__device__ __forceinline__ double to_yface(double qm, double q, double dym, double dyj)
{
    return (dyj * qm + dym * q) / (dym + dyj);
}

__global__ void __launch_bounds__(256) k_ns_rhs(const NsView G, const NsRhsArgs A)
{
    const int64_t Nx = G.Nx, Ny = G.Ny, Nz = G.Nz;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t j = blockIdx.y, k = blockIdx.z;
    if (i >= Nx) return;
    const int64_t km = (k == 0) ? Nz - 1 : k - 1, kp = (k == Nz - 1) ? 0 : k + 1;
    const double dx = A.dx, dz = A.dz, idx2 = 1.0 / (dx * dx), idz2 = 1.0 / (dz * dz);
    const double dyj = G.dy[j];
    const double dym = (j > 0) ? G.dy[j - 1] : 0.0;          // dy_{j-1}
    const double dyp = (j < Ny - 1) ? G.dy[j + 1] : 0.0;     // dy_{j+1}
    const int64_t o = (k * Ny + j) * Nx + i;
    const double cg = A.gamma, cz = A.zeta, ca = A.alpha, nu = A.nu, dt = A.dt;

    // y second difference of a cell-centred component (no-slip wall below cell
    // 0, zero flux through the top): lo q_{j-1} + diag q_j + up q_{j+1}
    auto lap_y_cell = [&](double qm, double q, double qp) {
        const double lo = (j >= 1) ? 1.0 / (dyj * (0.5 * (dym + dyj))) : 0.0;
        const double up = (j <= Ny - 2) ? 1.0 / (dyj * (0.5 * (dyj + dyp))) : 0.0;
        double diag = -(lo + up);
        if (j == 0) diag -= 2.0 / (dyj * dyj);
        return lo * qm + diag * q + up * qp;
    };
    // x second difference of a cell-centred component (slip walls at both ends)
    auto lap_x_cell = [&](double qm, double q, double qp) {
        const double lo = (i >= 1) ? idx2 : 0.0, up = (i <= Nx - 2) ? idx2 : 0.0;
        return lo * qm + (-(lo + up)) * q + up * qp;
    };
    auto lap_z = [&](double qm, double q, double qp) { return idz2 * qm + (-2.0 * idz2) * q + idz2 * qp; };

    // ---------------- u at x-face i (interior faces 1..Nx-1) ----------------
    {
        double R = 0.0, Nq = 0.0;
        if (i >= 1) {
            const double u0 = G.U(k, j, i);
            const double uxm = G.U(k, j, i - 1), uxp = G.U(k, j, i + 1);
            const double ucp = 0.5 * (u0 + uxp), ucm = 0.5 * (uxm + u0);
            const double duu = (ucp * ucp - ucm * ucm) / dx;
            // flux u v through the y-faces j (bottom) and j+1 (top) of the cell
            double Fb = 0.0, Ft = 0.0;
            const double uym = (j >= 1) ? G.U(k, j - 1, i) : 0.0;
            const double uyp = (j <= Ny - 2) ? G.U(k, j + 1, i) : 0.0;
            if (j >= 1) Fb = to_yface(uym, u0, dym, dyj) * (0.5 * (G.V(k, j, i - 1) + G.V(k, j, i)));
            if (j <= Ny - 2) Ft = to_yface(u0, uyp, dyj, dyp) * (0.5 * (G.V(k, j + 1, i - 1) + G.V(k, j + 1, i)));
            const double duv = (Ft - Fb) / dyj;
            // flux u w through the z-faces k and k+1
            const double uzm = G.U(km, j, i), uzp = G.U(kp, j, i);
            const double Gk = (0.5 * (uzm + u0)) * (0.5 * (G.W(k, j, i - 1) + G.W(k, j, i)));
            const double Gk1 = (0.5 * (u0 + uzp)) * (0.5 * (G.W(kp, j, i - 1) + G.W(kp, j, i)));
            const double duw = (Gk1 - Gk) / dz;
            Nq = -(duu + duv + duw);
            // u_Nx (the far wall) is stored as 0, so the x row needs no special case
            const double Lq = (idx2 * uxm + (-2.0 * idx2) * u0 + idx2 * ((i <= Nx - 2) ? uxp : 0.0)) +
                              lap_y_cell(uym, u0, uyp) + lap_z(uzm, u0, uzp);
            const double Gp = (G.Pc(k, j, i) - G.Pc(k, j, i - 1)) / dx;
            R = dt * (cg * Nq + (cz != 0.0 ? cz * A.Nu[o] : 0.0) + ca * (nu * Lq - Gp));
        }
        A.Nu[o] = Nq;
        A.du[o] = R;
    }
    // ---------------- v at y-face j (interior faces 1..Ny-1) ----------------
    {
        double R = 0.0, Nq = 0.0;
        if (j >= 1) {
            const double v0 = G.V(k, j, i);
            // flux v u through the x-faces i and i+1 (u = 0 on the x-walls)
            double Hl = 0.0, Hr = 0.0;
            const double vxm = (i >= 1) ? G.V(k, j, i - 1) : 0.0;
            const double vxp = (i <= Nx - 2) ? G.V(k, j, i + 1) : 0.0;
            if (i >= 1) Hl = (0.5 * (vxm + v0)) * to_yface(G.U(k, j - 1, i), G.U(k, j, i), dym, dyj);
            if (i <= Nx - 2) Hr = (0.5 * (v0 + vxp)) * to_yface(G.U(k, j - 1, i + 1), G.U(k, j, i + 1), dym, dyj);
            const double dvu = (Hr - Hl) / dx;
            const double vym = G.V(k, j - 1, i), vyp = G.V(k, j + 1, i);
            const double vcp = 0.5 * (v0 + vyp), vcm = 0.5 * (vym + v0);
            const double hj = 0.5 * (dym + dyj);
            const double dvv = (vcp * vcp - vcm * vcm) / hj;
            // flux v w through the z-faces k and k+1
            const double vzm = G.V(km, j, i), vzp = G.V(kp, j, i);
            const double Gk = (0.5 * (vzm + v0)) * to_yface(G.W(k, j - 1, i), G.W(k, j, i), dym, dyj);
            const double Gk1 = (0.5 * (v0 + vzp)) * to_yface(G.W(kp, j - 1, i), G.W(kp, j, i), dym, dyj);
            const double dvw = (Gk1 - Gk) / dz;
            Nq = -(dvu + dvv + dvw);
            // y second difference on the faces (walls at faces 0 and Ny, held 0)
            const double lo = 1.0 / (hj * dym), upf = 1.0 / (hj * dyj);
            const double up = (j <= Ny - 2) ? upf : 0.0;
            const double Ly = lo * vym + (-(lo + upf)) * v0 + up * vyp;
            const double Lq = lap_x_cell(vxm, v0, vxp) + Ly + lap_z(vzm, v0, vzp);
            const double Gp = (G.Pc(k, j, i) - G.Pc(k, j - 1, i)) / hj;
            R = dt * (cg * Nq + (cz != 0.0 ? cz * A.Nv[o] : 0.0) + ca * (nu * Lq - Gp));
        }
        A.Nv[o] = Nq;
        A.dv[o] = R;
    }
    // ---------------- w at z-face k ----------------------------------------
    {
        const double w0 = G.W(k, j, i);
        // flux w u through the x-faces i and i+1 (u = 0 on the x-walls)
        double Hl = 0.0, Hr = 0.0;
        const double wxm = (i >= 1) ? G.W(k, j, i - 1) : 0.0;
        const double wxp = (i <= Nx - 2) ? G.W(k, j, i + 1) : 0.0;
        if (i >= 1) Hl = (0.5 * (wxm + w0)) * (0.5 * (G.U(km, j, i) + G.U(k, j, i)));
        if (i <= Nx - 2) Hr = (0.5 * (w0 + wxp)) * (0.5 * (G.U(km, j, i + 1) + G.U(k, j, i + 1)));
        const double dwu = (Hr - Hl) / dx;
        // flux w v through the y-faces j and j+1 (v = 0 on the y-walls)
        double Fb = 0.0, Ft = 0.0;
        const double wym = (j >= 1) ? G.W(k, j - 1, i) : 0.0;
        const double wyp = (j <= Ny - 2) ? G.W(k, j + 1, i) : 0.0;
        if (j >= 1) Fb = to_yface(wym, w0, dym, dyj) * (0.5 * (G.V(km, j, i) + G.V(k, j, i)));
        if (j <= Ny - 2) Ft = to_yface(w0, wyp, dyj, dyp) * (0.5 * (G.V(km, j + 1, i) + G.V(k, j + 1, i)));
        const double dwv = (Ft - Fb) / dyj;
        const double wzm = G.W(km, j, i), wzp = G.W(kp, j, i);
        const double wcp = 0.5 * (w0 + wzp), wcm = 0.5 * (wzm + w0);
        const double dww = (wcp * wcp - wcm * wcm) / dz;
        const double Nq = -(dwu + dwv + dww);
        const double Lq = lap_x_cell(wxm, w0, wxp) + lap_y_cell(wym, w0, wyp) + lap_z(wzm, w0, wzp);
        const double Gp = (G.Pc(k, j, i) - G.Pc(km, j, i)) / dz;
        const double R = dt * (cg * Nq + (cz != 0.0 ? cz * A.Nw[o] : 0.0) + ca * (nu * Lq - Gp));
        A.Nw[o] = Nq;
        A.dw[o] = R;
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
    const NsView G{A.u, A.v, A.w, A.p, A.dy, A.Nx, A.Ny, A.Nz};
    const dim3 grid((unsigned)((A.Nx + 255) / 256), (unsigned)A.Ny, (unsigned)A.Nz);
    hipLaunchKernelGGL(k_ns_rhs, grid, dim3(256), 0, s, G, A);
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
