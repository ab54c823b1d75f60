// tri_ns.h -- launchers of the fractional-step time step's explicit kernels
// (tri_ns.hip): the momentum right-hand side of one Runge-Kutta sub-step, the
// velocity update and the pressure update.  Internal to libtri.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tri {

// Per-row constants of the stretched y mesh, NS_YCOEF doubles for each cell
// row j (cell widths dy, h_j = (dy_{j-1} + dy_j)/2, dy_{-1} = dy_{Ny} = 0):
//   0 1/dy_j   1 1/h_j
//   2 fm = dy_j/(dy_{j-1} + dy_j)   3 fp = dy_{j-1}/(dy_{j-1} + dy_j)
//     (a cell-centred q at y-face j: fm q_{j-1} + fp q_j)
//   4 gm = dy_{j+1}/(dy_j + dy_{j+1})   5 gp = dy_j/(dy_j + dy_{j+1})
//     (at y-face j+1: gm q_j + gp q_{j+1})
//   6..8  second difference of a cell-centred q in y (no-slip wall below cell
//         0, zero flux through the top): lo, diag, up
//   9..11 second difference of v on y-face j (walls at faces 0 and Ny): lo,
//         diag, up
// Computed on the host once (ns_create); the kernel reads its row's entries
// with scalar loads.
constexpr int NS_YCOEF = 12;
void ns_ycoef_row(const double *dy, int64_t Ny, int64_t j, double *out);

struct NsRhsArgs {
    const double *u = nullptr, *v = nullptr, *w = nullptr, *p = nullptr;
    const double *ycoef = nullptr;                   // [Ny][NS_YCOEF]
    int64_t Nx = 0, Ny = 0, Nz = 0;
    double idx = 0.0, idz = 0.0, idx2 = 0.0, idz2 = 0.0;   // 1/dx, 1/dz, 1/dx^2, 1/dz^2
    double dt = 0.0, nu = 0.0;
    double gamma = 0.0, zeta = 0.0, alpha = 0.0;     // the sub-step's coefficients
    double *Nu = nullptr, *Nv = nullptr, *Nw = nullptr;   // convection: previous in, this sub-step's out
    double *du = nullptr, *dv = nullptr, *dw = nullptr;   // right-hand sides of the ADI sweeps
};
hipError_t launch_ns_rhs(const NsRhsArgs &A, hipStream_t s);
hipError_t launch_ns_update(double *u, double *v, double *w, const double *du, const double *dv, const double *dw,
                            int64_t Nx, int64_t Ny, int64_t Nz, hipStream_t s);
hipError_t launch_ns_pressure(double *p, const double *phi, double scale, int64_t n, hipStream_t s);
// Whether launch_strided2 (two lines per lane) has an accumulating instance
// (a.acc set: a_b0 = 1, the target's line pairs 16-byte aligned) for this
// method and chunk instance (tri_kernels.hip).
bool strided2_acc_supported(int method, int chunk_max);
// The 3-D step's wall-parallel corrections (launch_grad_xy) that also add
// phi * ps to the pressure p (cells like phi): the pressure update of a
// sub-step from the same read of phi (tri_fft.hip).
hipError_t launch_grad_xy_pressure(double *u, double *v, const double *phi, const double *dy, double dx, int64_t Nx,
                                   int64_t Ny, int64_t Nz, double *p, double ps, hipStream_t s);

}  // namespace tri
