"""Projection step on a staggered (y, z) or (x, y, z) grid, FP64, numpy/scipy + the oracle's solves.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The fractional-step method of Sec. 2.2 ends each sub-step by projecting the
intermediate velocity onto a divergence-free field with the pseudo-pressure
phi: the Poisson equation for phi is solved with a Fourier transform in the
periodic spanwise direction and complex tridiagonal solves in y, then the
velocity is corrected by the gradient of phi.  Here every x-station is an
independent (y, z) plane, with

* cells j = 0..Ny-1 (wall-clustered widths dy_j), k = 0..Nz-1 (periodic, dz);
* v on y-faces j = 0..Ny (v = 0 on the wall y = 0 and on the top y = 1);
* w on z-faces k = 0..Nz-1 (face k between cells k-1 and k).

Discrete divergence D = (v_{j+1}-v_j)/dy_j + (w_{k+1}-w_k)/dz; the matching
Laplacian div(grad phi) has off-diagonals ay_j = 1/(dy_j h_{j-1/2}),
cy_j = 1/(dy_j h_{j+1/2}) in y and, after the real FFT in z, the shift
-lam_k = -(4/dz^2) sin^2(pi k/Nz); the k = 0 mode is gauge pinned.  Because
the operators are built to match, the corrected velocity is divergence free
to round-off, which pins the Poisson solve end to end.
"""
from __future__ import annotations

import numpy as np

from . import PPT, poisson


def divergence(v: np.ndarray, w: np.ndarray, dy: np.ndarray, dz: float) -> np.ndarray:
    """v[Nz][Ny+1][Nx], w[Nz][Ny][Nx] -> D[Nz][Ny][Nx] at cell centres."""
    dv = (v[:, 1:, :] - v[:, :-1, :]) / dy[None, :, None]
    dw = (np.roll(w, -1, axis=0) - w) / dz
    return dv + dw


def spanwise_rfft(x: np.ndarray) -> np.ndarray:
    """Real DFT along z (axis 0): X_k = sum_n x_n exp(-2 pi i k n/Nz), k = 0..Nz/2."""
    return np.ascontiguousarray(np.fft.rfft(x, axis=0))


def spanwise_irfft(X: np.ndarray, nz: int) -> np.ndarray:
    """Inverse of spanwise_rfft over the Hermitian extension, 1/Nz scaling."""
    return np.ascontiguousarray(np.fft.irfft(X, n=nz, axis=0))


def metric(dy: np.ndarray, nz: int, dz: float):
    """Poisson operator of the grid: ay, cy (d2/dy2 off-diagonals) and lam_k."""
    ny = dy.size
    yc_gap = 0.5 * (dy[:-1] + dy[1:])            # h_{j+1/2}, j = 0..Ny-2
    ay = np.zeros(ny)
    cy = np.zeros(ny)
    ay[1:] = 1.0 / (dy[1:] * yc_gap)
    cy[:-1] = 1.0 / (dy[:-1] * yc_gap)
    lam = (4.0 / dz ** 2) * np.sin(np.pi * np.arange(nz // 2 + 1) / nz) ** 2
    return ay, cy, lam


def correct(phihat: np.ndarray, v: np.ndarray, w: np.ndarray, dy: np.ndarray, dz: float):
    """phi = inverse FFT of phihat; return (v_new, w_new, phi) corrected by grad phi
    (interior y-faces only, w periodic)."""
    Nz, Ny, Nx = w.shape
    yc_gap = 0.5 * (dy[:-1] + dy[1:])
    phi = spanwise_irfft(phihat, Nz)
    v_new = v.copy()
    v_new[:, 1:Ny, :] -= (phi[:, 1:, :] - phi[:, :-1, :]) / yc_gap[None, :, None]
    w_new = w - (phi - np.roll(phi, 1, axis=0)) / dz
    return v_new, w_new, phi


# ---- the 3-D step: walls at both x-ends as well, cosine transform in x ------

def divergence3d(u: np.ndarray, v: np.ndarray, w: np.ndarray, dx: float, dy: np.ndarray,
                 dz: float) -> np.ndarray:
    """u[Nz][Ny][Nx+1] (x-faces), v, w as in divergence -> D[Nz][Ny][Nx]."""
    return (u[:, :, 1:] - u[:, :, :-1]) / dx + divergence(v, w, dy, dz)


def streamwise_dct(x: np.ndarray) -> np.ndarray:
    """Cosine transform along the last axis (x), real and imaginary parts alike:
    X_k = sum_n x_n cos(pi k (2n+1)/(2N))."""
    import scipy.fft as sf
    x = np.asarray(x)
    out = sf.dct(x.real, type=2, axis=-1) / 2
    if np.iscomplexobj(x):
        out = out + 1j * (sf.dct(x.imag, type=2, axis=-1) / 2)
    return np.ascontiguousarray(out)


def streamwise_idct(X: np.ndarray) -> np.ndarray:
    """Exact inverse of streamwise_dct."""
    import scipy.fft as sf
    X = np.asarray(X)
    out = sf.idct(2 * X.real, type=2, axis=-1)
    if np.iscomplexobj(X):
        out = out + 1j * sf.idct(2 * X.imag, type=2, axis=-1)
    return np.ascontiguousarray(out)


def metric_x(nx: int, dx: float) -> np.ndarray:
    """lam_x(i) = (4/dx^2) sin^2(pi i/(2 Nx)): eigenvalues (negated) of the cell-centred
    Neumann second difference in x, whose eigenvectors are the cosine modes."""
    return (4.0 / dx ** 2) * np.sin(np.pi * np.arange(nx) / (2 * nx)) ** 2


def correct3d(phihat: np.ndarray, u: np.ndarray, v: np.ndarray, w: np.ndarray, dx: float,
              dy: np.ndarray, dz: float):
    """correct(), and u on the interior x-faces by the x-gradient of phi."""
    v_new, w_new, phi = correct(phihat, v, w, dy, dz)
    u_new = u.copy()
    u_new[:, :, 1:-1] -= (phi[:, :, 1:] - phi[:, :, :-1]) / dx
    return u_new, v_new, w_new, phi


def project3d(u: np.ndarray, v: np.ndarray, w: np.ndarray, dx: float, dy: np.ndarray, dz: float,
              P: int = 8, method: int = PPT):
    """Return (u_new, v_new, w_new, phi) with div(u_new, v_new, w_new) = 0 to round-off."""
    from . import poisson_shifted_batch
    Nz, Ny, Nx = w.shape
    ay, cy, lamz = metric(dy, Nz, dz)
    lamx = metric_x(Nx, dx)
    Dhat = streamwise_dct(spanwise_rfft(divergence3d(u, v, w, dx, dy, dz)))
    poisson_shifted_batch(Dhat, ay, cy, lamz, lamx, P, method)
    return correct3d(streamwise_idct(Dhat), u, v, w, dx, dy, dz)


def project(v: np.ndarray, w: np.ndarray, dy: np.ndarray, dz: float, P: int = 4,
            method: int = PPT, nthreads: int = 0):
    """Return (v_new, w_new, phi) with div(v_new, w_new) = 0 to round-off."""
    Nz = w.shape[0]
    ay, cy, lam = metric(dy, Nz, dz)
    Dhat = spanwise_rfft(divergence(v, w, dy, dz))
    poisson(Dhat, ay, cy, lam, P=P, method=method, nthreads=nthreads)
    return correct(Dhat, v, w, dy, dz)
