"""Seeded synthetic inputs for the batched partitioned tridiagonal solves.

This module is shared by the FP64 oracle, the tests and the benchmark.  It
builds *inputs only*: meshes, tridiagonal coefficient vectors, modified
wavenumbers and random right-hand sides.  It contains none of the solver
arithmetic (no elimination, no partitioning, no reduced systems), so the
oracle and the HIP path stay independent of each other.

Recipes (all FP64, numpy PCG64 via ``numpy.random.default_rng(seed)``):

* Momentum (Crank-Nicolson viscous term, Sec. 2.2): ``I - r*delta^2`` with
  ``r = dt*nu/dx^2`` on a unit domain, so a = c = -r and b = 1 + 2r on the
  uniform x and z meshes; z is periodic (Sec. 2.1), so its a[0] and c[n-1]
  carry the wrap coupling.
* Wall-normal mesh (Sec. 2.1, clustered at the wall): faces
  ``y_j = 1 - tanh(g*(1 - j/Ny))/tanh(g)``, unknowns at cell centres,
  no-slip wall at y=0 (Dirichlet, folded into b[0]) and a stress-free top
  (Neumann, c[Ny-1] = 0).
* Poisson (Sec. 2.2 and the PPT passage of Sec. 3.2): cell-centred Neumann
  y-operator with off-diagonals ay, cy; the diagonal is formed by the solver
  as -(ay+cy) - lam_k with the second-order modified wavenumber
  ``lam_k = (4/dz^2) sin^2(pi k / Nz)`` of the spanwise Fourier transform.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "tanh_faces", "momentum_uniform", "momentum_periodic", "momentum_stretched",
    "poisson_metric", "modified_wavenumbers", "spanwise_rfft",
    "cfg_independent", "cfg_field", "cfg_poisson_rhs", "random_tridiag",
    "random_tridiag_nondominant", "pivot_probe", "RAGGED_SUBGRIDS",
]

NU = 1.0e-3
DT = 1.0e-3
STRETCH = 2.5

# Eight ragged sub-grids (Nx, Ny, Nz) covering every value of the batched
# workload's sets Nx in {256,512,1024,2048}, Ny in {128,256}, Nz in {96,288}.
RAGGED_SUBGRIDS = [
    (256, 128, 96), (256, 256, 288), (512, 128, 288), (512, 256, 96),
    (1024, 128, 96), (1024, 256, 288), (2048, 128, 288), (2048, 256, 96),
]


def tanh_faces(ny: int, stretch: float = STRETCH) -> np.ndarray:
    """Face coordinates y_0..y_ny of the wall-clustered mesh on [0, 1]."""
    j = np.arange(ny + 1, dtype=np.float64)
    return 1.0 - np.tanh(stretch * (1.0 - j / ny)) / np.tanh(stretch)


def momentum_uniform(n: int, dt: float = DT, nu: float = NU):
    """Non-periodic uniform-mesh momentum line: a=c=-r, b=1+2r, a[0]=c[n-1]=0."""
    r = dt * nu * float(n) ** 2
    a = np.full(n, -r)
    c = np.full(n, -r)
    b = np.full(n, 1.0 + 2.0 * r)
    a[0] = 0.0
    c[-1] = 0.0
    return a, b, c


def momentum_periodic(n: int, dt: float = DT, nu: float = NU):
    """Periodic uniform-mesh momentum line; a[0] and c[n-1] are the wrap couplings."""
    r = dt * nu * float(n) ** 2
    return np.full(n, -r), np.full(n, 1.0 + 2.0 * r), np.full(n, -r)


def _centres(ny: int, stretch: float):
    yf = tanh_faces(ny, stretch)
    dy = np.diff(yf)                      # cell widths, length ny
    yc = 0.5 * (yf[:-1] + yf[1:])         # cell centres
    h = np.diff(yc)                       # centre-to-centre, length ny-1
    return dy, h


def momentum_stretched(ny: int, dt: float = DT, nu: float = NU, stretch: float = STRETCH):
    """Wall-normal momentum coefficients on the tanh mesh.

    a_j = -dt*nu/(dy_j h_{j-1/2}), c_j = -dt*nu/(dy_j h_{j+1/2}),
    b_j = 1 - a_j - c_j; the wall ghost distance is dy_0/2 (its coupling stays
    in b_0, a_0 = 0); the stress-free top has c_{ny-1} = 0 and no c term in b.
    """
    dy, h = _centres(ny, stretch)
    k = dt * nu
    a = np.zeros(ny)
    c = np.zeros(ny)
    a[1:] = -k / (dy[1:] * h)
    c[:-1] = -k / (dy[:-1] * h)
    a_wall = -k / (dy[0] * 0.5 * dy[0])
    b = 1.0 - a - c
    b[0] = 1.0 - a_wall - c[0]
    return a, b, c


def poisson_metric(ny: int, stretch: float = STRETCH):
    """Off-diagonals (ay, cy) of the cell-centred Neumann d2/dy2 on the tanh mesh."""
    dy, h = _centres(ny, stretch)
    ay = np.zeros(ny)
    cy = np.zeros(ny)
    ay[1:] = 1.0 / (dy[1:] * h)
    cy[:-1] = 1.0 / (dy[:-1] * h)
    return ay, cy


def modified_wavenumbers(nz: int, nk: int | None = None, lz: float = 1.0) -> np.ndarray:
    """lam_k = (4/dz^2) sin^2(pi k/nz), k = 0..nk-1 (default nk = nz//2 + 1)."""
    if nk is None:
        nk = nz // 2 + 1
    dz = lz / nz
    k = np.arange(nk, dtype=np.float64)
    return (4.0 / dz ** 2) * np.sin(np.pi * k / nz) ** 2


def spanwise_rfft(field_kji: np.ndarray) -> np.ndarray:
    """Real FFT along z (axis 0) of a [Nz][Ny][Nx] field -> [Nz/2+1][Ny][Nx] complex128."""
    return np.ascontiguousarray(np.fft.rfft(field_kji, axis=0))


def cfg_independent(nlines: int = 4096, n: int = 64, seed: int = 0,
                    rlo: float = 0.1, rhi: float = 10.0):
    """Independent diagonally dominant systems a=c=-r_s, b=1+2r_s, one r_s per line.

    Draw order: r[nlines] then d[nlines, n].  Returns (r, d_line_major) with
    d_line_major[s, j] the right-hand side of line s.
    """
    rng = np.random.default_rng(seed)
    r = rng.uniform(rlo, rhi, nlines)
    d = rng.uniform(-1.0, 1.0, (nlines, n))
    return r, d


def cfg_field(nx: int, ny: int, nz: int, seed: int = 0) -> np.ndarray:
    """N(0,1) field laid out [Nz][Ny][Nx] (x fastest)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nz, ny, nx))


def cfg_poisson_rhs(nx: int, ny: int, nz: int, seed: int = 0) -> np.ndarray:
    """Spanwise rFFT of an N(0,1) divergence field -> [Nz/2+1][Ny][Nx] complex128."""
    return spanwise_rfft(cfg_field(nx, ny, nz, seed))


def random_tridiag_nondominant(n: int, rng: np.random.Generator, periodic: bool = False):
    """Random non-symmetric rows far from diagonal dominance: |a|, |c| ~ U(0.5, 1) with
    random signs, b ~ U(-0.3, 0.3) and b = 0 on every 7th row (so an elimination without
    pivoting meets zero pivots); a[0], c[n-1] are zero unless periodic."""
    sa = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    sc = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    a = sa * rng.uniform(0.5, 1.0, n)
    c = sc * rng.uniform(0.5, 1.0, n)
    b = rng.uniform(-0.3, 0.3, n)
    b[::7] = 0.0
    if not periodic:
        a[0] = 0.0
        c[-1] = 0.0
    return a, b, c


def random_tridiag(n: int, rng: np.random.Generator, margin: float = 1.0,
                   periodic: bool = False):
    """Random non-symmetric strictly dominant row set: |b| = |a| + |c| + margin*U(0.5,1.5).

    a and c are drawn independently (so a transposed operand shows up), signs
    mixed; a[0], c[n-1] are zero unless periodic.
    """
    a = rng.uniform(-1.0, 1.0, n)
    c = rng.uniform(-1.0, 1.0, n)
    if not periodic:
        a[0] = 0.0
        c[-1] = 0.0
    sgn = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    b = sgn * (np.abs(a) + np.abs(c) + margin * rng.uniform(0.5, 1.5, n))
    return a, b, c


def pivot_probe(n: int, P: int, rng: np.random.Generator):
    """A line whose diagonal-pivoting elimination is exact in FP64 and whose pivot
    kinds are fixed by construction.

    Every partition (m = n/P rows, decoupled from its neighbours: a = 0 at its first
    row, c = 0 at its last) is a random sequence of
    * single rows: b = +-2^e (e in 0..3), a = +-2^k coupling back (0 at the
      partition's first row), c = 0;
    * pairs of rows t, t+1 with b_t = b_{t+1} = 0 and c_t, a_{t+1} = +-2^k, a_t
      coupling back, c_{t+1} coupling forward (0 at the partition's last row);
    with k in {-1, 0, 1} and integer right-hand sides in [-8, 8].  A pair's first
    row reaches elimination with a zero diagonal entry and so needs a 2x2 pivot;
    every other row is a 1x1 pivot.  Returns (a, b, c, d, pair_starts)."""
    m = n // P
    pow2 = lambda: float(rng.choice([-1.0, 1.0])) * 2.0 ** int(rng.integers(-1, 2))
    a = np.zeros(n)
    b = np.zeros(n)
    c = np.zeros(n)
    d = rng.integers(-8, 9, n).astype(np.float64)
    starts = []
    for r in range(P):
        t = 0
        while t < m:
            j = r * m + t
            if t + 1 < m and rng.uniform() < 0.5:
                c[j] = pow2()
                a[j + 1] = pow2()
                if t > 0:
                    a[j] = pow2()
                if t + 2 < m:
                    c[j + 1] = pow2()
                starts.append(j)
                t += 2
            else:
                b[j] = float(rng.choice([-1.0, 1.0])) * 2.0 ** int(rng.integers(0, 4))
                if t > 0:
                    a[j] = pow2()
                t += 1
    return a, b, c, d, starts
