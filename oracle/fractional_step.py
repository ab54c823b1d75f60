"""Semi-implicit fractional-step time step (Sec. 2.1-2.2), FP64, numpy + the oracle's solves.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper integrates the incompressible Navier-Stokes equations on a staggered
grid with second-order central differences: convection explicitly by a
low-storage third-order Runge-Kutta scheme, viscous terms implicitly by
Crank-Nicolson, the implicit operator approximately factored by ADI into one
tridiagonal system per direction and velocity component, and every sub-step
closed by the projection with the pseudo-pressure.  It prints neither the
Runge-Kutta coefficients nor the discrete operators; this module takes the
standard choices written out below (the readings are listed with the
library's design notes).

Grid: Nx x Ny x Nz cells, uniform dx and dz, wall-clustered cell widths dy_j.
    u[Nz][Ny][Nx+1] on x-faces (faces 0 and Nx are walls: u = 0),
    v[Nz][Ny+1][Nx] on y-faces (face 0: the no-slip wall, face Ny: the top;
                   v = 0 on both),
    w[Nz][Ny][Nx]   on z-faces (face k between cells k-1 and k, periodic).
Boundary conditions of the tangential components: no-slip at y = 0 (mirror
value -q at distance dy_0), stress-free at the top (zero flux), slip walls at
both x-ends (zero flux); z periodic.

Sub-step s = 1, 2, 3 (gamma = 8/15, 5/12, 3/4; zeta = 0, -17/60, -5/12;
alpha = gamma + zeta; beta = alpha dt nu / 2):

    N  = -div(u_i u_j)                      (of the field entering the sub-step)
    R  = dt (gamma_s N + zeta_s N_prev + alpha_s (nu L u - grad p))
    (1 - beta L_x)(1 - beta L_y)(1 - beta L_z) du = R    (x, then y, then z)
    u* = u + du
    u_new = u* - grad phi,   div grad phi = div u*   (the 3-D projection)
    p_new = p + phi / (alpha_s dt)

(the pressure enters the predictor as its previous value and is updated by
the pseudo-pressure increment, the incremental form of the Runge-Kutta
fractional step; p = 0 at the start)

The increments du live on [Nz][Ny][Nx] arrays: du[.., i] for x-faces
i = 0..Nx-1 and dv[:, j] for y-faces j = 0..Ny-1 (face 0 a wall: the row is
the identity with right-hand side 0; the far wall face is implicit zero).
"""
from __future__ import annotations

import numpy as np

from . import PDD, PPT, adi_sweep

GAMMA = (8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0)
ZETA = (0.0, -17.0 / 60.0, -5.0 / 12.0)
ALPHA = tuple(g + z for g, z in zip(GAMMA, ZETA))        # 8/15, 2/15, 1/3


# ---- second differences (the viscous operator L, Sec. 2.2) -------------------

def _hs(dy):
    """Distances between neighbouring cell centres h_{j+1/2}, j = 0..Ny-2."""
    return 0.5 * (dy[:-1] + dy[1:])


def lap_rows(kind: str, n: int, dx: float = 1.0, dy=None):
    """(lo, diag, up) of the 1-D second difference, one row per unknown of a line:
    row t reads lo_t q_{t-1} + diag_t q_t + up_t q_{t+1}.

    kind:
      'face_dirichlet_x' -- u along x: faces 0..n-1 (n = Nx), face 0 and face n are
                            walls (q = 0); row 0 is empty (the wall is held)
      'cell_slip_x'      -- v, w along x: cells, zero flux through both x-ends
      'cell_wall_y'      -- u, w along y: cells, mirror -q at the wall below cell 0,
                            zero flux through the top
      'face_dirichlet_y' -- v along y: faces 0..n-1 (n = Ny), walls at faces 0 and n
      'periodic_z'       -- every component along z (uniform, periodic)
    """
    lo, diag, up = np.zeros(n), np.zeros(n), np.zeros(n)
    if kind == "face_dirichlet_x":
        lo[1:] = up[1:] = 1.0 / dx ** 2
        diag[1:] = -2.0 / dx ** 2
        up[n - 1] = 0.0                       # couples to the wall face n (q = 0)
    elif kind in ("cell_slip_x", "periodic_z"):
        lo[:] = up[:] = 1.0 / dx ** 2
        if kind == "cell_slip_x":
            lo[0] = up[n - 1] = 0.0
        diag[:] = -(lo + up)
        if kind == "periodic_z":
            diag[:] = -2.0 / dx ** 2
    elif kind == "cell_wall_y":
        h = _hs(dy)
        lo[1:] = 1.0 / (dy[1:] * h)
        up[:-1] = 1.0 / (dy[:-1] * h)
        diag[:] = -(lo + up)
        diag[0] -= 2.0 / dy[0] ** 2           # mirror value -q_0 at distance dy_0 across the wall
    elif kind == "face_dirichlet_y":
        # face j between cells j-1 and j, h_j = (dy_{j-1} + dy_j)/2
        hj = 0.5 * (dy[:-1] + dy[1:])         # j = 1..n-1
        lo[1:] = 1.0 / (hj * dy[:-1])
        up[1:] = 1.0 / (hj * dy[1:])
        diag[1:] = -(lo[1:] + up[1:])
        up[n - 1] = 0.0                       # couples to the top face n (q = 0)
    else:
        raise ValueError(kind)
    return lo, diag, up


def _apply(q, rows, axis, periodic=False):
    """lo q_{t-1} + diag q_t + up q_{t+1} along `axis` (rows broadcast along it)."""
    lo, diag, up = rows
    q = np.moveaxis(q, axis, -1)
    qm, qp = np.roll(q, 1, -1), np.roll(q, -1, -1)
    if not periodic:
        qm[..., 0] = 0.0
        qp[..., -1] = 0.0
    return np.moveaxis(lo * qm + diag * q + up * qp, -1, axis)


def viscous(u, v, w, dx, dy, dz):
    """(Lu, Lv, Lw) on the interior unknowns, zero on the wall faces."""
    Nz, Ny, Nx = w.shape
    uu = u[:, :, :Nx]                         # faces 0..Nx-1 (face Nx is a wall)
    Lu = (_apply(uu, lap_rows("face_dirichlet_x", Nx, dx), 2)
          + _apply(uu, lap_rows("cell_wall_y", Ny, dy=dy), 1)
          + _apply(uu, lap_rows("periodic_z", Nz, dz), 0, periodic=True))
    Lu[:, :, 0] = 0.0
    vv = v[:, :Ny, :]                         # faces 0..Ny-1 (face Ny is the top)
    Lv = (_apply(vv, lap_rows("cell_slip_x", Nx, dx), 2)
          + _apply(vv, lap_rows("face_dirichlet_y", Ny, dy=dy), 1)
          + _apply(vv, lap_rows("periodic_z", Nz, dz), 0, periodic=True))
    Lv[:, 0, :] = 0.0
    Lw = (_apply(w, lap_rows("cell_slip_x", Nx, dx), 2)
          + _apply(w, lap_rows("cell_wall_y", Ny, dy=dy), 1)
          + _apply(w, lap_rows("periodic_z", Nz, dz), 0, periodic=True))
    return Lu, Lv, Lw


# ---- convection N = -d(u_i u_j)/dx_j, second-order central (Sec. 2.2) ---------

def _to_yface(q, dy):
    """Cell-centred (in y) q[Nz][Ny][.] linearly interpolated to the interior y-faces
    j = 1..Ny-1 (distance weighted on the stretched mesh); shape [Nz][Ny-1][.]."""
    a = dy[1:][None, :, None]                 # weight of q_{j-1} is dy_j
    b = dy[:-1][None, :, None]                # weight of q_j is dy_{j-1}
    return (a * q[:, :-1, :] + b * q[:, 1:, :]) / (a + b)


def convection(u, v, w, dx, dy, dz):
    """(Nu, Nv, Nw) on the layouts of the increments ([Nz][Ny][Nx]); zero on wall faces."""
    Nz, Ny, Nx = w.shape
    dyc = dy[None, :, None]
    # --- u on x-faces i = 1..Nx-1 ---
    uc = 0.5 * (u[:, :, :-1] + u[:, :, 1:])                       # cell centres [Nz][Ny][Nx]
    duu = (uc[:, :, 1:] ** 2 - uc[:, :, :-1] ** 2) / dx            # faces 1..Nx-1
    # flux u v at (x-face i, y-face j): u to the y-face, v to the x-face
    uy = _to_yface(u, dy)                                          # [Nz][Ny-1][Nx+1], faces j = 1..Ny-1
    vx = 0.5 * (v[:, 1:Ny, :-1] + v[:, 1:Ny, 1:])                  # [Nz][Ny-1][Nx-1], x-faces 1..Nx-1
    F = np.zeros((Nz, Ny + 1, Nx - 1))                             # y-faces 0..Ny (walls: v = 0)
    F[:, 1:Ny, :] = uy[:, :, 1:Nx] * vx
    duv = (F[:, 1:, :] - F[:, :-1, :]) / dyc
    # flux u w at (x-face i, z-face k)
    uz = 0.5 * (np.roll(u, 1, 0) + u)                              # u at z-face k
    wx = 0.5 * (w[:, :, :-1] + w[:, :, 1:])                        # w at x-faces 1..Nx-1
    G = uz[:, :, 1:Nx] * wx
    duw = (np.roll(G, -1, 0) - G) / dz
    Nu = np.zeros((Nz, Ny, Nx))
    Nu[:, :, 1:] = -(duu + duv + duw)
    # --- v on y-faces j = 1..Ny-1 ---
    vv_ = v[:, 1:Ny, :]                                            # faces 1..Ny-1 [Nz][Ny-1][Nx]
    # flux v u at (x-face i, y-face j): v to the x-face, u to the y-face; x-walls: u = 0
    H = np.zeros((Nz, Ny - 1, Nx + 1))
    H[:, :, 1:Nx] = 0.5 * (vv_[:, :, :-1] + vv_[:, :, 1:]) * uy[:, :, 1:Nx]
    dvu = (H[:, :, 1:] - H[:, :, :-1]) / dx
    vc = 0.5 * (v[:, :-1, :] + v[:, 1:, :])                        # cell centres [Nz][Ny][Nx]
    hj = 0.5 * (dy[:-1] + dy[1:])[None, :, None]
    dvv = (vc[:, 1:, :] ** 2 - vc[:, :-1, :] ** 2) / hj
    # flux v w at (y-face j, z-face k)
    vz = 0.5 * (np.roll(vv_, 1, 0) + vv_)
    wy = _to_yface(w, dy)                                          # [Nz][Ny-1][Nx]
    G = vz * wy
    dvw = (np.roll(G, -1, 0) - G) / dz
    Nv = np.zeros((Nz, Ny, Nx))
    Nv[:, 1:, :] = -(dvu + dvv + dvw)
    # --- w on z-faces ---
    # flux w u at (x-face i, z-face k): x-walls u = 0
    H = np.zeros((Nz, Ny, Nx + 1))
    H[:, :, 1:Nx] = 0.5 * (w[:, :, :-1] + w[:, :, 1:]) * uz[:, :, 1:Nx]
    dwu = (H[:, :, 1:] - H[:, :, :-1]) / dx
    # flux w v at (y-face j, z-face k): y-walls v = 0
    F = np.zeros((Nz, Ny + 1, Nx))
    F[:, 1:Ny, :] = wy * 0.5 * (np.roll(v[:, 1:Ny, :], 1, 0) + v[:, 1:Ny, :])
    dwv = (F[:, 1:, :] - F[:, :-1, :]) / dyc
    wc = 0.5 * (w + np.roll(w, -1, 0))                             # cell centres in z
    dww = (wc ** 2 - np.roll(wc, 1, 0) ** 2) / dz
    Nw = -(dwu + dwv + dww)
    return Nu, Nv, Nw


# ---- ADI coefficient rows of one sub-step ------------------------------------

def adi_rows(beta: float, Nx: int, Ny: int, Nz: int, dx: float, dy, dz: float):
    """{(component, direction): (a, b, c)} of (1 - beta L_d) for u, v, w and d = x, y, z."""
    def mk(rows):
        lo, diag, up = rows
        return -beta * lo, 1.0 - beta * diag, -beta * up
    z = mk(lap_rows("periodic_z", Nz, dz))
    return {("u", 0): mk(lap_rows("face_dirichlet_x", Nx, dx)), ("v", 0): mk(lap_rows("cell_slip_x", Nx, dx)),
            ("w", 0): mk(lap_rows("cell_slip_x", Nx, dx)),
            ("u", 1): mk(lap_rows("cell_wall_y", Ny, dy=dy)), ("v", 1): mk(lap_rows("face_dirichlet_y", Ny, dy=dy)),
            ("w", 1): mk(lap_rows("cell_wall_y", Ny, dy=dy)),
            ("u", 2): z, ("v", 2): z, ("w", 2): z}


def pressure_gradient(p, dx, dy, dz):
    """(G_x p, G_y p, G_z p) on the layouts of the increments; zero on wall faces."""
    Nz, Ny, Nx = p.shape
    Gu = np.zeros((Nz, Ny, Nx))
    Gu[:, :, 1:] = (p[:, :, 1:] - p[:, :, :-1]) / dx
    Gv = np.zeros((Nz, Ny, Nx))
    Gv[:, 1:, :] = (p[:, 1:, :] - p[:, :-1, :]) / (0.5 * (dy[:-1] + dy[1:]))[None, :, None]
    Gw = (p - np.roll(p, 1, 0)) / dz
    return Gu, Gv, Gw


def predictor(u, v, w, N_prev, s: int, dt: float, nu: float, dx: float, dy, dz: float,
              P=(8, 4, 16), method: int = PDD, convect: bool = True, p=None):
    """One sub-step up to the projection: returns (u*, v*, w*, N) with N the
    convection of the entering field (the next sub-step's N_prev).  p: the
    pressure of the previous sub-step (None: no pressure gradient term)."""
    Nz, Ny, Nx = w.shape
    N = convection(u, v, w, dx, dy, dz) if convect else (np.zeros((Nz, Ny, Nx)),) * 3
    L = viscous(u, v, w, dx, dy, dz)
    G = pressure_gradient(p, dx, dy, dz) if p is not None else (0.0, 0.0, 0.0)
    rows = adi_rows(ALPHA[s] * dt * nu / 2.0, Nx, Ny, Nz, dx, dy, dz)
    out = []
    for c, (q, Nq, Np, Lq, Gq) in enumerate(zip((u, v, w), N, N_prev, L, G)):
        R = dt * (GAMMA[s] * Nq + ZETA[s] * Np + ALPHA[s] * (nu * Lq - Gq))
        R = np.ascontiguousarray(R)
        for d in range(3):
            a, b, cc = rows[("uvw"[c], d)]
            adi_sweep(method, d, R, a, b, cc, P[d], d == 2)
        qs = q.copy()
        if c == 0:
            qs[:, :, :Nx] += R
        elif c == 1:
            qs[:, :Ny, :] += R
        else:
            qs += R
        out.append(qs)
    return out[0], out[1], out[2], N


def time_step(u, v, w, dt: float, nu: float, dx: float, dy, dz: float, P=(8, 4, 16), P_poisson: int = 8,
              method: int = PDD, project: bool = True, convect: bool = True, on_substep=None, p=None):
    """One time step (three sub-steps).  Returns (u, v, w, p); p (cells) is the
    pressure, p = 0 when None is given.  on_substep(s, u*, v*, w*, u, v, w) is
    called after each projection (for the pins)."""
    from .projection import project3d
    Nz, Ny, Nx = w.shape
    p = np.zeros((Nz, Ny, Nx)) if p is None else p
    N_prev = (np.zeros((Nz, Ny, Nx)),) * 3
    for s in range(3):
        us, vs, ws, N_prev = predictor(u, v, w, N_prev, s, dt, nu, dx, dy, dz, P, method, convect,
                                       p if project else None)
        if project:
            u, v, w, phi = project3d(us, vs, ws, dx, dy, dz, P=P_poisson, method=PPT)
            p = p + phi / (ALPHA[s] * dt)
        else:
            u, v, w = us, vs, ws
        if on_substep is not None:
            on_substep(s, us, vs, ws, u, v, w)
    return u, v, w, p
