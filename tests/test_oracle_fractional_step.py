"""Pins of the fractional-step oracle (oracle/fractional_step.py; Sec. 2.1-2.2:
staggered grid, second-order central differences, low-storage RK3 convection,
Crank-Nicolson viscous terms by ADI, projection).

What pins it, none of it the oracle's own formulas:
* every 1-D second difference has the closed-form eigenvectors of its boundary
  conditions on a uniform mesh (sine, cosine, quarter-wave, circulant modes);
  on the stretched mesh it is self-adjoint in the cell-width inner product and
  conserves the integral up to the wall flux;
* convection and viscous terms converge at second order to the analytic
  -d(u_i u_j)/dx_j and Laplacian of smooth fields that satisfy the boundary
  conditions, on uniform and stretched meshes;
* with convection off, a product of eigenvectors (no divergence) is multiplied
  per sub-step by exactly the ADI Crank-Nicolson factor
  1 + 2 beta lam / prod_d (1 - beta lam_d);
* with viscosity and projection off, the Runge-Kutta scheme converges at third
  order in time;
* the full step leaves the velocity divergence free to 1e-13 of the
  predictor's divergence after every sub-step, holds the wall faces at zero,
  and converges at second order in time.
"""
import numpy as np
import pytest

import workloads as W

EPS = np.finfo(float).eps


@pytest.fixture(scope="module")
def fs(orc):
    from oracle import fractional_step
    return fractional_step


def _dense(rows, periodic=False):
    lo, diag, up = rows
    n = diag.size
    A = np.diag(diag) + np.diag(lo[1:], -1) + np.diag(up[:-1], 1)
    if periodic:
        A[0, -1] += lo[0]
        A[-1, 0] += up[-1]
    return A


@pytest.mark.parametrize("n", [8, 12, 32])
def test_second_differences_have_the_closed_form_eigenvectors(fs, n):
    h = 1.0 / n
    i = np.arange(n)
    for p in range(1, n):
        lam = -(4 / h ** 2) * np.sin(np.pi * p / (2 * n)) ** 2
        # u along x on faces 1..n-1 (walls at 0 and n): sin(pi p i / n)
        A = _dense(fs.lap_rows("face_dirichlet_x", n, h))
        q = np.sin(np.pi * p * i / n)
        assert np.allclose((A @ q)[1:], lam * q[1:], atol=1e-9 * abs(lam))
        # v along y on a uniform mesh: the same modes
        A = _dense(fs.lap_rows("face_dirichlet_y", n, dy=np.full(n, h)))
        assert np.allclose((A @ q)[1:], lam * q[1:], atol=1e-9 * abs(lam))
    for p in range(n):
        lam = -(4 / h ** 2) * np.sin(np.pi * p / (2 * n)) ** 2
        # cell-centred, zero flux at both ends: cos(pi p (i + 1/2) / n)
        q = np.cos(np.pi * p * (i + 0.5) / n)
        A = _dense(fs.lap_rows("cell_slip_x", n, h))
        assert np.allclose(A @ q, lam * q, atol=1e-9 * max(1.0, abs(lam)))
        # cell-centred, wall (q = 0) below, zero flux at the top: sin(pi (p + 1/2)(i + 1/2) / n)
        lw = -(4 / h ** 2) * np.sin(np.pi * (p + 0.5) / (2 * n)) ** 2
        q = np.sin(np.pi * (p + 0.5) * (i + 0.5) / n)
        A = _dense(fs.lap_rows("cell_wall_y", n, dy=np.full(n, h)))
        assert np.allclose(A @ q, lw * q, atol=1e-9 * abs(lw))
        # periodic: cos(2 pi p i / n)
        lp = -(4 / h ** 2) * np.sin(np.pi * p / n) ** 2
        q = np.cos(2 * np.pi * p * i / n)
        A = _dense(fs.lap_rows("periodic_z", n, h), periodic=True)
        assert np.allclose(A @ q, lp * q, atol=1e-9 * max(1.0, abs(lp)))


def test_stretched_second_differences_are_conservative_and_self_adjoint(fs):
    ny = 48
    dy = np.diff(W.tanh_faces(ny))
    rng = np.random.default_rng(1)
    q = rng.standard_normal(ny)
    # cells: symmetric in the dy-weighted product; sum dy (L q) = wall flux only
    A = _dense(fs.lap_rows("cell_wall_y", ny, dy=dy))
    Dw = np.diag(dy)
    assert np.allclose(Dw @ A, (Dw @ A).T, rtol=1e-13, atol=0)
    assert np.isclose(dy @ (A @ q), -2.0 * q[0] / dy[0], rtol=1e-11)
    # faces 1..ny-1 (walls at 0 and ny): symmetric in the h-weighted product
    A = _dense(fs.lap_rows("face_dirichlet_y", ny, dy=dy))[1:, 1:]
    Dh = np.diag(0.5 * (dy[:-1] + dy[1:]))
    assert np.allclose(Dh @ A, (Dh @ A).T, rtol=1e-13, atol=0)


def _fields(Nx, Ny, Nz, dy):
    """Smooth fields with the boundary conditions of the grid and their analytic
    derivatives.  x in [0, 1] (walls), y in [0, 1] (no-slip / top), z periodic."""
    xf = np.arange(Nx + 1) / Nx                  # x-faces
    xc = (np.arange(Nx) + 0.5) / Nx
    yf = np.concatenate([[0.0], np.cumsum(dy)])  # y-faces
    yc = 0.5 * (yf[:-1] + yf[1:])
    zf = np.arange(Nz) / Nz                      # z-faces
    zc = (np.arange(Nz) + 0.5) / Nz
    tp = 2 * np.pi
    # u = sin(pi x) sin(pi y/2) (1 + 0.5 cos 2pi z): zero at the x-walls, no-slip, stress-free top
    U = lambda x, y, z: np.sin(np.pi * x) * np.sin(np.pi * y / 2) * (1 + 0.5 * np.cos(tp * z))
    # v = cos(pi x) sin(pi y) (1 + 0.3 sin 2pi z): zero at both y-walls, slip at x-ends
    V = lambda x, y, z: np.cos(np.pi * x) * np.sin(np.pi * y) * (1 + 0.3 * np.sin(tp * z))
    # w = cos(pi x) sin(pi y/2) cos(2 pi z): slip at x-ends, no-slip, stress-free top
    Wf = lambda x, y, z: np.cos(np.pi * x) * np.sin(np.pi * y / 2) * np.cos(tp * z)
    g = lambda fx, fy, fz: np.meshgrid(fz, fy, fx, indexing="ij")[::-1]
    Xu, Yu, Zu = g(xf, yc, zc)
    Xv, Yv, Zv = g(xc, yf, zc)
    Xw, Yw, Zw = g(xc, yc, zf)
    return (U, V, Wf), (U(Xu, Yu, Zu), V(Xv, Yv, Zv), Wf(Xw, Yw, Zw)), ((Xu, Yu, Zu), (Xv, Yv, Zv), (Xw, Yw, Zw))


def _analytic(funcs, pts, h=1e-5):
    """-d(u_i u_j)/dx_j and the Laplacian at the points, by central differences of the
    analytic functions with a tiny step (fourth-order Richardson)."""
    U, V, Wf = funcs
    comps = (U, V, Wf)

    def d(f, X, Y, Z, ax):
        e = [np.zeros_like(X) for _ in range(3)]
        def at(s):
            e2 = [X, Y, Z]
            e2 = [c + (s * h if k == ax else 0.0) for k, c in enumerate(e2)]
            return f(*e2)
        return (8 * (at(1) - at(-1)) - (at(2) - at(-2))) / (12 * h)

    def d2(f, X, Y, Z, ax):
        def at(s):
            e2 = [X, Y, Z]
            e2 = [c + (s * h * 100 if k == ax else 0.0) for k, c in enumerate(e2)]
            return f(*e2)
        hh = 100 * h
        return (-at(2) + 16 * at(1) - 30 * at(0) + 16 * at(-1) - at(-2)) / (12 * hh ** 2)

    conv, lap = [], []
    for c, (X, Y, Z) in enumerate(pts):
        total = 0.0
        for j in range(3):
            prod = lambda x, y, z, c=c, j=j: comps[c](x, y, z) * comps[j](x, y, z)
            total = total + d(prod, X, Y, Z, j)
        conv.append(-total)
        lap.append(sum(d2(comps[c], X, Y, Z, ax) for ax in range(3)))
    return conv, lap


@pytest.mark.parametrize("stretched", [False, True])
def test_convection_and_viscous_terms_converge_at_second_order(fs, stretched):
    errs_c, errs_l = [], []
    for n in (16, 32, 64):
        Nx, Ny, Nz = n, n, n
        dy = np.diff(W.tanh_faces(Ny, 1.2)) if stretched else np.full(Ny, 1.0 / Ny)
        funcs, (u, v, w), pts = _fields(Nx, Ny, Nz, dy)
        Nu, Nv, Nw = fs.convection(u, v, w, 1.0 / Nx, dy, 1.0 / Nz)
        Lu, Lv, Lw = fs.viscous(u, v, w, 1.0 / Nx, dy, 1.0 / Nz)
        conv, lap = _analytic(funcs, pts)
        # compare on the interior unknowns (faces 1..Nx-1 for u, 1..Ny-1 for v); rows next
        # to a boundary are first-order accurate in a staggered scheme, so skip one layer
        sl_u = (slice(None), slice(1, Ny - 1), slice(2, Nx - 1))
        sl_v = (slice(None), slice(2, Ny - 1), slice(1, Nx - 1))
        sl_w = (slice(None), slice(1, Ny - 1), slice(1, Nx - 1))
        ec = max(np.max(np.abs(Nu[sl_u] - conv[0][:, :, :Nx][sl_u])),
                 np.max(np.abs(Nv[sl_v] - conv[1][:, :Ny, :][sl_v])),
                 np.max(np.abs(Nw[sl_w] - conv[2][sl_w])))
        el = max(np.max(np.abs(Lu[sl_u] - lap[0][:, :, :Nx][sl_u])),
                 np.max(np.abs(Lv[sl_v] - lap[1][:, :Ny, :][sl_v])),
                 np.max(np.abs(Lw[sl_w] - lap[2][sl_w])))
        errs_c.append(ec)
        errs_l.append(el)
    oc = np.log2(np.array(errs_c[:-1]) / np.array(errs_c[1:]))
    ol = np.log2(np.array(errs_l[:-1]) / np.array(errs_l[1:]))
    assert np.all(oc > 1.8), (errs_c, oc)
    assert np.all(ol > 1.8), (errs_l, ol)


def _grid(Nx, Ny, Nz, stretch=2.5):
    return 1.0 / Nx, np.diff(W.tanh_faces(Ny, stretch)), 1.0 / Nz


def _eigvec(A, weights, which):
    """Eigenpair of a (weight-symmetric) tridiagonal operator, by index of |eigenvalue|."""
    s = np.sqrt(weights)
    B = (A * s[:, None]) / s[None, :]
    lam, V = np.linalg.eigh(0.5 * (B + B.T))
    order = np.argsort(np.abs(lam))
    k = order[which]
    return lam[k], V[:, k] / s


@pytest.mark.parametrize("comp", ["u", "v", "w"])
def test_diffusion_mode_decays_by_the_adi_crank_nicolson_factor(fs, orc, comp):
    """Convection off: an eigenvector of L_x L_y (constant in z) is multiplied per
    sub-step by exactly 1 + 2 beta lam / ((1 - beta lam_x)(1 - beta lam_y)), beta =
    alpha_s dt nu / 2, lam = lam_x + lam_y (the w mode has no divergence, so the
    projection leaves it as it is; u and v are checked before the projection)."""
    Nx, Ny, Nz = 16, 24, 8
    dx, dy, dz = _grid(Nx, Ny, Nz)
    dt, nu = 0.02, 0.05
    u = np.zeros((Nz, Ny, Nx + 1)); v = np.zeros((Nz, Ny + 1, Nx)); w = np.zeros((Nz, Ny, Nx))
    i = np.arange(Nx)
    if comp == "u":
        p = 3
        X = np.sin(np.pi * p * i / Nx)                               # faces 0..Nx-1 (0 at the wall)
        lx = -(4 / dx ** 2) * np.sin(np.pi * p / (2 * Nx)) ** 2
        ly, Y = _eigvec(_dense(fs.lap_rows("cell_wall_y", Ny, dy=dy)), dy, 2)
        u[:, :, :Nx] = X[None, None, :] * Y[None, :, None]
        q0 = u.copy()
    elif comp == "v":
        p = 2
        X = np.cos(np.pi * p * (i + 0.5) / Nx)
        lx = -(4 / dx ** 2) * np.sin(np.pi * p / (2 * Nx)) ** 2
        A = _dense(fs.lap_rows("face_dirichlet_y", Ny, dy=dy))[1:, 1:]
        ly, Yi = _eigvec(A, 0.5 * (dy[:-1] + dy[1:]), 1)
        Y = np.concatenate([[0.0], Yi])                               # face 0 is the wall
        v[:, :Ny, :] = Y[None, :, None] * X[None, None, :]
        q0 = v.copy()
    else:
        p = 5
        X = np.cos(np.pi * p * (i + 0.5) / Nx)
        lx = -(4 / dx ** 2) * np.sin(np.pi * p / (2 * Nx)) ** 2
        ly, Y = _eigvec(_dense(fs.lap_rows("cell_wall_y", Ny, dy=dy)), dy, 0)
        w[:] = Y[None, :, None] * X[None, None, :]
        q0 = w.copy()
    lam = lx + ly
    g = 1.0
    N0 = (np.zeros((Nz, Ny, Nx)),) * 3
    q = (u, v, w)
    for s in range(3):
        beta = fs.ALPHA[s] * dt * nu / 2
        g *= 1 + 2 * beta * lam / ((1 - beta * lx) * (1 - beta * ly))
        if comp == "w":
            q = fs.time_step(*q, dt, nu, dx, dy, dz, P=(4, 4, 2), P_poisson=4, method=orc.PPT,
                             convect=False)[:3] if s == 0 else q
        else:
            q = fs.predictor(*q, N0, s, dt, nu, dx, dy, dz, P=(4, 4, 2), method=orc.PPT, convect=False)[:3]
    got = q["uvw".index(comp)]
    assert 0.05 < abs(g) < 0.999                                     # a real decay, not the identity
    assert np.max(np.abs(got - g * q0)) <= 1e-12 * np.max(np.abs(q0)), np.max(np.abs(got - g * q0))


def _smooth_state(Nx, Ny, Nz, dy, amp=1.0):
    _, (u, v, w), _ = _fields(Nx, Ny, Nz, dy)
    return amp * u, amp * v, amp * w


def test_runge_kutta_convection_is_third_order(fs, orc):
    """Viscosity and projection off: the three sub-steps integrate dq/dt = N(q) at
    third order (self-convergence over dt, dt/2, dt/4, dt/8)."""
    Nx, Ny, Nz = 16, 16, 8
    dx, dy, dz = _grid(Nx, Ny, Nz, 1.5)
    u0, v0, w0 = _smooth_state(Nx, Ny, Nz, dy)
    T_end = 0.08
    res = []
    for nsteps in (2, 4, 8, 16):
        dt = T_end / nsteps
        q = (u0, v0, w0)
        for _ in range(nsteps):
            q = fs.time_step(*q, dt, 0.0, dx, dy, dz, P=(4, 4, 2), method=orc.PPT, project=False)[:3]
        res.append(np.concatenate([x.ravel() for x in q]))
    d = [np.max(np.abs(res[k] - res[k + 1])) for k in range(3)]
    orders = np.log2(np.array(d[:-1]) / np.array(d[1:]))
    assert np.all(orders > 2.7), (d, orders)


def test_full_step_is_divergence_free_after_every_substep(fs, orc):
    Nx, Ny, Nz = 16, 24, 12
    dx, dy, dz = _grid(Nx, Ny, Nz)
    rng = np.random.default_rng(4)
    u = 0.3 * rng.standard_normal((Nz, Ny, Nx + 1)); u[:, :, 0] = u[:, :, -1] = 0
    v = 0.3 * rng.standard_normal((Nz, Ny + 1, Nx)); v[:, 0, :] = v[:, -1, :] = 0
    w = 0.3 * rng.standard_normal((Nz, Ny, Nx))
    from oracle.projection import divergence3d
    seen = []

    def check(s, us, vs, ws, un, vn, wn):
        d0 = np.max(np.abs(divergence3d(us, vs, ws, dx, dy, dz)))
        d1 = np.max(np.abs(divergence3d(un, vn, wn, dx, dy, dz)))
        seen.append(s)
        assert d0 > 1.0 and d1 <= 1e-13 * d0, (s, d0, d1)
        assert np.all(un[:, :, 0] == 0) and np.all(un[:, :, -1] == 0)       # wall faces held
        assert np.all(vn[:, 0, :] == 0) and np.all(vn[:, -1, :] == 0)
    fs.time_step(u, v, w, 2e-3, 1e-2, dx, dy, dz, P=(4, 4, 4), P_poisson=4, on_substep=check)
    assert seen == [0, 1, 2]


def test_full_step_converges_in_time(fs, orc):
    """Everything on (convection, Crank-Nicolson ADI, the previous pressure in the
    predictor, projection) from a smooth divergence-free state: second order in
    time (self-convergence over dt, dt/2, dt/4, dt/8; without the pressure term
    the splitting error at the walls leaves about first order)."""
    Nx, Ny, Nz = 16, 16, 8
    dx, dy, dz = _grid(Nx, Ny, Nz, 1.5)
    from oracle.projection import project3d
    u0, v0, w0, _ = project3d(*_smooth_state(Nx, Ny, Nz, dy), dx, dy, dz, P=4)
    T_end, nu = 0.08, 0.02
    res = []
    for nsteps in (2, 4, 8, 16):
        dt = T_end / nsteps
        q, p = (u0, v0, w0), None
        for _ in range(nsteps):
            *q, p = fs.time_step(*q, dt, nu, dx, dy, dz, P=(4, 4, 2), P_poisson=4, method=orc.PPT, p=p)
        res.append(np.concatenate([x.ravel() for x in q]))
    d = [np.max(np.abs(res[k] - res[k + 1])) for k in range(3)]
    orders = np.log2(np.array(d[:-1]) / np.array(d[1:]))
    assert np.all(orders > 1.8), (d, orders)
