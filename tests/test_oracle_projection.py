"""Pin of the Poisson wavenumber solves through the projection step.

After the spanwise FFT, the per-wavenumber wall-normal solves (PPT, k = 0
gauge pinned) and the inverse FFT, the gradient-corrected velocity must be
discretely divergence free to round-off (fractional step of Sec. 2.2).  A
wrong coefficient index, sign, wavenumber or gauge choice leaves an O(1)
divergence.
"""
import numpy as np
import pytest

import workloads as W


@pytest.mark.parametrize("P,method", [(4, "PPT"), (1, "EXACT"), (8, "PPT")])
def test_projection_divergence_free(orc, P, method):
    from oracle import projection
    Nz, Ny, Nx = 24, 32, 3
    rng = np.random.default_rng(2024)
    dy = np.diff(W.tanh_faces(Ny))
    dz = 1.0 / Nz
    v = rng.standard_normal((Nz, Ny + 1, Nx))
    v[:, 0, :] = 0.0
    v[:, Ny, :] = 0.0
    w = rng.standard_normal((Nz, Ny, Nx))
    div0 = np.max(np.abs(projection.divergence(v, w, dy, dz)))
    v1, w1, phi = projection.project(v, w, dy, dz, P=P, method=getattr(orc, method))
    div1 = np.max(np.abs(projection.divergence(v1, w1, dy, dz)))
    assert div0 > 10.0
    assert div1 <= 1e-13 * div0, (div1, div0)
    # walls untouched, k = 0 compatibility of the discrete divergence
    assert np.all(v1[:, 0, :] == 0) and np.all(v1[:, Ny, :] == 0)
    D = projection.divergence(v, w, dy, dz)
    assert abs(np.sum(D * dy[None, :, None])) < 1e-11 * np.sum(np.abs(D) * dy[None, :, None])


def test_projection_pdd_fails_at_low_k(orc):
    """The same projection with PDD (P = 4) leaves a visible divergence: the low
    wavenumber systems are too weakly dominant for the truncated Z."""
    from oracle import projection
    Nz, Ny, Nx = 24, 64, 2
    rng = np.random.default_rng(9)
    dy = np.diff(W.tanh_faces(Ny))
    dz = 1.0 / Nz
    v = rng.standard_normal((Nz, Ny + 1, Nx))
    v[:, 0, :] = v[:, Ny, :] = 0.0
    w = rng.standard_normal((Nz, Ny, Nx))
    div0 = np.max(np.abs(projection.divergence(v, w, dy, dz)))
    v1, w1, _ = projection.project(v, w, dy, dz, P=4, method=orc.PDD)
    assert np.max(np.abs(projection.divergence(v1, w1, dy, dz))) > 1e-6 * div0


# ---- the spanwise transform of the pressure step (Sec. 2.2) ---------------

@pytest.mark.parametrize("nz", [2, 6, 10, 24])
def test_spanwise_rfft_is_the_dft_sum(nz):
    """Brute force on tiny lines: X_k = sum_n x_n (cos(2 pi k n/N) - i sin(2 pi k n/N))."""
    import math
    from oracle import projection
    rng = np.random.default_rng(nz)
    x = rng.standard_normal((nz, 3))
    X = projection.spanwise_rfft(x)
    assert X.shape == (nz // 2 + 1, 3)
    for g in range(3):
        for k in range(nz // 2 + 1):
            re = sum(x[n, g] * math.cos(2 * math.pi * k * n / nz) for n in range(nz))
            im = -sum(x[n, g] * math.sin(2 * math.pi * k * n / nz) for n in range(nz))
            assert abs(X[k, g] - complex(re, im)) < 1e-13 * nz


@pytest.mark.parametrize("nz,q", [(288, 1), (288, 7), (96, 48), (120, 0)])
def test_spanwise_rfft_of_a_cosine(nz, q):
    """Closed form: cos(2 pi q n/N) has X_q = N/2 (N at q = 0 or N/2), all other modes 0;
    the inverse returns the cosine."""
    from oracle import projection
    n = np.arange(nz)
    x = np.cos(2 * np.pi * q * n / nz)[:, None]
    X = projection.spanwise_rfft(x)[:, 0]
    want = np.zeros(nz // 2 + 1, complex)
    want[q] = nz if q in (0, nz // 2) else nz / 2
    assert np.max(np.abs(X - want)) < 1e-12 * nz
    back = projection.spanwise_irfft(want[:, None], nz)[:, 0]
    assert np.max(np.abs(back - x[:, 0])) < 1e-14


def test_spanwise_rfft_parseval_and_round_trip():
    """sum x^2 = (|X_0|^2 + 2 sum_{0<k<N/2} |X_k|^2 + |X_{N/2}|^2)/N, and irfft(rfft x) = x."""
    from oracle import projection
    rng = np.random.default_rng(5)
    nz = 288
    x = rng.standard_normal((nz, 4))
    X = projection.spanwise_rfft(x)
    p = np.abs(X) ** 2
    energy = (p[0] + 2 * p[1:-1].sum(axis=0) + p[-1]) / nz
    assert np.allclose(energy, (x ** 2).sum(axis=0), rtol=1e-13)
    assert np.max(np.abs(projection.spanwise_irfft(X, nz) - x)) < 1e-14


# ---- shifted wall-normal systems (both homogeneous directions transformed) ----

@pytest.mark.parametrize("P,method,driver", [(P, m, d) for P, m in [(4, "PPT"), (8, "PPT"), (1, "EXACT")]
                                               for d in ("loop", "batch")] + [(1, "EXACT_LD", "batch")])
def test_shifted_poisson_manufactured_cosines(orc, P, method, driver):
    """Uniform Neumann mesh: cos(pi q (j + 1/2)/N) is an eigenvector of the cell-centred
    d2/dy2 with eigenvalue -(4/h^2) sin^2(pi q/(2N)); with the shift sigma the solution is
    d / (eigenvalue - sigma) for every line, whatever its shift.  Both drivers (the
    per-line Python loop and the C batch over every line) are held to it."""
    ny, h = 64, 1.0 / 64
    ay = np.full(ny, 1 / h ** 2)
    cy = np.full(ny, 1 / h ** 2)
    ay[0] = 0.0
    cy[-1] = 0.0
    rng = np.random.default_rng(11)
    lamz = rng.uniform(0.5, 3e4, 3)
    lamx = rng.uniform(0.5, 3e4, 5)
    j = np.arange(ny)
    ph = np.empty((3, ny, 5), complex)
    want = np.empty_like(ph)
    for k in range(3):
        for i in range(5):
            q, q2 = rng.integers(0, ny, 2)
            e1 = -(4 / h ** 2) * np.sin(np.pi * q / (2 * ny)) ** 2
            e2 = -(4 / h ** 2) * np.sin(np.pi * q2 / (2 * ny)) ** 2
            d1, d2 = np.cos(np.pi * q * (j + 0.5) / ny), np.cos(np.pi * q2 * (j + 0.5) / ny)
            sig = lamz[k] + lamx[i]
            ph[k, :, i] = d1 + 1j * d2
            want[k, :, i] = d1 / (e1 - sig) + 1j * d2 / (e2 - sig)
    fn = orc.poisson_shifted if driver == "loop" else orc.poisson_shifted_batch
    fn(ph, ay, cy, lamz, lamx, P, getattr(orc, method))
    assert np.max(np.abs(ph - want)) <= 1e-12 * np.max(np.abs(want))


def test_shifted_poisson_gauge_pinned_line(orc):
    """The line with zero shift: x_0 = 0 and the other rows of A x = d hold; other lines
    are untouched by the pin (same as the unshifted solve where lamx = 0)."""
    import workloads as W
    ny = 32
    ay, cy = W.poisson_metric(ny)
    lamz = W.modified_wavenumbers(12)           # lamz_0 = 0
    lamx = np.zeros(4)
    rng = np.random.default_rng(2)
    ph = rng.standard_normal((7, ny, 4)) + 1j * rng.standard_normal((7, ny, 4))
    ref = ph.copy()
    orc.poisson(ref, ay, cy, lamz, P=4)
    got = ph.copy()
    orc.poisson_shifted(got, ay, cy, lamz, lamx, 4)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.all(got[0, 0, :] == 0)
    got_b = ph.copy()
    orc.poisson_shifted_batch(got_b, ay, cy, lamz, lamx, 4)
    assert np.array_equal(got_b, got)           # same arithmetic, line by line


# ---- the 3-D step: cosine transform in x -------------------------------------

@pytest.mark.parametrize("nx", [2, 6, 10, 24])
def test_streamwise_dct_is_the_cosine_sum(nx):
    import math
    from oracle import projection
    rng = np.random.default_rng(nx)
    x = rng.standard_normal((3, nx)) + 1j * rng.standard_normal((3, nx))
    X = projection.streamwise_dct(x)
    for r in range(3):
        for k in range(nx):
            want = sum(x[r, n] * math.cos(math.pi * k * (2 * n + 1) / (2 * nx)) for n in range(nx))
            assert abs(X[r, k] - want) < 1e-13 * nx
    assert np.max(np.abs(projection.streamwise_idct(X) - x)) < 1e-14


@pytest.mark.parametrize("nx,q", [(2048, 0), (2048, 5), (96, 95)])
def test_streamwise_dct_of_a_cosine_mode(nx, q):
    """cos(pi q (n + 1/2)/N) transforms to N/2 at k = q (N at q = 0) and 0 elsewhere."""
    from oracle import projection
    n = np.arange(nx)
    X = projection.streamwise_dct(np.cos(np.pi * q * (n + 0.5) / nx))
    want = np.zeros(nx)
    want[q] = nx if q == 0 else nx / 2
    assert np.max(np.abs(X - want)) < 1e-12 * nx


@pytest.mark.parametrize("P,method", [(8, "PPT"), (4, "PPT"), (1, "EXACT")])
def test_projection3d_divergence_free(orc, P, method):
    """x, y and z corrections together: the 3-D divergence vanishes to round-off;
    wall faces (x-ends, y-walls) are untouched."""
    from oracle import projection
    nx, ny, nz = 12, 32, 10
    rng = np.random.default_rng(31)
    dy = np.diff(W.tanh_faces(ny))
    dx, dz = 1.0 / nx, 1.0 / nz
    u = rng.standard_normal((nz, ny, nx + 1))
    u[:, :, 0] = u[:, :, nx] = 0.0
    v = rng.standard_normal((nz, ny + 1, nx))
    v[:, 0, :] = v[:, ny, :] = 0.0
    w = rng.standard_normal((nz, ny, nx))
    div0 = np.max(np.abs(projection.divergence3d(u, v, w, dx, dy, dz)))
    u1, v1, w1, phi = projection.project3d(u, v, w, dx, dy, dz, P=P, method=getattr(orc, method))
    assert div0 > 10
    assert np.max(np.abs(projection.divergence3d(u1, v1, w1, dx, dy, dz))) <= 1e-13 * div0
    assert np.all(u1[:, :, 0] == 0) and np.all(u1[:, :, nx] == 0)
    assert np.all(v1[:, 0, :] == 0) and np.all(v1[:, ny, :] == 0)
