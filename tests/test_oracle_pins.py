"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test names what it pins: dense LU / exact rationals (plain definition of
x = A^{-1} d), the paper's printed n = 12, p = 4 example (index bookkeeping of
Sec. 3.2), closed forms (Toeplitz spikes, sinusoidal eigenvectors), the PDD
truncation bound, and the two accuracy statements of Sec. 3.2 (PDD for the
momentum sweeps, PDD versus PPT for the Poisson solves).
"""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from conftest import load_golden


def dense(a, b, c, periodic=False):
    n = len(b)
    A = np.diag(np.asarray(b, float))
    if n > 1:
        A += np.diag(np.asarray(a, float)[1:], -1) + np.diag(np.asarray(c, float)[:-1], 1)
    if periodic:
        A[0, -1] += a[0]
        A[-1, 0] += c[-1]
    return A


def relerr(x, ref):
    return float(np.max(np.abs(x - ref)) / max(np.max(np.abs(ref)), 1e-300))


# --------------------------------------------------------------------------
# Plain definition: x = A^{-1} d
# --------------------------------------------------------------------------
@pytest.mark.parametrize("n", [1, 2, 3, 5, 12, 64, 257])
def test_thomas_matches_dense_lu(orc, n):
    rng = np.random.default_rng(100 + n)
    a, b, c = W.random_tridiag(n, rng)
    d = rng.uniform(-1, 1, n)
    x = orc.thomas(a, b, c, d)
    assert relerr(x, np.linalg.solve(dense(a, b, c), d)) < 1e-14


def _exact_fraction_solve(A, d):
    """Gaussian elimination in exact rational arithmetic on the FP64 inputs."""
    n = len(d)
    M = [[Fraction(float(A[i, j])) for j in range(n)] + [Fraction(float(d[i]))] for i in range(n)]
    for k in range(n):
        p = next(i for i in range(k, n) if M[i][k] != 0)
        M[k], M[p] = M[p], M[k]
        for i in range(k + 1, n):
            f = M[i][k] / M[k][k]
            if f:
                M[i] = [M[i][t] - f * M[k][t] for t in range(n + 1)]
    x = [Fraction(0)] * n
    for k in range(n - 1, -1, -1):
        s = M[k][n] - sum(M[k][t] * x[t] for t in range(k + 1, n))
        x[k] = s / M[k][k]
    return np.array([float(v) for v in x])


@pytest.mark.parametrize("periodic", [False, True])
def test_exact_rational_small(orc, periodic):
    rng = np.random.default_rng(7)
    n = 12
    a, b, c = W.random_tridiag(n, rng, periodic=periodic)
    d = rng.uniform(-1, 1, n)
    xr = _exact_fraction_solve(dense(a, b, c, periodic), d)
    assert relerr(orc.exact(a, b, c, d, periodic), xr) < 1e-15
    for P in (1, 2, 3, 4, 6):
        assert relerr(orc.ppt(a, b, c, d, P, periodic), xr) < 4e-15, P


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("n,P", [(12, 4), (64, 4), (64, 8), (96, 16), (90, 5), (288, 4), (256, 2)])
def test_ppt_is_exact_at_every_P(orc, n, P, periodic):
    """Eqs. (9)-(11) are an identity: PPT equals A^{-1} d for any partition count."""
    rng = np.random.default_rng(n * 31 + P)
    a, b, c = W.random_tridiag(n, rng, margin=0.3, periodic=periodic)
    d = rng.uniform(-1, 1, n)
    ref = np.linalg.solve(dense(a, b, c, periodic), d)
    assert relerr(orc.ppt(a, b, c, d, P, periodic), ref) < 1e-13


@pytest.mark.parametrize("periodic", [False, True])
def test_exact_ld_matches_rationals(orc, periodic):
    """The extended-precision solve is the reference for refinement: pinned to
    exact rational elimination, and (well conditioned) to the FP64 solve."""
    rng = np.random.default_rng(17)
    n = 12
    a, b, c = W.random_tridiag(n, rng, margin=0.05, periodic=periodic)
    d = rng.uniform(-1, 1, n)
    xr = _exact_fraction_solve(dense(a, b, c, periodic), d)
    assert relerr(orc.exact_ld(a, b, c, d, periodic), xr) < 2e-16
    a, b, c = W.random_tridiag(200, rng, periodic=periodic)
    d = rng.uniform(-1, 1, 200)
    assert relerr(orc.exact_ld(a, b, c, d, periodic), orc.exact(a, b, c, d, periodic)) < 1e-14


def test_exact_ld_beats_fp64_on_ill_conditioned(orc):
    """On a near-singular Neumann operator (cond ~ 1e8) the FP64 and long-double
    solves differ by far more than the long-double solve differs from exact
    rationals: the extended reference resolves what FP64 cannot."""
    n = 10
    eps = 1e-7
    a = np.full(n, -1.0); c = np.full(n, -1.0); b = np.full(n, 2.0 + eps)
    a[0] = c[-1] = 0.0
    b[0] = b[-1] = 1.0 + eps
    d = np.cos(np.arange(n) * 0.7)
    xr = _exact_fraction_solve(dense(a, b, c), d)
    e_ld = relerr(orc.exact_ld(a, b, c, d), xr)
    e_64 = relerr(orc.thomas(a, b, c, d), xr)
    assert e_ld < 1e-12 and e_ld < e_64 / 50


def test_cyclic_matches_dense(orc):
    rng = np.random.default_rng(3)
    for n in (3, 4, 17, 288):
        a, b, c = W.random_tridiag(n, rng, periodic=True)
        d = rng.uniform(-1, 1, n)
        assert relerr(orc.cyclic(a, b, c, d), np.linalg.solve(dense(a, b, c, True), d)) < 1e-14


def test_ppt_non_dominant_blocks(orc):
    """PPT makes no approximation (Sec. 3.2): exact on a matrix far from dominance
    whose partition blocks stay non-singular without pivoting."""
    rng = np.random.default_rng(11)
    n = 48
    a = rng.uniform(-1, 1, n)
    c = rng.uniform(-1, 1, n)
    a[0] = c[-1] = 0
    b = 0.6 * (np.abs(a) + np.abs(c)) + 0.4 + rng.uniform(0, 0.2, n)
    d = rng.uniform(-1, 1, n)
    ref = np.linalg.solve(dense(a, b, c), d)
    for P in (2, 4, 8):
        assert relerr(orc.ppt(a, b, c, d, P), ref) < 1e-11


# --------------------------------------------------------------------------
# Index bookkeeping: the paper's printed n = 12, p = 4 example
# --------------------------------------------------------------------------
def _symbol_value(sym, rs, m):
    if sym in (".", "0"):
        return 0.0
    if sym == "1":
        return 1.0
    name, part = sym.split("_")
    r = int(part)
    pos = {"1": 0, "2": 1, "m": m - 1}[name[1:]]
    vec = rs["v"] if name[0] == "v" else rs["w"]
    return vec[r * m + pos]


def test_reduced_system_matches_printed_example(orc):
    g = load_golden("sec32_example_n12_p4.txt")
    n, P, m = 12, 4, 3
    rng = np.random.default_rng(12)
    a, b, c = W.random_tridiag(n, rng)
    d = rng.uniform(-1, 1, n)
    rs = orc.reduced_system(a, b, c, d, P)
    Z_gold = np.array([[_symbol_value(s, rs, m) for s in row] for row in g["Z"]])
    Zb_gold = np.array([[_symbol_value(s, rs, m) for s in row] for row in g["Zbar"]])
    # every printed entry, value for value (the spikes themselves are pinned below)
    assert np.array_equal(rs["Z"], Z_gold)
    assert np.array_equal(rs["Zbar"], Zb_gold)
    # Zbar = Z P with the printed P
    Pm = np.array([[1.0 if s == "1" else 0.0 for s in row] for row in g["P"]])
    assert np.array_equal(rs["Z"] @ Pm, rs["Zbar"])
    assert np.array_equal(Pm @ Pm, np.eye(6))
    # E^T x~ picks the printed columns
    cols = [int(t) - 1 for t in g["ET_cols"][0]]
    assert np.array_equal(rs["rhs"], rs["xt"][cols])
    # Y = A~^{-1} V reproduces the printed spike layout, and with the printed
    # Delta A and E^T columns: A = A~ + V E^T and A~ Y = V
    Y = np.array([[_symbol_value(s, rs, m) for s in row] for row in g["Y"]])
    dA = np.zeros((n, n))
    V = np.zeros((n, 6))
    A = dense(a, b, c)
    for row, col, sym in g["DeltaA"]:
        i, j = int(row) - 1, int(col) - 1
        dA[i, j] = A[i, j]
        V[i, cols.index(j)] = A[i, j]
    At = A - dA
    ET = np.zeros((6, n))
    ET[range(6), cols] = 1.0
    assert np.array_equal(V @ ET, dA)
    assert np.allclose(At @ Y, V, atol=1e-15)
    assert np.allclose(At @ rs["xt"], d, atol=1e-15)
    assert np.allclose(np.eye(6) + ET @ Y, rs["Z"], atol=0)


def test_zbar_tridiagonal_general_P(orc):
    rng = np.random.default_rng(5)
    for P in (2, 3, 5, 8, 16):
        n = 4 * P
        a, b, c = W.random_tridiag(n, rng)
        rs = orc.reduced_system(a, b, c, rng.uniform(-1, 1, n), P)
        Zb = rs["Zbar"]
        K = Zb.shape[0]
        assert K == 2 * (P - 1)
        band = np.abs(np.subtract.outer(np.arange(K), np.arange(K))) <= 1
        assert np.all(Zb[~band] == 0)
        # off-diagonal ones of Zbar sit between the two unknowns of an interface
        for i in range(P - 1):
            assert Zb[2 * i, 2 * i + 1] == 1.0 and Zb[2 * i + 1, 2 * i] == 1.0


def test_periodic_reduced_system_cyclic(orc):
    """Periodic lines: the wrap interface makes Z 2P x 2P and Zbar cyclic tridiagonal."""
    rng = np.random.default_rng(6)
    P = 4
    n = 20
    a, b, c = W.random_tridiag(n, rng, periodic=True)
    d = rng.uniform(-1, 1, n)
    rs = orc.reduced_system(a, b, c, d, P, periodic=True)
    K = 2 * P
    Zb = rs["Zbar"]
    dist = np.abs(np.subtract.outer(np.arange(K), np.arange(K)))
    allowed = (dist <= 1) | (dist == K - 1)
    assert np.all(Zb[~allowed] == 0)
    assert Zb[0, K - 1] != 0 and Zb[K - 1, 0] != 0
    # y = E^T x of the exact solution solves Z y = E^T x~
    x = np.linalg.solve(dense(a, b, c, True), d)
    m = n // P
    ET_rows = []
    for i in range(1, P + 1):
        L, R = i - 1, i % P
        ET_rows += [L * m + m - 1, R * m]
    assert np.allclose(rs["Z"] @ x[ET_rows], rs["rhs"], atol=1e-14)


def test_reduced_unknowns_are_interface_values(orc):
    """From A x = d: x = x~ - Y E^T x, so the exact interface values solve Eq. (7)."""
    rng = np.random.default_rng(8)
    n, P = 40, 5
    a, b, c = W.random_tridiag(n, rng, margin=0.2)
    d = rng.uniform(-1, 1, n)
    rs = orc.reduced_system(a, b, c, d, P)
    x = np.linalg.solve(dense(a, b, c), d)
    m = n // P
    ET_rows = []
    for i in range(1, P):
        ET_rows += [(i - 1) * m + m - 1, i * m]
    assert np.allclose(rs["Z"] @ x[ET_rows], rs["rhs"], atol=1e-14)


# --------------------------------------------------------------------------
# Closed forms
# --------------------------------------------------------------------------
@pytest.mark.parametrize("r,m", [(0.1, 16), (1.0, 16), (10.0, 16), (4.194304, 256), (0.0829, 72)])
def test_toeplitz_spikes_closed_form(orc, r, m):
    """Block tridiag(-r, 1+2r, -r): with cosh(t) = (1+2r)/(2r),
    v_j = -sinh((m-j)t)/sinh((m+1)t), w_j = -sinh((j+1)t)/sinh((m+1)t)."""
    P = 3
    n = P * m
    a = np.full(n, -r)
    c = np.full(n, -r)
    b = np.full(n, 1 + 2 * r)
    a[0] = c[-1] = 0
    rs = orc.reduced_system(a, b, c, np.zeros(n), P)
    t = np.arccosh((1 + 2 * r) / (2 * r))
    j = np.arange(m)

    def ratio(p, q):  # sinh(p t)/sinh(q t) without overflow
        return np.exp((p - q) * t) * (1 - np.exp(-2 * p * t)) / (1 - np.exp(-2 * q * t))

    v_cf = -ratio(m - j, m + 1)
    w_cf = -ratio(j + 1, m + 1)
    v1 = rs["v"][m:2 * m]          # partition 1 has both spikes
    w1 = rs["w"][m:2 * m]
    assert np.max(np.abs(v1 - v_cf)) < 1e-14
    assert np.max(np.abs(w1 - w_cf)) < 1e-14
    assert np.all(rs["v"][:m] == 0) and np.all(rs["w"][2 * m:] == 0)


@pytest.mark.parametrize("method", ["thomas", "ppt4", "ppt8"])
def test_manufactured_dirichlet_sine(orc, method):
    """Symmetric Toeplitz: d_j = sin(pi q (j+1)/(n+1)) is an eigenvector."""
    n = 64
    a0, b0 = -0.7, 2.3
    a = np.full(n, a0)
    c = np.full(n, a0)
    b = np.full(n, b0)
    a[0] = c[-1] = 0
    for q in (1, 5, 33, 64):
        d = np.sin(np.pi * q * (np.arange(n) + 1) / (n + 1))
        x_cf = d / (b0 + 2 * a0 * np.cos(np.pi * q / (n + 1)))
        if method == "thomas":
            x = orc.thomas(a, b, c, d)
        else:
            x = orc.ppt(a, b, c, d, int(method[3:]))
        # cond(A) <= (b0 + 2|a0|)/(b0 - 2|a0|) ~ 4.1; bound cond * n * eps ~ 3e-14
        assert relerr(x, x_cf) < 5e-14


@pytest.mark.parametrize("P", [1, 2, 4, 6])
def test_manufactured_circulant_cosine(orc, P):
    """Periodic Toeplitz (circulant): d_j = cos(2 pi q j/n) is an eigenvector."""
    n = 48
    a0, b0 = -0.35, 1.9
    a = np.full(n, a0)
    c = np.full(n, a0)
    b = np.full(n, b0)
    for q in (0, 1, 7, 24):
        d = np.cos(2 * np.pi * q * np.arange(n) / n)
        x_cf = d / (b0 + 2 * a0 * np.cos(2 * np.pi * q / n))
        assert relerr(orc.ppt(a, b, c, d, P, periodic=True), x_cf) < 1e-14
        assert relerr(orc.cyclic(a, b, c, d), x_cf) < 1e-14


def test_manufactured_neumann_poisson(orc):
    """Uniform cell-centred Neumann operator: cos(pi q (j+1/2)/n) has eigenvalue
    -(4/h^2) sin^2(pi q/(2n)) - lam (the lam = 0 mode is gauge pinned)."""
    Ny, Nx, Nk = 64, 3, 4
    h = 1.0 / Ny
    ay = np.full(Ny, 1 / h ** 2)
    cy = np.full(Ny, 1 / h ** 2)
    ay[0] = 0
    cy[-1] = 0
    lam = np.array([0.0, 3.0, 40.0, 1e4])
    j = np.arange(Ny)
    phihat = np.zeros((Nk, Ny, Nx), complex)
    expect = np.zeros_like(phihat)
    for k in range(1, Nk):
        for i in range(Nx):
            q = 1 + 5 * i + k
            e = np.cos(np.pi * q * (j + 0.5) / Ny) * (1.0 + 0.5j * (i + 1))
            ev = -(4 / h ** 2) * np.sin(np.pi * q / (2 * Ny)) ** 2 - lam[k]
            phihat[k, :, i] = e * ev
            expect[k, :, i] = e
    orc.poisson(phihat, ay, cy, lam, P=4)
    assert np.max(np.abs(phihat[1:] - expect[1:])) < 1e-12
    assert np.all(phihat[0] == 0)   # zero RHS in the pinned mode stays zero


# --------------------------------------------------------------------------
# PDD: structure, exact cases and the truncation bound
# --------------------------------------------------------------------------
def test_pdd_two_partitions_is_exact(orc):
    """With p = 2 (non-periodic) Z has no dropped entries, so PDD is exact."""
    rng = np.random.default_rng(21)
    n = 50
    a, b, c = W.random_tridiag(n, rng, margin=0.05)
    d = rng.uniform(-1, 1, n)
    assert relerr(orc.pdd(a, b, c, d, 2), np.linalg.solve(dense(a, b, c), d)) < 1e-13


def test_pdd_exact_when_spikes_are_cut(orc):
    """A row with a = c = 0 inside every partition stops the spikes, so the
    dropped Z entries are exactly zero and PDD must equal A^{-1} d."""
    rng = np.random.default_rng(22)
    P, m = 5, 10
    n = P * m
    a, b, c = W.random_tridiag(n, rng, margin=0.1)
    for r in range(P):
        k = r * m + m // 2
        a[k] = c[k] = 0.0
    d = rng.uniform(-1, 1, n)
    ref = np.linalg.solve(dense(a, b, c), d)
    assert relerr(orc.pdd(a, b, c, d, P), ref) < 1e-14
    a2, b2, c2 = a.copy(), b.copy(), c.copy()
    a2[0], c2[-1] = rng.uniform(-0.5, 0.5, 2)
    ref2 = np.linalg.solve(dense(a2, b2, c2, True), d)
    assert relerr(orc.pdd(a2, b2, c2, d, P, periodic=True), ref2) < 1e-14


def test_pdd_matches_truncated_Z_solve(orc):
    """PDD = Eq. (8) with the 2x2-block part of Z (Sec. 3.2): dropping v_m^(L)
    and w_1^(R) from the assembled Z and solving densely gives the same x."""
    rng = np.random.default_rng(23)
    n, P = 60, 6
    a, b, c = W.random_tridiag(n, rng, margin=0.05)
    d = rng.uniform(-1, 1, n)
    rs = orc.reduced_system(a, b, c, d, P)
    m = n // P
    Zt = np.zeros_like(rs["Z"])
    for i in range(1, P):
        u1, u2 = 2 * i - 2, 2 * i - 1
        Zt[u1, u1] = Zt[u2, u2] = 1.0
        Zt[u1, u2] = rs["Z"][u1, u2]
        Zt[u2, u1] = rs["Z"][u2, u1]
    y = np.linalg.solve(Zt, rs["rhs"])
    x = rs["xt"].copy()
    for r in range(P):
        sl = slice(r * m, r * m + m)
        if r >= 1:
            x[sl] -= rs["v"][sl] * y[2 * r - 2]
        if r <= P - 2:
            x[sl] -= rs["w"][sl] * y[2 * r + 1]
    assert np.max(np.abs(orc.pdd(a, b, c, d, P) - x)) < 1e-14


@pytest.mark.parametrize("r", [0.5, 2.0, 5.0, 10.0])
def test_pdd_truncation_bound(orc, r):
    """||x_PDD - x||_inf <= 4 delta ||x||_inf, delta = largest dropped entry,
    here the closed form sinh(t)/sinh((m+1)t) of the Toeplitz spikes."""
    n, P = 64, 4
    m = n // P
    a = np.full(n, -r)
    c = np.full(n, -r)
    b = np.full(n, 1 + 2 * r)
    a[0] = c[-1] = 0
    t = np.arccosh((1 + 2 * r) / (2 * r))
    delta = np.exp(-m * t) * (1 - np.exp(-2 * t)) / (1 - np.exp(-2 * (m + 1) * t))
    rng = np.random.default_rng(int(r * 10))
    worst = 0.0
    for _ in range(20):
        d = rng.uniform(-1, 1, n)
        x = np.linalg.solve(dense(a, b, c), d)
        e = np.max(np.abs(orc.pdd(a, b, c, d, P) - x)) / np.max(np.abs(x))
        worst = max(worst, e)
        assert e <= 4 * delta + 1e-15
    assert worst > 0.05 * delta     # the bound is not vacuous: PDD really drops something


def test_pdd_momentum_claim(orc):
    """Sec. 3.2: for the ADI matrices (|b| = |a| + |c| + 1) PDD matches the exact
    solution to machine accuracy, at the partition counts the sweeps use."""
    rng = np.random.default_rng(0)
    cases = [(W.momentum_uniform(2048), 8, False), (W.momentum_stretched(256), 4, False),
             (W.momentum_periodic(288), 4, True)]
    for (a, b, c), P, per in cases:
        n = len(b)
        assert np.all(np.abs(b) >= np.abs(a) + np.abs(c) + 1 - 1e-12)
        d = rng.standard_normal(n)
        assert relerr(orc.pdd(a, b, c, d, P, per), orc.exact(a, b, c, d, per)) < 1e-14


def test_pdd_poisson_claim(orc):
    """Sec. 3.2: at low modified wavenumbers the Poisson matrices are barely
    dominant (eps ~ 1e-6 relative) and PDD is inaccurate while PPT is exact."""
    Ny = 256
    ay, cy = W.poisson_metric(Ny)
    lam = W.modified_wavenumbers(288)
    rng = np.random.default_rng(0)
    d = rng.standard_normal(Ny)
    for k, pdd_min in ((1, 1e-3), (2, 1e-3), (10, 1e-6)):
        b = -(ay + cy) - lam[k]
        eps = lam[k] / np.max(ay + cy)
        assert 1e-8 < eps < 1e-3
        ref = np.linalg.solve(dense(ay, b, cy), d)
        assert relerr(orc.pdd(ay, b, cy, d, 4), ref) > pdd_min
        assert relerr(orc.ppt(ay, b, cy, d, 4), ref) < 1e-12
    b = -(ay + cy) - lam[144]
    ref = np.linalg.solve(dense(ay, b, cy), d)
    assert relerr(orc.pdd(ay, b, cy, d, 4), ref) < 1e-14


# --------------------------------------------------------------------------
# Batched drivers
# --------------------------------------------------------------------------
def test_solve_batch_strided_layouts(orc):
    rng = np.random.default_rng(31)
    n, nb0, nb1, P = 24, 5, 3, 4
    coef = [W.random_tridiag(n, rng) for _ in range(nb0 * nb1)]
    A = np.array([t[0] for t in coef]).reshape(nb1, nb0, n)
    B = np.array([t[1] for t in coef]).reshape(nb1, nb0, n)
    C = np.array([t[2] for t in coef]).reshape(nb1, nb0, n)
    D = rng.uniform(-1, 1, (nb1, n, nb0))           # layout [b1][j][b0]
    for method in (orc.EXACT, orc.PDD, orc.PPT):
        flat = D.copy().ravel()
        orc.solve_batch(method, flat, n, nb0, nb1, s_j=nb0, s_b0=1, s_b1=n * nb0,
                        a=A.ravel(), b=B.ravel(), c=C.ravel(), cs_j=1, cs_b0=n, cs_b1=n * nb0, P=P)
        got = flat.reshape(nb1, n, nb0)
        for b1 in range(nb1):
            for b0 in range(nb0):
                args = (A[b1, b0], B[b1, b0], C[b1, b0], D[b1, :, b0])
                ref = {orc.EXACT: lambda: orc.thomas(*args), orc.PDD: lambda: orc.pdd(*args, P),
                       orc.PPT: lambda: orc.ppt(*args, P)}[method]()
                assert np.array_equal(got[b1, :, b0], ref)


def test_adi_sweep_directions(orc):
    rng = np.random.default_rng(32)
    Nz, Ny, Nx = 12, 8, 16
    u = rng.standard_normal((Nz, Ny, Nx))
    for direction, n, per, P in ((0, Nx, False, 4), (1, Ny, False, 2), (2, Nz, True, 3)):
        a, b, c = W.random_tridiag(n, rng, periodic=per)
        got = u.copy()
        orc.adi_sweep(orc.PPT, direction, got, a, b, c, P, per)
        ref = np.moveaxis(u, 2 - direction, -1).copy()
        shp = ref.shape
        ref = ref.reshape(-1, n)
        A = dense(a, b, c, per)
        ref = np.linalg.solve(A, ref.T).T.reshape(shp)
        assert np.max(np.abs(got - np.moveaxis(ref, -1, 2 - direction))) < 1e-13


def test_error_paths(orc):
    a, b, c = W.momentum_uniform(10)
    with pytest.raises(orc.OracleError) as e:
        orc.pdd(a, b, c, np.ones(10), 3)
    assert e.value.code == 2
    b0 = b.copy()
    b0[0] = 0.0
    with pytest.raises(orc.OracleError) as e:
        orc.thomas(a, b0, c, np.ones(10))
    assert e.value.code == 3


@pytest.mark.parametrize("periodic", [False, True])
def test_dense_solve_non_dominant_exact_rational(orc, periodic):
    """The reference for non-dominant systems equals exact rational elimination on a
    system with zero diagonal entries (where elimination without pivoting divides by 0)."""
    rng = np.random.default_rng(8)
    n = 12
    a, b, c = W.random_tridiag_nondominant(n, rng, periodic=periodic)
    assert b[0] == 0.0 and b[7] == 0.0
    d = rng.uniform(-1, 1, n)
    xr = _exact_fraction_solve(dense(a, b, c, periodic), d)
    assert relerr(orc.dense_solve(a, b, c, d, periodic), xr) < 1e-13
