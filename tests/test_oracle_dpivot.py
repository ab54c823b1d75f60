"""Pins of the oracle's diagonal-pivoting block solver and of PPT built on it
(the local solver the PPT paragraph of Sec. 3.2 names; pivot test of reading
20: 1x1 pivot at row k unless |delta| sigma < kappa |a_{k+1} c_k|).

What pins it, none of it the oracle itself:
* exact rational elimination of systems with zero diagonal entries;
* lines built so that the elimination is exact in FP64 and the pivot kinds are
  known by construction (bitwise solution, exact pivot pattern);
* hand-worked pivot decisions on both sides of kappa = (sqrt 5 - 1)/2, one case
  for each entry that makes up sigma;
* on diagonally dominant rows every pivot is 1x1 (provable: |delta_k| > |c_k|
  and sigma >= |b_{k+1}| > |a_{k+1}|), so the result is bit for bit the
  Thomas-based PPT;
* backward stability and agreement with the dense solve on random non-dominant
  lines, at every partition count, periodic or not.
"""
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from test_oracle_pins import _exact_fraction_solve, dense, relerr

EPS = np.finfo(float).eps


def _fraction_solution(a, b, c, d):
    """Exact rational solution as Fractions (no rounding at the end)."""
    n = len(d)
    A = dense(a, b, c)
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
        x[k] = (M[k][n] - sum(M[k][t] * x[t] for t in range(k + 1, n))) / M[k][k]
    return x


@pytest.mark.parametrize("periodic", [False, True])
def test_ppt_dp_exact_rational_zero_diagonals(orc, periodic):
    """Rows with zero diagonal entries (every 7th row) and |b| < |a| + |c| elsewhere:
    PPT with diagonal pivoting equals exact rational elimination at every P."""
    rng = np.random.default_rng(21)
    for n in (12, 16):
        a, b, c = W.random_tridiag_nondominant(n, rng, periodic=periodic)
        d = rng.uniform(-1, 1, n)
        xr = _exact_fraction_solve(dense(a, b, c, periodic), d)
        cond = np.linalg.cond(dense(a, b, c, periodic), np.inf)
        for P in (1, 2, 3, 4):
            if n % P or (periodic and n // P < 2):
                continue
            try:
                x, piv = orc.ppt_dp(a, b, c, d, P, periodic)
            except orc.OracleError as e:        # a singular partition block: not this test's case
                assert e.code == 3
                continue
            assert relerr(x, xr) < 64 * EPS * cond, (n, P, relerr(x, xr), cond)
            assert set(np.unique(piv)) <= {0, 1, 2}


@pytest.mark.parametrize("n,P", [(16, 1), (32, 2), (64, 4), (96, 3), (128, 8)])
def test_ppt_dp_forced_pivots_exact(orc, n, P):
    """Lines whose elimination is exact (powers of two, integer right-hand sides) and
    whose 2x2 pivots sit at rows fixed by construction: the pivot kinds match the
    construction row by row and x equals the exact rational solution bit for bit."""
    rng = np.random.default_rng(100 + n + P)
    for _ in range(4):
        a, b, c, d, starts = W.pivot_probe(n, P, rng)
        xf = _fraction_solution(a, b, c, d)
        assert all(Fraction(float(v)) == v for v in xf), "probe solution not representable"
        want = np.ones(n, dtype=np.uint8)
        for j in starts:
            want[j], want[j + 1] = 2, 0
        x, piv = orc.ppt_dp(a, b, c, d, P)
        assert np.array_equal(piv, want)
        assert np.array_equal(x, np.array([float(v) for v in xf]))
        # the plain Thomas elimination meets the zero diagonal and fails
        if starts:
            with pytest.raises(orc.OracleError):
                orc.ppt(a, b, c, d, P)


def _block(delta, c0, a1, b1, c1=0.0, a2=0.0, b2=1.0):
    """Rows 0..2 of a block: [delta c0 .], [a1 b1 c1], [. a2 b2]."""
    return (np.array([0.0, a1, a2]), np.array([delta, b1, b2]), np.array([c0, c1, 0.0]))


KAPPA = (np.sqrt(5.0) - 1.0) / 2.0      # 0.6180...


@pytest.mark.parametrize("case,first", [
    # sigma = 1 from |c_0| = |a_1| = |b_1| = 1: 2x2 iff |delta| < 0.618
    (_block(0.61, 1.0, 1.0, 1.0), 2),
    (_block(-0.61, 1.0, 1.0, 1.0), 2),
    (_block(0.625, 1.0, 1.0, 1.0), 1),
    (_block(-0.625, 1.0, 1.0, 1.0), 1),
    # |delta| = 0.5 (2x2 at sigma = 1); one entry of sigma raised to 2 or 3 makes it 1x1
    (_block(0.5, 1.0, 1.0, 1.0), 2),
    (_block(0.5, 1.0, 1.0, 3.0), 1),          # |b_1|
    (_block(0.5, 1.0, 1.0, 1.0, c1=2.0), 1),  # |c_1|
    (_block(0.5, 1.0, 1.0, 1.0, a2=2.0), 1),  # |a_2|
    (_block(0.5, 2.0, 0.5, 1.0), 1),          # |c_0| (the product a_1 c_0 stays 1)
    (_block(0.5, 0.5, 2.0, 1.0), 1),          # |a_1|
    # no coupling in the pivot's column: always 1x1
    (_block(1e-3, 0.0, 1.0, 1.0), 1),
])
def test_dpivot_decision_hand_worked(orc, case, first):
    a, b, c = case
    rhs = np.array([1.0, 2.0, 3.0])
    x, piv = orc.dpivot(a, b, c, rhs)
    assert piv[0] == first
    if first == 2:
        assert piv[1] == 0 and piv[2] == 1
    assert relerr(x, np.linalg.solve(dense(a, b, c), rhs)) < 1e-14


def test_ppt_dp_dominant_rows_equal_thomas_ppt(orc):
    """Diagonally dominant rows take 1x1 pivots only, and then every step is the
    Thomas step: ppt_dp equals ppt bit for bit (and P = 1 equals thomas)."""
    rng = np.random.default_rng(23)
    for n, P, periodic in [(64, 1, False), (64, 4, False), (96, 8, False), (48, 4, True), (60, 3, True)]:
        for margin in (1.0, 1e-3):
            a, b, c = W.random_tridiag(n, rng, margin=margin, periodic=periodic)
            d = rng.uniform(-1, 1, n)
            x, piv = orc.ppt_dp(a, b, c, d, P, periodic)
            assert np.all(piv == 1)
            ref = orc.ppt(a, b, c, d, P, periodic) if (P > 1 or periodic) else orc.thomas(a, b, c, d)
            assert np.array_equal(x, ref), (n, P, periodic, margin)
    # the cell-centred Neumann Poisson rows (weakly dominant, the gauge-pinned k = 0 mode)
    ay, cy = W.poisson_metric(64)
    b = -(ay + cy)
    b[0], cy0 = 1.0, cy.copy()
    cy0[0] = 0.0
    d = rng.standard_normal(64)
    d[0] = 0.0
    x, piv = orc.ppt_dp(ay, b, cy0, d, 4)
    assert np.all(piv == 1)
    assert np.array_equal(x, orc.ppt(ay, b, cy0, d, 4))


@pytest.mark.parametrize("periodic", [False, True])
def test_ppt_dp_non_dominant_backward_stable(orc, periodic):
    """Random non-dominant lines (zero diagonals every 7th row): at every P the
    residual is at round-off of |A||x| (backward stable) and x agrees with the dense
    partial-pivoting solve to within the conditioning."""
    rng = np.random.default_rng(24)
    n = 64
    tried = solved = 0
    for _ in range(40):
        a, b, c = W.random_tridiag_nondominant(n, rng, periodic=periodic)
        d = rng.uniform(-1, 1, n)
        A = dense(a, b, c, periodic)
        xr = np.linalg.solve(A, d)
        cond = np.linalg.cond(A, np.inf)
        for P in ((1, 2, 4, 8) if not periodic else (1, 2, 4)):
            tried += 1
            try:
                x, piv = orc.ppt_dp(a, b, c, d, P, periodic)
            except orc.OracleError as e:
                assert e.code == 3       # a singular partition block
                continue
            solved += 1
            assert np.any(piv == 2)
            res = np.max(np.abs(d - A @ x)) / np.max(np.abs(A) @ np.abs(x))
            assert res < 2e3 * EPS, (P, res)
            assert relerr(x, xr) < 1e3 * EPS * cond, (P, relerr(x, xr), cond)
    assert solved >= 0.9 * tried


def test_dpivot_singular_block_reports_zero_pivot(orc):
    """A singular block (two equal rows) is reported, not divided by zero."""
    a = np.array([0.0, 1.0, 1.0])
    b = np.array([1.0, 1.0, 1.0])
    c = np.array([1.0, 1.0, 0.0])
    with pytest.raises(orc.OracleError) as e:
        orc.dpivot(a, np.array([0.0, 0.0, 1.0]), np.array([0.0, 0.0, 0.0]), np.ones(3))
    assert e.value.code == 3
    x, piv = orc.dpivot(a, b, c, np.ones(3))
    assert np.all(np.isfinite(x))
