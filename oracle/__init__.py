"""FP64 CPU oracle for the partitioned tridiagonal solves (PDD / PPT).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg.  The product library never imports it, and
it imports nothing from the product package.

The arithmetic lives in ``oracle.c`` (plain C, built with gcc
``-O2 -ffp-contract=off -fopenmp``); this module builds it on demand and
wraps it for numpy arrays:

* ``thomas`` / ``cyclic`` / ``exact``  -- plain solution x = A^{-1} d
* ``exact_ld`` -- the same in long double (extended) arithmetic, the
  reference for results that converge to the exact solution
* ``pdd``  -- Sec. 3.2, PDD paragraph and Algorithm 1 (depends on P)
* ``ppt``  -- Sec. 3.2, Eqs. (9)-(11) (exact; periodic wrap as interface P)
* ``dpivot`` / ``ppt_dp`` / ``ppt_dp_batch`` -- the block solver with
  diagonal pivoting that the PPT paragraph of Sec. 3.2 names, alone and as
  PPT's local solver; both also return every row's pivot kind
* ``reduced_system`` -- Z (Eq. (7)), Zbar (Eq. (10)), E^T x~ and spikes
* ``solve_batch`` / ``adi_sweep`` / ``poisson`` / ``poisson_shifted_batch`` --
  batched strided drivers

Function for function, every pin that checks these lives in
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

EXACT, PDD, PPT, EXACT_LD = 0, 1, 2, 3
_STATUS = {0: "ok", 1: "invalid argument", 2: "bad shape", 3: "zero pivot", 7: "out of memory"}


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what}: {_STATUS.get(code, code)}")
        self.code = code


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-std=c11",
                               "-Wall", "-Wextra", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        for name in ("orc_thomas", "orc_cyclic", "orc_pdd", "orc_ppt", "orc_exact"):
            getattr(L, name).restype = ctypes.c_int
        L.orc_thomas.argtypes = [_I64, _D, _D, _D, _D, _D, _D]
        L.orc_cyclic.argtypes = [_I64, _D, _D, _D, _D, _D, _D]
        L.orc_pdd.argtypes = [_I64, ctypes.c_int, ctypes.c_int, _D, _D, _D, _D, _D, _D]
        L.orc_ppt.argtypes = [_I64, ctypes.c_int, ctypes.c_int, _D, _D, _D, _D, _D, _D]
        L.orc_exact.argtypes = [_I64, ctypes.c_int, _D, _D, _D, _D, _D, _D]
        L.orc_exact_ld.restype = ctypes.c_int
        L.orc_exact_ld.argtypes = [_I64, ctypes.c_int, _D, _D, _D, _D, _D]
        L.orc_line_work.restype = _I64
        L.orc_line_work.argtypes = [_I64, ctypes.c_int]
        L.orc_reduced_system.restype = ctypes.c_int
        L.orc_reduced_system.argtypes = [_I64, ctypes.c_int, ctypes.c_int, _D, _D, _D, _D,
                                         _D, _D, _D, _D, _D, _D]
        L.orc_solve_batch.restype = ctypes.c_int
        L.orc_solve_batch.argtypes = [ctypes.c_int, _I64, ctypes.c_int, ctypes.c_int,
                                      _D, _D, _D, _I64, _I64, _I64,
                                      _D, _I64, _I64, _I64, _I64, _I64, ctypes.c_int]
        L.orc_adi_sweep.restype = ctypes.c_int
        L.orc_adi_sweep.argtypes = [ctypes.c_int, ctypes.c_int, _D, _I64, _I64, _I64,
                                    _D, _D, _D, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_poisson.restype = ctypes.c_int
        L.orc_poisson.argtypes = [ctypes.c_int, _D, _I64, _I64, _I64, _D, _D, _D,
                                  ctypes.c_int, ctypes.c_int]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_poisson_shifted.restype = ctypes.c_int
        L.orc_poisson_shifted.argtypes = [ctypes.c_int, _D, _I64, _I64, _I64, _D, _D, _D, _D,
                                          ctypes.c_int, ctypes.c_int]
        _U8 = ctypes.POINTER(ctypes.c_uint8)
        L.orc_dpivot.restype = ctypes.c_int
        L.orc_dpivot.argtypes = [_I64, _D, _D, _D, ctypes.c_int, _D, _U8, _D]
        L.orc_ppt_dp.restype = ctypes.c_int
        L.orc_ppt_dp.argtypes = [_I64, ctypes.c_int, ctypes.c_int, _D, _D, _D, _D, _D, _D, _U8]
        L.orc_ppt_dp_batch.restype = ctypes.c_int
        L.orc_ppt_dp_batch.argtypes = [_I64, ctypes.c_int, ctypes.c_int, _D, _D, _D, _I64, _I64, _I64,
                                       _D, _I64, _I64, _I64, _I64, _I64, _U8, ctypes.c_int]
        _lib = L
    return _lib


def _p(arr: np.ndarray):
    return arr.ctypes.data_as(_D)


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def _check(code: int, what: str):
    if code != 0:
        raise OracleError(code, what)


def thomas(a, b, c, d) -> np.ndarray:
    a, b, c, d = map(_f64, (a, b, c, d))
    n = d.size
    x = np.empty(n)
    cp = np.empty(n)
    _check(lib().orc_thomas(n, _p(a), _p(b), _p(c), _p(d), _p(x), _p(cp)), "thomas")
    return x


def cyclic(a, b, c, d) -> np.ndarray:
    a, b, c, d = map(_f64, (a, b, c, d))
    n = d.size
    x = np.empty(n)
    work = np.empty(5 * n)
    _check(lib().orc_cyclic(n, _p(a), _p(b), _p(c), _p(d), _p(x), _p(work)), "cyclic")
    return x


def exact(a, b, c, d, periodic: bool = False) -> np.ndarray:
    return cyclic(a, b, c, d) if periodic else thomas(a, b, c, d)


def dense_solve(a, b, c, d, periodic: bool = False) -> np.ndarray:
    """x = A^{-1} d for any nonsingular tridiagonal (cyclic if periodic) row set: the
    plain definition, by Gaussian elimination with partial pivoting on the assembled
    dense matrix (LAPACK through numpy).  The reference for general, non-dominant
    systems, where eliminations without pivoting break down."""
    a, b, c, d = map(_f64, (a, b, c, d))
    n = b.size
    A = np.diag(b)
    if n > 1:
        A += np.diag(a[1:], -1) + np.diag(c[:-1], 1)
        if periodic:
            A[0, n - 1] += a[0]
            A[n - 1, 0] += c[n - 1]
    return np.linalg.solve(A, d)


def exact_ld(a, b, c, d, periodic: bool = False) -> np.ndarray:
    """x = A^{-1} d by Thomas (or the cyclic Sherman-Morrison solve) in long double."""
    a, b, c, d = map(_f64, (a, b, c, d))
    x = np.empty(d.size)
    _check(lib().orc_exact_ld(d.size, int(bool(periodic)), _p(a), _p(b), _p(c), _p(d), _p(x)), "exact_ld")
    return x


def _line(fn, name, a, b, c, d, P, periodic):
    a, b, c, d = map(_f64, (a, b, c, d))
    n = d.size
    x = np.empty(n)
    work = np.empty(int(lib().orc_line_work(n, P)) + 5 * n)
    _check(fn(n, int(P), int(bool(periodic)), _p(a), _p(b), _p(c), _p(d), _p(x), _p(work)), name)
    return x


def pdd(a, b, c, d, P: int, periodic: bool = False) -> np.ndarray:
    return _line(lib().orc_pdd, "pdd", a, b, c, d, P, periodic)


def ppt(a, b, c, d, P: int, periodic: bool = False) -> np.ndarray:
    return _line(lib().orc_ppt, "ppt", a, b, c, d, P, periodic)


def _u8(arr: np.ndarray):
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


# pivot kinds returned by dpivot / ppt_dp
PIV_1X1, PIV_2X2_FIRST, PIV_2X2_SECOND = 1, 2, 0


def dpivot(a, b, c, rhs):
    """Solve one tridiagonal block (a[0], c[m-1] unused) by diagonal pivoting.
    rhs: (m,) or (k, m) right-hand sides.  Returns (x, piv) with piv[t] = 1 (1x1
    pivot), 2 (first row of a 2x2 pivot) or 0 (its second row)."""
    a, b, c = map(_f64, (a, b, c))
    R = np.array(rhs, dtype=np.float64, copy=True, order="C")
    one = R.ndim == 1
    R = np.atleast_2d(R)
    m = b.size
    assert R.shape[1] == m
    piv = np.zeros(m, dtype=np.uint8)
    work = np.empty(2 * m + 1)
    _check(lib().orc_dpivot(m, _p(a), _p(b), _p(c), R.shape[0], _p(R), _u8(piv), _p(work)), "dpivot")
    return (R[0] if one else R), piv


def ppt_dp(a, b, c, d, P: int, periodic: bool = False):
    """PPT (Eqs. (9)-(11)) whose partition blocks are solved by diagonal pivoting.
    Returns (x, piv), piv the pivot kind of every row (see dpivot)."""
    a, b, c, d = map(_f64, (a, b, c, d))
    n = d.size
    x = np.empty(n)
    piv = np.zeros(n, dtype=np.uint8)
    work = np.empty(int(lib().orc_line_work(n, P)) + 2 * n + 2 * (n // max(P, 1)) + 8)
    _check(lib().orc_ppt_dp(n, int(P), int(bool(periodic)), _p(a), _p(b), _p(c), _p(d), _p(x), _p(work),
                            _u8(piv)), "ppt_dp")
    return x, piv


def ppt_dp_batch(d: np.ndarray, n: int, nb0: int, nb1: int, s_j: int, s_b0: int, s_b1: int, a, b, c,
                 cs_j: int, cs_b0: int, cs_b1: int, P: int, periodic: bool = False,
                 nthreads: int = 0) -> np.ndarray:
    """In-place ppt_dp over strided lines of the flat FP64 array d (per-line
    coefficients at j*cs_j + b0*cs_b0 + b1*cs_b1).  Returns the pivot kinds as
    a (nb1*nb0, n) uint8 array, line (b0, b1) in row b1*nb0 + b0."""
    assert d.dtype == np.float64 and d.flags.c_contiguous
    a, b, c = map(_f64, (a, b, c))
    piv = np.zeros((nb0 * nb1, n), dtype=np.uint8)
    _check(lib().orc_ppt_dp_batch(n, int(P), int(bool(periodic)), _p(a), _p(b), _p(c), cs_j, cs_b0, cs_b1,
                                  _p(d), nb0, nb1, s_j, s_b0, s_b1, _u8(piv), int(nthreads)), "ppt_dp_batch")
    return piv


def reduced_system(a, b, c, d, P: int, periodic: bool = False) -> dict:
    """Z, Zbar (K x K), E^T x~ (K) and x~, v, w (n) of one line."""
    a, b, c, d = map(_f64, (a, b, c, d))
    n = d.size
    K = 2 * (P if periodic else P - 1)
    Z = np.empty((K, K))
    Zbar = np.empty((K, K))
    rhs = np.empty(K)
    xt, v, w = np.empty(n), np.empty(n), np.empty(n)
    _check(lib().orc_reduced_system(n, int(P), int(bool(periodic)), _p(a), _p(b), _p(c), _p(d),
                                    _p(Z), _p(Zbar), _p(rhs), _p(xt), _p(v), _p(w)),
           "reduced_system")
    return {"Z": Z, "Zbar": Zbar, "rhs": rhs, "xt": xt, "v": v, "w": w}


def solve_batch(method: int, d: np.ndarray, n: int, nb0: int, nb1: int,
                s_j: int, s_b0: int, s_b1: int, a, b, c,
                cs_j: int = 1, cs_b0: int = 0, cs_b1: int = 0,
                P: int = 1, periodic: bool = False, nthreads: int = 0) -> None:
    """In-place batched solve over strided lines of the flat FP64 array d."""
    assert d.dtype == np.float64 and d.flags.c_contiguous
    a, b, c = map(_f64, (a, b, c))
    _check(lib().orc_solve_batch(int(method), n, int(P), int(bool(periodic)),
                                 _p(a), _p(b), _p(c), cs_j, cs_b0, cs_b1,
                                 _p(d), nb0, nb1, s_j, s_b0, s_b1, int(nthreads)), "solve_batch")


def adi_sweep(method: int, direction: int, u: np.ndarray, a, b, c, P: int,
              periodic: bool = False, nthreads: int = 0) -> None:
    """In-place sweep of u[Nz][Ny][Nx] along direction 0 (x), 1 (y) or 2 (z)."""
    assert u.dtype == np.float64 and u.flags.c_contiguous and u.ndim == 3
    Nz, Ny, Nx = u.shape
    a, b, c = map(_f64, (a, b, c))
    _check(lib().orc_adi_sweep(int(method), int(direction), _p(u), Nx, Ny, Nz,
                               _p(a), _p(b), _p(c), int(P), int(bool(periodic)), int(nthreads)),
           "adi_sweep")


def poisson(phihat: np.ndarray, ay, cy, lam, P: int, method: int = PPT,
            nthreads: int = 0) -> None:
    """In-place wall-normal solves of phihat[Nk][Ny][Nx] complex128."""
    assert phihat.dtype == np.complex128 and phihat.flags.c_contiguous and phihat.ndim == 3
    Nk, Ny, Nx = phihat.shape
    ay, cy, lam = map(_f64, (ay, cy, lam))
    assert lam.size == Nk
    flat = phihat.view(np.float64)
    _check(lib().orc_poisson(int(method), _p(flat), Nx, Ny, Nk, _p(ay), _p(cy), _p(lam),
                             int(P), int(nthreads)), "poisson")


def poisson_shifted_batch(phihat: np.ndarray, ay, cy, lamz, lamx, P: int, method: int = PPT,
                          nthreads: int = 0) -> None:
    """The solves of poisson_shifted below, every line in C (OpenMP over lines);
    method PPT, PDD, EXACT or EXACT_LD."""
    assert phihat.dtype == np.complex128 and phihat.flags.c_contiguous and phihat.ndim == 3
    Nk, Ny, Nx = phihat.shape
    ay, cy, lamz, lamx = map(_f64, (ay, cy, lamz, lamx))
    assert lamz.size == Nk and lamx.size == Nx
    _check(lib().orc_poisson_shifted(int(method), _p(phihat.view(np.float64)), Nx, Ny, Nk, _p(ay), _p(cy),
                                     _p(lamz), _p(lamx), int(P), int(nthreads)), "poisson_shifted")


def poisson_shifted(phihat: np.ndarray, ay, cy, lamz, lamx, P: int, method: int = PPT) -> None:
    """In-place wall-normal solves of phihat[Nk][Ny][Nx] complex128 with one matrix per
    line (k, i): a = ay, c = cy, b = -(ay + cy) - (lamz_k + lamx_i) -- the Poisson systems
    once both homogeneous directions are transformed (Sec. 2.2; PPT paragraph of
    Sec. 3.2).  A line whose shift is 0 is gauge pinned (row 0 becomes x_0 = 0).  Real
    and imaginary parts are solved as two real lines with the same matrix."""
    assert phihat.dtype == np.complex128 and phihat.ndim == 3
    Nk, Ny, Nx = phihat.shape
    ay, cy, lamz, lamx = map(_f64, (ay, cy, lamz, lamx))
    if method == EXACT:
        fn = lambda a, b, c, d, P: exact(a, b, c, d)
    else:
        fn = ppt if method == PPT else pdd
    for k in range(Nk):
        for i in range(Nx):
            sigma = lamz[k] + lamx[i]
            a, c = ay.copy(), cy.copy()
            b = -(ay + cy) - sigma
            rhs = phihat[k, :, i].copy()
            if sigma == 0.0:
                b[0], c[0], rhs[0] = 1.0, 0.0, 0.0
            phihat[k, :, i] = fn(a, b, c, rhs.real, P) + 1j * fn(a, b, c, rhs.imag, P)


def max_threads() -> int:
    return int(lib().orc_max_threads())
