"""GPU parity of libtri's FP64 path against the FP64 oracle.

Every call goes through the C ABI (include/tri.h) via the ctypes binding.
Bar: per-line relative error max_j|x - x_oracle| / max_j|x_oracle| <= 1e-12
(PDD against the oracle's PDD at the same P; PPT against the oracle's PPT),
bitwise equality for the exactly representable indexing probes.
Sizes span several workgroups and end in ragged tails; full BASELINE shapes
are covered by sampled lines in test_gpu_fullsize.py.
"""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from gpu_helpers import TOL, dev, host, line_relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import paper_1812_01178_amd as T
    T.lib()
    return T


@pytest.fixture(scope="module")
def ctx(T):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    h = T.tri_create(0, torch.cuda.current_stream().cuda_stream)
    yield h
    T.tri_destroy(h)


METHODS = [("PDD", 0), ("PPT", 1)]


def _oracle_method(orc, name):
    return orc.PDD if name == "PDD" else orc.PPT


# ---------------------------------------------------------------------------
# cfg 1 shape: independent systems, one r per line (general kernel)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mname,method", METHODS)
@pytest.mark.parametrize("nlines", [4096, 1000])
def test_independent_lines_strided(T, ctx, orc, mname, method, nlines):
    n, P = 64, 4
    r, dl = W.cfg_independent(nlines, n, seed=0)
    a, b, c = -r, 1 + 2 * r, -r
    d = np.ascontiguousarray(dl.T)                       # [j][line], line fastest
    ref = d.copy().ravel()
    orc.solve_batch(_oracle_method(orc, mname), ref, n, nlines, 1, s_j=nlines, s_b0=1, s_b1=0,
                    a=a, b=b, c=c, cs_j=0, cs_b0=1, cs_b1=0, P=P)
    dd = dev(d)
    fn = T.tri_pdd_solve if method == 0 else T.tri_ppt_solve
    fn(ctx, dev(a), dev(b), dev(c), dd, (n, nlines, 1, nlines, 1, 0), coef_strides=(0, 1, 0), P=P)
    T.tri_sync_status(ctx)
    got = host(dd)
    assert line_relerr(got, ref.reshape(n, nlines), axis=0) <= TOL


@pytest.mark.parametrize("mname,method", METHODS)
def test_independent_lines_contiguous_general(T, ctx, orc, mname, method):
    n, P, nlines = 64, 4, 300
    r, d = W.cfg_independent(nlines, n, seed=1)
    a, b, c = -r, 1 + 2 * r, -r
    ref = d.copy().ravel()
    orc.solve_batch(_oracle_method(orc, mname), ref, n, nlines, 1, s_j=1, s_b0=n, s_b1=0,
                    a=a, b=b, c=c, cs_j=0, cs_b0=1, cs_b1=0, P=P)
    dd = dev(d)
    fn = T.tri_pdd_solve if method == 0 else T.tri_ppt_solve
    fn(ctx, dev(a), dev(b), dev(c), dd, (n, nlines, 1, 1, n, 0), coef_strides=(0, 1, 0), P=P)
    assert line_relerr(host(dd), ref.reshape(nlines, n), axis=1) <= TOL


@pytest.mark.parametrize("mname,method", METHODS)
@pytest.mark.parametrize("periodic", [False, True])
def test_general_per_element_coefficients(T, ctx, orc, mname, method, periodic):
    """Fully general rows (a, b, c per element, non-symmetric) through the general kernel."""
    n, P, nlines = 48, 4, 130
    rng = np.random.default_rng(40)
    A = np.empty((nlines, n)); B = np.empty((nlines, n)); C = np.empty((nlines, n))
    for s in range(nlines):
        A[s], B[s], C[s] = W.random_tridiag(n, rng, margin=0.5, periodic=periodic)
    D = rng.uniform(-1, 1, (n, nlines))                  # [j][line]
    At, Bt, Ct = (np.ascontiguousarray(X.T) for X in (A, B, C))
    ref = D.copy().ravel()
    orc.solve_batch(_oracle_method(orc, mname), ref, n, nlines, 1, s_j=nlines, s_b0=1, s_b1=0,
                    a=At.ravel(), b=Bt.ravel(), c=Ct.ravel(), cs_j=nlines, cs_b0=1, cs_b1=0,
                    P=P, periodic=periodic)
    dd = dev(D)
    fn = T.tri_pdd_solve if method == 0 else T.tri_ppt_solve
    fn(ctx, dev(At), dev(Bt), dev(Ct), dd, (n, nlines, 1, nlines, 1, 0),
       coef_strides=(nlines, 1, 0), P=P, periodic=periodic)
    T.tri_sync_status(ctx)
    assert line_relerr(host(dd), ref.reshape(n, nlines), axis=0) <= TOL


# ---------------------------------------------------------------------------
# ADI sweeps (shared matrices): strided y/z kernel, contiguous x kernel
# ---------------------------------------------------------------------------
def _sweep_case(direction, Nz, Ny, Nx, P, periodic, mname, T, ctx, orc, coef=None, seed=3):
    u = W.cfg_field(Nx, Ny, Nz, seed=seed)
    n = (Nx, Ny, Nz)[direction]
    if coef is None:
        rng = np.random.default_rng(seed + 100)
        coef = W.random_tridiag(n, rng, margin=0.7, periodic=periodic)
    a, b, c = coef
    ref = u.copy()
    orc.adi_sweep(_oracle_method(orc, mname), direction, ref, a, b, c, P, periodic)
    du = dev(u)
    T.adi_sweep(ctx, direction, du, dev(a), dev(b), dev(c), P, periodic=periodic,
                method=0 if mname == "PDD" else 1)
    T.tri_sync_status(ctx)
    got = host(du)
    axis = 2 - direction
    return line_relerr(got, ref, axis=axis)


@pytest.mark.parametrize("mname", ["PDD", "PPT"])
@pytest.mark.parametrize("Nx,P", [(256, 8), (200, 8), (2048, 8), (96, 3), (64, 16), (1024, 2)])
def test_adi_x_contiguous(T, ctx, orc, mname, Nx, P):
    assert _sweep_case(0, 5, 7, Nx, P, False, mname, T, ctx, orc) <= TOL


@pytest.mark.parametrize("mname", ["PDD", "PPT"])
@pytest.mark.parametrize("Ny,P,Nx", [(256, 4, 200), (64, 4, 130), (128, 16, 64), (160, 2, 70),
                                     (24, 3, 65), (256, 8, 64)])
def test_adi_y_strided(T, ctx, orc, mname, Ny, P, Nx):
    assert _sweep_case(1, 3, Ny, Nx, P, False, mname, T, ctx, orc) <= TOL


@pytest.mark.parametrize("mname", ["PDD", "PPT"])
@pytest.mark.parametrize("Nz,P", [(288, 4), (96, 4), (48, 1), (30, 5), (64, 16)])
def test_adi_z_periodic(T, ctx, orc, mname, Nz, P):
    assert _sweep_case(2, Nz, 6, 70, P, True, mname, T, ctx, orc) <= TOL


@pytest.mark.parametrize("mname", ["PDD", "PPT"])
def test_adi_momentum_coefficients(T, ctx, orc, mname):
    """The momentum matrices of the benchmark (uniform x, tanh y, periodic z)."""
    Nz, Ny, Nx = 24, 256, 2048
    assert _sweep_case(0, 4, 8, Nx, 8, False, mname, T, ctx, orc, coef=W.momentum_uniform(Nx)) <= TOL
    assert _sweep_case(1, 3, Ny, 130, 4, False, mname, T, ctx, orc, coef=W.momentum_stretched(Ny)) <= TOL
    assert _sweep_case(2, 288, 4, 70, 4, True, mname, T, ctx, orc, coef=W.momentum_periodic(288)) <= TOL


def test_adi_composition_xyz(T, ctx, orc):
    """x, then y, then periodic z over the same field, in place."""
    Nz, Ny, Nx = 24, 64, 256
    u = W.cfg_field(Nx, Ny, Nz, seed=5)
    cx, cy, cz = W.momentum_uniform(Nx), W.momentum_stretched(Ny), W.momentum_periodic(Nz)
    ref = u.copy()
    du = dev(u)
    for direction, (a, b, c), P, per in ((0, cx, 8, False), (1, cy, 4, False), (2, cz, 4, True)):
        orc.adi_sweep(orc.PDD, direction, ref, a, b, c, P, per)
        T.adi_sweep(ctx, direction, du, dev(a), dev(b), dev(c), P, periodic=per, method=0)
    got = host(du)
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) <= TOL


# ---------------------------------------------------------------------------
# Poisson wavenumber solves (complex field, per-k matrices, k = 0 pinned)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("Nx,Ny,Nz,P", [(70, 64, 48, 4), (130, 256, 24, 4), (64, 128, 16, 8),
                                        (33, 32, 12, 2)])
def test_poisson_wavenumber(T, ctx, orc, Nx, Ny, Nz, P):
    phihat = W.cfg_poisson_rhs(Nx, Ny, Nz, seed=0)
    ay, cy = W.poisson_metric(Ny)
    lam = W.modified_wavenumbers(Nz)
    ref = phihat.copy()
    orc.poisson(ref, ay, cy, lam, P=P)
    dphi = torch.as_tensor(phihat).cuda()
    T.poisson_wavenumber_solve(ctx, dphi, dev(ay), dev(cy), dev(lam), P=P)
    T.tri_sync_status(ctx)
    got = host(dphi)
    assert np.all(got[0, 0, :] == 0)                    # gauge-pinned row of the k = 0 mode
    assert line_relerr(got, ref, axis=1) <= TOL


def test_tri_ppt_complex_field(T, ctx, orc):
    """tri_ppt_solve on an interleaved complex field, one real matrix per b1."""
    Ny, Nx, Nk, P = 64, 40, 5, 4
    rng = np.random.default_rng(8)
    mats = [W.random_tridiag(Ny, rng, margin=0.2) for _ in range(Nk)]
    A = np.array([m[0] for m in mats]); B = np.array([m[1] for m in mats]); C = np.array([m[2] for m in mats])
    phi = rng.standard_normal((Nk, Ny, Nx)) + 1j * rng.standard_normal((Nk, Ny, Nx))
    ref = phi.copy()
    for k in range(Nk):
        for i in range(Nx):
            ref[k, :, i] = (orc.ppt(A[k], B[k], C[k], phi[k, :, i].real, P)
                            + 1j * orc.ppt(A[k], B[k], C[k], phi[k, :, i].imag, P))
    dphi = torch.as_tensor(phi).cuda()
    T.tri_ppt_solve(ctx, dev(A), dev(B), dev(C), dphi, (Ny, Nx, Nk, Nx, 1, Nx * Ny),
                    coef_strides=(1, 0, Ny), complex_field=True, P=P)
    assert line_relerr(host(dphi), ref, axis=1) <= TOL


# ---------------------------------------------------------------------------
# Bit-exact indexing and partitioning probes
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("layout", ["x", "y", "z"])
@pytest.mark.parametrize("P", [1, 2, 4, 8])
def test_bitexact_diagonal_probe(T, ctx, orc, layout, P):
    """a = c = 0, b = powers of two, integer d: every result is exact, so any
    misplaced row, line or partition shows up as a bitwise difference."""
    Nz, Ny, Nx = 16, 32, 136
    direction = "xyz".index(layout)
    n = (Nx, Ny, Nz)[direction]
    rng = np.random.default_rng(50 + P)
    u = rng.integers(-1000, 1000, (Nz, Ny, Nx)).astype(np.float64)
    a = np.zeros(n); c = np.zeros(n)
    b = 2.0 ** rng.integers(-3, 4, n)
    per = layout == "z"
    for mname in ("PDD", "PPT"):
        ref = u.copy()
        orc.adi_sweep(_oracle_method(orc, mname), direction, ref, a, b, c, P, per)
        du = dev(u)
        T.adi_sweep(ctx, direction, du, dev(a), dev(b), dev(c), P, periodic=per,
                    method=0 if mname == "PDD" else 1)
        assert np.array_equal(host(du), ref), mname


@pytest.mark.parametrize("P", [2, 4])
@pytest.mark.parametrize("which", ["c", "a"])
def test_bitexact_one_sided_coupling(T, ctx, orc, P, which):
    """b = 1 and only one off-diagonal (1/4): short lines stay exact in FP64 through
    the elimination, the spikes, the interface solve and the correction."""
    n, nlines = 16, 128
    rng = np.random.default_rng(60 + P)
    a = np.zeros(n); c = np.zeros(n); b = np.ones(n)
    (c if which == "c" else a)[:] = 0.25
    a[0] = 0.0; c[-1] = 0.0
    D = rng.integers(-64, 64, (n, nlines)).astype(np.float64)
    for mname, fn in (("PDD", T.tri_pdd_solve), ("PPT", T.tri_ppt_solve)):
        ref = D.copy().ravel()
        orc.solve_batch(_oracle_method(orc, mname), ref, n, nlines, 1, nlines, 1, 0, a, b, c, P=P)
        exact = orc.thomas(a, b, c, D[:, 0])
        dd = dev(D)
        fn(ctx, dev(a), dev(b), dev(c), dd, (n, nlines, 1, nlines, 1, 0), P=P)
        got = host(dd)
        assert np.array_equal(got, ref.reshape(n, nlines)), mname
        if mname == "PPT":
            assert np.array_equal(got[:, 0], exact)


# ---------------------------------------------------------------------------
# Edge cases and error paths
# ---------------------------------------------------------------------------
def test_empty_batches_are_noops(T, ctx):
    a = dev(np.zeros(8)); b = dev(np.ones(8))
    d = dev(np.zeros(1))
    T.tri_pdd_solve(ctx, a, b, a, d, (8, 0, 5, 1, 8, 0), P=2)
    T.tri_ppt_solve(ctx, a, b, a, d, (8, 3, 0, 1, 8, 0), P=2)
    T.tri_sync_status(ctx)


@pytest.mark.parametrize("n,P", [(2, 1), (4, 2), (32, 16), (3, 1), (6, 3)])
def test_minimal_partitions(T, ctx, orc, n, P):
    nlines = 70
    rng = np.random.default_rng(n * 10 + P)
    a, b, c = W.random_tridiag(n, rng, margin=0.5)
    D = rng.uniform(-1, 1, (n, nlines))
    for mname, fn in (("PDD", T.tri_pdd_solve), ("PPT", T.tri_ppt_solve)):
        ref = D.copy().ravel()
        orc.solve_batch(_oracle_method(orc, mname), ref, n, nlines, 1, nlines, 1, 0, a, b, c, P=P)
        dd = dev(D)
        fn(ctx, dev(a), dev(b), dev(c), dd, (n, nlines, 1, nlines, 1, 0), P=P)
        assert line_relerr(host(dd), ref.reshape(n, nlines), axis=0) <= TOL


@pytest.mark.parametrize("direction,n,P,per", [(1, 640, 4, False), (1, 640, 16, False), (2, 640, 8, True),
                                           (1, 640, 1, False), (0, 4096, 8, False), (0, 8192, 16, False)])
@pytest.mark.parametrize("mname", ["PDD", "PPT"])
def test_longest_supported_lines(T, ctx, orc, direction, n, P, per, mname):
    """The longest lines each layout takes: strided lines of 640 rows (at most
    16 wavefronts of at most 80 rows, 40 above 8 wavefronts); contiguous lines
    of 4096 (register-factor kernel, P = 8) and 8192 (1024 lanes of 8 rows,
    P = 16)."""
    shape = {0: (3, 5, n), 1: (2, n, 70), 2: (n, 3, 70)}[direction]
    rng = np.random.default_rng(n + P)
    coef = W.random_tridiag(n, rng, margin=0.7, periodic=per)
    assert _sweep_case(direction, *shape, P, per, mname, T, ctx, orc, coef=coef) <= TOL


@pytest.mark.parametrize("direction,n,P", [(1, 656, 4), (1, 656, 16), (0, 16384, 16)])
def test_lines_beyond_the_limits_are_refused(T, ctx, direction, n, P):
    """One step past the longest supported lines: TRI_E_UNSUPPORTED, data untouched."""
    shape = {0: (1, 2, n), 1: (1, n, 64)}[direction]
    u0 = np.arange(np.prod(shape), dtype=np.float64).reshape(shape)
    du = dev(u0)
    a, b, c = (dev(v) for v in W.momentum_uniform(n))
    with pytest.raises(T.TriError) as e:
        T.adi_sweep(ctx, direction, du, a, b, c, P)
    assert e.value.status == T.TRI_E_UNSUPPORTED
    T.tri_sync_status(ctx)
    assert np.array_equal(host(du), u0)


def test_shape_errors_leave_data_untouched(T, ctx):
    d0 = np.arange(60.0).reshape(12, 5)
    dd = dev(d0)
    a = dev(np.zeros(12)); b = dev(np.ones(12))
    for P, code in ((5, T.TRI_E_SHAPE), (0, T.TRI_E_SHAPE), (17, T.TRI_E_SHAPE), (12, T.TRI_E_SHAPE)):
        with pytest.raises(T.TriError) as e:
            T.tri_pdd_solve(ctx, a, b, a, dd, (12, 5, 1, 5, 1, 0), P=P)
        assert e.value.status == code
    assert np.array_equal(host(dd), d0)


def test_zero_pivot_reported(T, ctx):
    n, nlines = 16, 64
    a = np.zeros(n); c = np.zeros(n); b = np.ones(n)
    b[5] = 0.0
    dd = dev(np.ones((n, nlines)))
    T.tri_ppt_solve(ctx, dev(a), dev(b), dev(c), dd, (n, nlines, 1, nlines, 1, 0), P=2)
    with pytest.raises(T.TriError) as e:
        T.tri_sync_status(ctx)
    assert e.value.status == T.TRI_E_ZERO_PIVOT
    T.tri_sync_status(ctx)          # cleared after being reported


def test_pdd_drop_reported(T, ctx):
    """tri_info.pdd_drop_max: the largest entry PDD drops; tiny for the
    momentum matrices, O(1) for the low-k Poisson ones."""
    Nz, Ny, Nx = 4, 256, 64
    a, b, c = W.momentum_stretched(Ny)
    du = dev(W.cfg_field(Nx, Ny, Nz))
    info = T.adi_sweep(ctx, 1, du, dev(a), dev(b), dev(c), 4, method=0, info=True)
    assert info["pdd_drop_max"] < 1e-14
    info = T.adi_sweep(ctx, 1, du, dev(a), dev(b), dev(c), 16, method=0, info=True)
    assert info["pdd_drop_max"] > 1e-8


def _pdd_dropped_max(A, B, C, P, periodic):
    """Largest entry PDD drops, from the exact partition spikes: per partition, the
    left spike at its last row and the right spike at its first row, where both
    interfaces exist."""
    nlines, n = B.shape
    m = n // P
    worst = 0.0
    for s in range(nlines):
        for r in range(P):
            if not periodic and (r == 0 or r == P - 1):
                continue
            lo = r * m
            blk = np.diag(B[s, lo:lo + m]) + np.diag(A[s, lo + 1:lo + m], -1) + np.diag(C[s, lo:lo + m - 1], 1)
            e1 = np.zeros(m); e1[0] = A[s, lo]
            em = np.zeros(m); em[-1] = C[s, lo + m - 1]
            worst = max(worst, abs(np.linalg.solve(blk, e1)[-1]), abs(np.linalg.solve(blk, em)[0]))
    return worst


def test_strict_pdd_shared_matrix(T, ctx):
    """tri_set_pdd_tolerance: with a tolerance set, a shared-matrix PDD solve whose
    dropped entries exceed it makes tri_sync_status report TRI_E_PDD_UNSAFE; one
    whose dropped entries stay below it does not; tolerance 0 turns the check off."""
    Nz, Ny, Nx = 4, 256, 64
    a, b, c = (dev(v) for v in W.momentum_stretched(Ny))
    du = dev(W.cfg_field(Nx, Ny, Nz))
    T.tri_sync_status(ctx)
    try:
        T.tri_set_pdd_tolerance(ctx, 1e-12)
        T.adi_sweep(ctx, 1, du, a, b, c, 4, method=T.TRI_PDD)          # drops < 1e-14
        T.tri_sync_status(ctx)
        T.adi_sweep(ctx, 1, du, a, b, c, 16, method=T.TRI_PDD)         # drops > 1e-8
        with pytest.raises(T.TriError) as e:
            T.tri_sync_status(ctx)
        assert e.value.status == T.TRI_E_PDD_UNSAFE
        T.tri_sync_status(ctx)                                          # cleared once reported
        T.adi_sweep(ctx, 1, du, a, b, c, 16, method=T.TRI_PPT)         # PPT drops nothing
        T.tri_sync_status(ctx)
        T.tri_set_pdd_tolerance(ctx, 0.0)
        T.adi_sweep(ctx, 1, du, a, b, c, 16, method=T.TRI_PDD)
        T.tri_sync_status(ctx)
    finally:
        T.tri_set_pdd_tolerance(ctx, 0.0)
    L = T.lib()
    assert L.tri_set_pdd_tolerance(ctx, ctypes.c_double(-1.0)) == T.TRI_E_ARG
    assert L.tri_set_pdd_tolerance(ctx, ctypes.c_double(float("nan"))) == T.TRI_E_ARG



def test_strict_pdd_plan_reports_at_creation(T, ctx, monkeypatch):
    """A plan created under a tolerance checks its PDD items when it computes
    their tables: a y item at P = 16 (dropped entries > 1e-8) is reported by the
    next tri_sync_status, the same item at P = 4 is not, and executing the plan
    reports nothing further."""
    monkeypatch.setenv("TRI_AUTOTUNE", "0")
    Nz, Ny, Nx = 4, 256, 64
    a, b, c = (dev(v) for v in W.momentum_stretched(Ny))
    u = dev(W.cfg_field(Nx, Ny, Nz))
    item = lambda P: [dict(kind=T.TRI_ITEM_ADI_Y, field=u, Nx=Nx, Ny=Ny, Nz=Nz, a=a, b=b, c=c, P=P,
                           periodic=0, method=T.TRI_PDD)]
    T.tri_sync_status(ctx)
    try:
        T.tri_set_pdd_tolerance(ctx, 1e-12)
        safe = T.tri_plan_create(ctx, item(4))
        T.tri_sync_status(ctx)
        unsafe = T.tri_plan_create(ctx, item(16))
        with pytest.raises(T.TriError) as e:
            T.tri_sync_status(ctx)
        assert e.value.status == T.TRI_E_PDD_UNSAFE
        T.tri_plan_execute(unsafe)
        T.tri_plan_execute(safe)
        T.tri_sync_status(ctx)
        T.tri_plan_destroy(unsafe)
        T.tri_plan_destroy(safe)
    finally:
        T.tri_set_pdd_tolerance(ctx, 0.0)

@pytest.mark.parametrize("periodic", [False, True])
def test_strict_pdd_per_line_coefficients(T, ctx, orc, periodic):
    """The same check in the per-line kernel: strongly dominant lines in long
    partitions stay below the tolerance (and match the oracle's PDD); weakly
    dominant lines in short partitions exceed it."""
    nlines, n, tol = 100, 128, 1e-12
    rng = np.random.default_rng(77 + periodic)
    cases = ((4, 3.0, False), (16, 0.02, True))        # (P, margin, expect the report)
    try:
        T.tri_set_pdd_tolerance(ctx, tol)
        for P, margin, unsafe in cases:
            A = np.empty((nlines, n)); B = np.empty((nlines, n)); C = np.empty((nlines, n))
            for s in range(nlines):
                A[s], B[s], C[s] = W.random_tridiag(n, rng, periodic=periodic, margin=margin)
            assert (_pdd_dropped_max(A, B, C, P, periodic) > tol) == unsafe   # the fixture's side
            D = rng.uniform(-1, 1, (n, nlines))
            At, Bt, Ct = (np.ascontiguousarray(X.T) for X in (A, B, C))
            dd = dev(D)
            T.tri_pdd_solve(ctx, dev(At), dev(Bt), dev(Ct), dd, (n, nlines, 1, nlines, 1, 0),
                            coef_strides=(nlines, 1, 0), P=P, periodic=periodic)
            if unsafe:
                with pytest.raises(T.TriError) as e:
                    T.tri_sync_status(ctx)
                assert e.value.status == T.TRI_E_PDD_UNSAFE
            else:
                T.tri_sync_status(ctx)
                ref = D.copy().ravel()
                orc.solve_batch(orc.PDD, ref, n, nlines, 1, s_j=nlines, s_b0=1, s_b1=0, a=At.ravel(),
                                b=Bt.ravel(), c=Ct.ravel(), cs_j=nlines, cs_b0=1, cs_b1=0, P=P,
                                periodic=periodic)
                assert line_relerr(host(dd), ref.reshape(n, nlines), axis=0) <= TOL
    finally:
        T.tri_set_pdd_tolerance(ctx, 0.0)


# ---------------------------------------------------------------------------
# Plans and HIP graphs
# ---------------------------------------------------------------------------
def test_plan_execute_and_graph_replay(T, ctx, orc, monkeypatch):
    monkeypatch.setenv("TRI_AUTOTUNE", "0")     # same launch shapes as the one-shot calls
    Nz, Ny, Nx = 24, 64, 256
    u0 = W.cfg_field(Nx, Ny, Nz, seed=9)
    phi0 = W.cfg_poisson_rhs(Nx, Ny, Nz, seed=9)
    cx, cy, cz = W.momentum_uniform(Nx), W.momentum_stretched(Ny), W.momentum_periodic(Nz)
    ay, cyp = W.poisson_metric(Ny)
    lam = W.modified_wavenumbers(Nz)
    coefs = [tuple(dev(v) for v in cf) for cf in (cx, cy, cz)]
    pa, pc, pl = dev(ay), dev(cyp), dev(lam)
    # eager reference through the one-shot calls
    ue = dev(u0); pe = torch.as_tensor(phi0).cuda()
    for direction, P, per in ((0, 8, False), (1, 4, False), (2, 4, True)):
        T.adi_sweep(ctx, direction, ue, *coefs[direction], P, periodic=per, method=0)
    T.poisson_wavenumber_solve(ctx, pe, pa, pc, pl, P=4)
    ue_h, pe_h = host(ue), host(pe)
    # oracle
    ref = u0.copy()
    for direction, (a, b, c), P, per in ((0, cx, 8, False), (1, cy, 4, False), (2, cz, 4, True)):
        orc.adi_sweep(orc.PDD, direction, ref, a, b, c, P, per)
    assert np.max(np.abs(ue_h - ref)) / np.max(np.abs(ref)) <= TOL
    # plan (strided solves of one kernel instance batched, the others in their
    # own launches: the same kernels as the one-shot calls, so the same bits)
    monkeypatch.setenv("TRI_BATCH", "1")
    up = dev(u0); pp = torch.as_tensor(phi0).cuda()
    items = [dict(kind=T.TRI_ITEM_ADI_X, field=up, Nx=Nx, Ny=Ny, Nz=Nz, a=coefs[0][0], b=coefs[0][1],
                  c=coefs[0][2], P=8, periodic=0, method=0),
             dict(kind=T.TRI_ITEM_ADI_Y, field=up, Nx=Nx, Ny=Ny, Nz=Nz, a=coefs[1][0], b=coefs[1][1],
                  c=coefs[1][2], P=4, periodic=0, method=0),
             dict(kind=T.TRI_ITEM_ADI_Z, field=up, Nx=Nx, Ny=Ny, Nz=Nz, a=coefs[2][0], b=coefs[2][1],
                  c=coefs[2][2], P=4, periodic=1, method=0),
             dict(kind=T.TRI_ITEM_POISSON, field=pp, Nx=Nx, Ny=Ny, Nz=Nz // 2 + 1, a=pa, c=pc, lam=pl,
                  P=4, method=1)]
    plan = T.tri_plan_create(ctx, items)
    try:
        T.tri_plan_execute(plan)
        assert np.array_equal(host(up), ue_h)
        assert np.array_equal(host(pp), pe_h)
        T.tri_plan_capture(plan)
        for rep in range(3):
            up.copy_(dev(u0)); pp.copy_(torch.as_tensor(phi0).cuda())
            torch.cuda.synchronize()
            T.tri_plan_graph_launch(plan)
            _ = (up * 2).sum()            # unrelated eager work between replays
            assert np.array_equal(host(up), ue_h), rep
            assert np.array_equal(host(pp), pe_h), rep
    finally:
        T.tri_plan_destroy(plan)


# ---------------------------------------------------------------------------
# Every launch shape the tuner can pick (forced through the environment)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("direction,n,P,per,kc", [
    (1, 256, 4, False, 1), (1, 256, 4, False, 2), (1, 256, 4, False, 4), (1, 128, 2, False, 4),
    (2, 288, 4, True, 1), (2, 288, 4, True, 2), (2, 288, 4, True, 3), (2, 288, 2, True, 2),
    (2, 288, 2, True, 4), (1, 96, 16, False, 1), (1, 192, 8, False, 2)])
@pytest.mark.parametrize("mname", ["PDD", "PPT"])
def test_strided_chunk_counts(T, ctx, orc, monkeypatch, direction, n, P, per, kc, mname):
    monkeypatch.setenv("TRI_FORCE_KC", str(kc))
    shape = {1: (3, n, 200), 2: (n, 5, 130)}[direction]
    assert _sweep_case(direction, *shape, P, per, mname, T, ctx, orc) <= TOL


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("direction,n,P,per,kc", [(1, 256, 4, False, 2), (2, 288, 4, True, 1), (1, 96, 3, False, 1)])
@pytest.mark.parametrize("mname", ["PDD", "PPT"])
def test_strided_workgroup_orders(T, ctx, orc, monkeypatch, order, direction, n, P, per, kc, mname):
    """Workgroup -> line-group orders the tuner may pick (outer index fastest;
    contiguous ranges per XCD) on ragged batches (line groups and workgroup
    counts not multiples of 64 or 8)."""
    monkeypatch.setenv("TRI_FORCE_KC", str(kc))
    monkeypatch.setenv("TRI_BLK_MAP", str(order))
    shape = {1: (7, n, 201), 2: (n, 11, 130)}[direction]
    assert _sweep_case(direction, *shape, P, per, mname, T, ctx, orc) <= TOL


@pytest.mark.parametrize("direction,n,P,per", [(1, 64, 4, False), (2, 288, 16, True), (1, 96, 4, False),
                                           (2, 48, 2, True), (1, 256, 16, False)])
@pytest.mark.parametrize("mname", ["PDD", "PPT"])
def test_strided_two_lines_per_lane(T, ctx, orc, monkeypatch, direction, n, P, per, mname):
    """Two neighbouring lines per lane (16-byte accesses), one wavefront per
    partition (line counts that are not multiples of 128)."""
    monkeypatch.setenv("TRI_LPL", "2")
    monkeypatch.setenv("TRI_FORCE_KC", "1")
    shape = {1: (3, n, 130), 2: (n, 5, 130)}[direction]
    assert _sweep_case(direction, *shape, P, per, mname, T, ctx, orc) <= TOL


@pytest.mark.parametrize("mname,method", METHODS)
def test_strided_two_lines_per_lane_odd_tail(T, ctx, orc, monkeypatch, mname, method):
    """An odd number of adjacent lines (131) in rows padded to 132: the last
    lane holds one line and uses 8-byte accesses."""
    monkeypatch.setenv("TRI_LPL", "2")
    monkeypatch.setenv("TRI_FORCE_KC", "1")
    n, P, nb0, nb1, sj = 64, 4, 131, 3, 132
    rng = np.random.default_rng(91)
    a, b, c = W.random_tridiag(n, rng, margin=0.6, periodic=False)
    buf = rng.standard_normal(n * sj * nb1)
    ref = buf.copy()
    orc.solve_batch(_oracle_method(orc, mname), ref, n, nb0, nb1, s_j=sj, s_b0=1, s_b1=n * sj,
                    a=a, b=b, c=c, cs_j=1, cs_b0=0, cs_b1=0, P=P)
    dd = dev(buf)
    fn = T.tri_pdd_solve if method == 0 else T.tri_ppt_solve
    fn(ctx, dev(a), dev(b), dev(c), dd, (n, nb0, nb1, sj, 1, n * sj), coef_strides=(1, 0, 0), P=P)
    T.tri_sync_status(ctx)
    got = host(dd)
    idx = (np.arange(nb1)[:, None, None] * n * sj + np.arange(n)[None, :, None] * sj +
           np.arange(nb0)[None, None, :])
    assert line_relerr(got[idx], ref[idx], axis=1) <= TOL
    pad = np.ones(buf.size, bool)
    pad[idx.ravel()] = False
    assert np.array_equal(got[pad], buf[pad])            # padding untouched


def test_poisson_two_lines_per_lane(T, ctx, orc, monkeypatch):
    monkeypatch.setenv("TRI_LPL", "2")
    monkeypatch.setenv("TRI_FORCE_KC", "1")
    Nx, Ny, Nz, P = 70, 256, 24, 16
    phihat = W.cfg_poisson_rhs(Nx, Ny, Nz, seed=5)
    ay, cy = W.poisson_metric(Ny)
    lam = W.modified_wavenumbers(Nz)
    ref = phihat.copy()
    orc.poisson(ref, ay, cy, lam, P=P)
    dphi = torch.as_tensor(phihat).cuda()
    T.poisson_wavenumber_solve(ctx, dphi, dev(ay), dev(cy), dev(lam), P=P)
    assert line_relerr(host(dphi), ref, axis=1) <= TOL


@pytest.mark.parametrize("Nx,P,C", [(2048, 8, 4), (2048, 8, 8), (2048, 8, 16), (256, 8, 4), (256, 8, 8),
                                    (256, 8, 16), (512, 2, 16), (384, 4, 8), (1024, 16, 4)])
@pytest.mark.parametrize("mname", ["PDD", "PPT"])
def test_contiguous_rows_per_lane(T, ctx, orc, monkeypatch, Nx, P, C, mname):
    monkeypatch.setenv("TRI_FORCE_C", str(C))
    assert _sweep_case(0, 5, 7, Nx, P, False, mname, T, ctx, orc) <= TOL


@pytest.mark.parametrize("Nx,P,C,per", [(2048, 8, 8, False), (2048, 8, 4, False), (256, 8, 4, False),
                                        (512, 2, 8, False), (512, 2, 4, True), (1024, 16, 8, True),
                                        (1024, 16, 4, False), (2048, 4, 8, True)])
@pytest.mark.parametrize("mname", ["PDD", "PPT"])
def test_contiguous_register_factor_kernel(T, ctx, orc, monkeypatch, Nx, P, C, per, mname):
    """Register-factor contiguous kernel (tuning value 100 + C), fewer lines than workgroups."""
    monkeypatch.setenv("TRI_FORCE_C", str(100 + C))
    assert _sweep_case(0, 5, 7, Nx, P, per, mname, T, ctx, orc) <= TOL


@pytest.mark.parametrize("C", [4, 8])
@pytest.mark.parametrize("mname", ["PDD", "PPT"])
def test_contiguous_register_factor_persistent(T, ctx, orc, monkeypatch, C, mname):
    """Many more lines than resident workgroups, so every workgroup loops over
    several lines through both staging buffers; the line count is odd."""
    monkeypatch.setenv("TRI_FORCE_C", str(100 + C))
    assert _sweep_case(0, 41, 37, 2048, 8, False, mname, T, ctx, orc, coef=W.momentum_uniform(2048)) <= TOL


@pytest.mark.parametrize("mname,method", METHODS)
def test_contiguous_register_factor_padded_batch(T, ctx, orc, monkeypatch, mname, method):
    """Contiguous lines in a 2-D batch whose outer stride is padded (lines are
    not evenly spaced), one shared matrix."""
    monkeypatch.setenv("TRI_FORCE_C", "108")
    n, P, nb0, nb1, pad = 1024, 8, 30, 23, 6
    s_b0, s_b1 = n + 2, (n + 2) * nb0 + pad
    rng = np.random.default_rng(77)
    a, b, c = W.random_tridiag(n, rng, margin=0.6, periodic=False)
    buf = rng.standard_normal(s_b1 * nb1)
    ref = buf.copy()
    orc.solve_batch(_oracle_method(orc, mname), ref, n, nb0, nb1, s_j=1, s_b0=s_b0, s_b1=s_b1,
                    a=a, b=b, c=c, cs_j=1, cs_b0=0, cs_b1=0, P=P)
    dd = dev(buf)
    fn = T.tri_pdd_solve if method == 0 else T.tri_ppt_solve
    fn(ctx, dev(a), dev(b), dev(c), dd, (n, nb0, nb1, 1, s_b0, s_b1), coef_strides=(1, 0, 0), P=P)
    T.tri_sync_status(ctx)
    got = host(dd)
    idx = (np.arange(nb1)[:, None, None] * s_b1 + np.arange(nb0)[None, :, None] * s_b0 +
           np.arange(n)[None, None, :])
    assert line_relerr(got[idx], ref[idx], axis=2) <= TOL
    gap = np.ones(buf.size, bool)
    gap[idx.ravel()] = False
    assert np.array_equal(got[gap], buf[gap])           # padding untouched


def test_poisson_chunked(T, ctx, orc, monkeypatch):
    monkeypatch.setenv("TRI_FORCE_KC", "2")
    Nx, Ny, Nz, P = 70, 256, 24, 4
    phihat = W.cfg_poisson_rhs(Nx, Ny, Nz, seed=2)
    ay, cy = W.poisson_metric(Ny)
    lam = W.modified_wavenumbers(Nz)
    ref = phihat.copy()
    orc.poisson(ref, ay, cy, lam, P=P)
    dphi = torch.as_tensor(phihat).cuda()
    T.poisson_wavenumber_solve(ctx, dphi, dev(ay), dev(cy), dev(lam), P=P)
    assert line_relerr(host(dphi), ref, axis=1) <= TOL


def test_autotuned_plan_matches_oracle(T, ctx, orc, monkeypatch):
    """Plan creation times the candidate launch shapes on scratch memory and
    keeps the fastest; the caller's field must be left untouched until execute."""
    monkeypatch.setenv("TRI_AUTOTUNE", "1")
    Nz, Ny, Nx = 48, 256, 512
    u0 = W.cfg_field(Nx, Ny, Nz, seed=11)
    cy_ = W.momentum_stretched(Ny)
    cz_ = W.momentum_periodic(Nz)
    cx_ = W.momentum_uniform(Nx)
    u = dev(u0)
    coefs = [tuple(dev(v) for v in c) for c in (cx_, cy_, cz_)]
    items = [dict(kind=d, field=u, Nx=Nx, Ny=Ny, Nz=Nz, a=coefs[d][0], b=coefs[d][1], c=coefs[d][2],
                  P=(8, 4, 4)[d], periodic=int(d == 2), method=0) for d in range(3)]
    plan = T.tri_plan_create(ctx, items)
    try:
        assert np.array_equal(host(u), u0)              # tuning never touches the field
        descr = [T.tri_plan_item_describe(plan, i) for i in range(3)]
        assert all("tuned=" in d for d in descr), descr
        T.tri_plan_execute(plan)
        ref = u0.copy()
        for d, (a, b, c) in enumerate((cx_, cy_, cz_)):
            orc.adi_sweep(orc.PDD, d, ref, a, b, c, (8, 4, 4)[d], d == 2)
        got = host(u)
        assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) <= TOL
    finally:
        T.tri_plan_destroy(plan)


@pytest.mark.parametrize("n,P,periodic", [(48, 4, False), (48, 2, False), (64, 2, False), (48, 8, False),
                                          (24, 4, True), (36, 3, True)])
def test_general_non_dominant_diagonal_pivoting(T, ctx, orc, n, P, periodic):
    """Rows far from diagonal dominance (zero diagonal entries every 7th row): the
    per-line PPT solve picks 2x2 pivots where a 1x1 pivot would be zero or small, and
    reaches A^{-1} d.  Each line's error is held to max(1e-12, 64 eps kappa), kappa the
    largest condition number of the line and of its partition blocks."""
    nlines = 150
    rng = np.random.default_rng(900 + n + P)
    A = np.empty((nlines, n)); B = np.empty((nlines, n)); C = np.empty((nlines, n))
    for s in range(nlines):
        A[s], B[s], C[s] = W.random_tridiag_nondominant(n, rng, periodic=periodic)
    D = rng.uniform(-1, 1, (n, nlines))
    At, Bt, Ct = (np.ascontiguousarray(X.T) for X in (A, B, C))
    dd = dev(D)
    T.tri_ppt_solve(ctx, dev(At), dev(Bt), dev(Ct), dd, (n, nlines, 1, nlines, 1, 0),
                    coef_strides=(nlines, 1, 0), P=P, periodic=periodic)
    T.tri_sync_status(ctx)                      # no zero pivot reported
    got = host(dd)
    m = n // P
    for s in range(nlines):
        ref = orc.dense_solve(A[s], B[s], C[s], D[:, s], periodic)
        full = np.diag(B[s]) + np.diag(A[s, 1:], -1) + np.diag(C[s, :-1], 1)
        if periodic:
            full[0, -1] += A[s, 0]
            full[-1, 0] += C[s, -1]
        kappa = np.linalg.cond(full)
        for r in range(P):
            blk = full[r * m:(r + 1) * m, r * m:(r + 1) * m]
            kappa = max(kappa, np.linalg.cond(blk))
        err = np.max(np.abs(got[:, s] - ref)) / np.max(np.abs(ref))
        assert err <= max(TOL, 64 * 2.2e-16 * kappa), (s, err, kappa)


def test_general_pivoting_keeps_dominant_rows_on_1x1_pivots(T, ctx, orc):
    """On diagonally dominant rows the pivot test never takes a 2x2 block: the result
    matches the oracle's PPT (Thomas blocks) as before."""
    n, P, nlines = 64, 4, 130
    rng = np.random.default_rng(41)
    A = np.empty((nlines, n)); B = np.empty((nlines, n)); C = np.empty((nlines, n))
    for s in range(nlines):
        A[s], B[s], C[s] = W.random_tridiag(n, rng, margin=0.05)
    D = rng.uniform(-1, 1, (n, nlines))
    At, Bt, Ct = (np.ascontiguousarray(X.T) for X in (A, B, C))
    ref = D.copy().ravel()
    orc.solve_batch(orc.PPT, ref, n, nlines, 1, s_j=nlines, s_b0=1, s_b1=0, a=At.ravel(), b=Bt.ravel(),
                    c=Ct.ravel(), cs_j=nlines, cs_b0=1, cs_b1=0, P=P)
    dd = dev(D)
    T.tri_ppt_solve(ctx, dev(At), dev(Bt), dev(Ct), dd, (n, nlines, 1, nlines, 1, 0), coef_strides=(nlines, 1, 0), P=P)
    T.tri_sync_status(ctx)
    assert line_relerr(host(dd), ref.reshape(n, nlines), axis=0) <= TOL
