"""GPU parity of the FP32-elimination + FP64-refinement path.

The refinement forms the true residual in FP64, so it converges to the exact
A^{-1} d whatever the inner (FP32, partitioned) solver is: the reference is
the oracle's exact solution computed in extended precision (Thomas / cyclic
in long double), at the same 1e-12 per-line bar as the FP64 path.  (An FP64
direct solve can itself sit cond(A) * 1e-16 away from A^{-1} d, which for
the low Poisson modes is close to the bar.)
"""
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


def _exact_sweep(orc, direction, u, a, b, c, periodic):
    ref = u.copy()
    orc.adi_sweep(orc.EXACT_LD, direction, ref, a, b, c, 1, periodic)
    return ref


def _poisson_exact(orc, phihat, ay, cy, lam):
    Nk, Ny, Nx = phihat.shape
    ref = np.empty_like(phihat)
    for k in range(Nk):
        b = -(ay + cy) - lam[k]
        c_ = cy.copy()
        rhs = phihat[k].copy()
        if lam[k] == 0.0:
            b = b.copy(); b[0] = 1.0; c_[0] = 0.0; rhs[0] = 0.0
        re = np.ascontiguousarray(rhs.real); im = np.ascontiguousarray(rhs.imag)
        orc.solve_batch(orc.EXACT_LD, re.ravel(), Ny, Nx, 1, Nx, 1, 0, ay, b, c_)
        orc.solve_batch(orc.EXACT_LD, im.ravel(), Ny, Nx, 1, Nx, 1, 0, ay, b, c_)
        ref[k] = re + 1j * im
    return ref


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("direction,n,P,per,coef", [
    (1, 256, 4, False, "stretched"), (2, 288, 4, True, "periodic"), (1, 64, 4, False, "random"),
    (2, 96, 2, True, "random"), (1, 200, 8, False, "random"),
    (0, 2048, 8, False, "uniform"), (0, 512, 4, False, "random"), (0, 1024, 16, True, "random"),
    (0, 256, 8, False, "random"),
    # sixteen wavefronts of 16-row chunks in one workgroup: P = 16, one chunk a
    # partition; P = 8, two chunks; periodic (dominant rows: with PDD as the
    # inner solver the iteration contracts by about the dropped entries, which
    # at 16 rows a partition of the stretched momentum rows are too large for
    # three refinements; the status says so)
    (1, 256, 16, False, "random"), (1, 256, 8, False, "random"), (2, 256, 16, True, "random")])
def test_refine_sweeps_match_exact(T, ctx, orc, method, direction, n, P, per, coef):
    shape = {0: (5, 7, n), 1: (3, n, 130), 2: (n, 4, 70)}[direction]
    Nz, Ny, Nx = shape
    u = W.cfg_field(Nx, Ny, Nz, seed=21)
    rng = np.random.default_rng(n + P)
    a, b, c = {"stretched": lambda: W.momentum_stretched(n), "periodic": lambda: W.momentum_periodic(n),
               "uniform": lambda: W.momentum_uniform(n),
               "random": lambda: W.random_tridiag(n, rng, margin=1.0, periodic=per)}[coef]()
    ref = _exact_sweep(orc, direction, u, a, b, c, per)
    du = dev(u)
    info = T.adi_sweep(ctx, direction, du, dev(a), dev(b), dev(c), P, periodic=per, method=method,
                       prec=T.TRI_F32_REFINE, info=True)
    T.tri_sync_status(ctx)
    assert line_relerr(host(du), ref, axis=2 - direction) <= TOL
    assert 1 <= info["sweeps"] <= 3
    assert info["resid_max"] <= 1e-13


def test_refine_reaches_exact_not_pdd(T, ctx, orc):
    """With a PDD inner solver whose dropped entries are O(1e-5), the refined
    result is the exact solution, not the PDD approximation."""
    n, P, nlines = 64, 4, 256
    r = 2.0
    a = np.full(n, -r); c = np.full(n, -r); b = np.full(n, 1 + 2 * r)
    a[0] = c[-1] = 0
    rng = np.random.default_rng(3)
    D = rng.uniform(-1, 1, (n, nlines))
    exact = D.copy().ravel()
    orc.solve_batch(orc.EXACT_LD, exact, n, nlines, 1, nlines, 1, 0, a, b, c)
    exact = exact.reshape(n, nlines)
    pdd = D.copy().ravel()
    orc.solve_batch(orc.PDD, pdd, n, nlines, 1, nlines, 1, 0, a, b, c, P=P)
    assert line_relerr(pdd.reshape(n, nlines), exact, axis=0) > 1e-6
    dd = dev(D)
    T.tri_pdd_solve(ctx, dev(a), dev(b), dev(c), dd, (n, nlines, 1, nlines, 1, 0), P=P, prec=T.TRI_F32_REFINE)
    T.tri_sync_status(ctx)
    assert line_relerr(host(dd), exact, axis=0) <= TOL


@pytest.mark.parametrize("Nx,Ny,Nz", [(70, 64, 48), (130, 256, 24)])
def test_refine_poisson_low_modes_fp64(T, ctx, orc, Nx, Ny, Nz):
    phihat = W.cfg_poisson_rhs(Nx, Ny, Nz, seed=4)
    ay, cy = W.poisson_metric(Ny)
    lam = W.modified_wavenumbers(Nz)
    ref = _poisson_exact(orc, phihat, ay, cy, lam)
    dphi = torch.as_tensor(phihat).cuda()
    info = T.poisson_wavenumber_solve(ctx, dphi, dev(ay), dev(cy), dev(lam), P=4, prec=T.TRI_F32_REFINE,
                                      fp64_kmax=2, info=True)
    T.tri_sync_status(ctx)
    got = host(dphi)
    assert line_relerr(got, ref, axis=1) <= TOL
    assert info["sweeps"] >= 1
    assert info["resid_max"] <= 1e-13


def test_refine_reports_non_convergence(T, ctx, orc):
    """A well-conditioned matrix scaled to 1e-40: fine in FP64, but its pivot
    reciprocals overflow FP32, so the FP32 inner solves cannot contract and the
    device status must report non-convergence (forced by the data; every
    kernel still exits normally).  The FP64 path solves the same system."""
    n, P, nlines = 64, 4, 128
    s = 1e-40
    a = np.full(n, -0.25 * s); c = np.full(n, -0.25 * s); b = np.full(n, s)
    a[0] = c[-1] = 0.0
    rng = np.random.default_rng(6)
    D = rng.uniform(-1, 1, (n, nlines))
    dd = dev(D)
    T.tri_ppt_solve(ctx, dev(a), dev(b), dev(c), dd, (n, nlines, 1, nlines, 1, 0), P=P, prec=T.TRI_F32_REFINE)
    with pytest.raises(T.TriError) as e:
        T.tri_sync_status(ctx)
    assert e.value.status == T.TRI_E_NOT_CONVERGED
    T.tri_sync_status(ctx)
    dd = dev(D)
    T.tri_ppt_solve(ctx, dev(a), dev(b), dev(c), dd, (n, nlines, 1, nlines, 1, 0), P=P)
    T.tri_sync_status(ctx)
    ref = D.copy().ravel()
    orc.solve_batch(orc.PPT, ref, n, nlines, 1, nlines, 1, 0, a, b, c, P=P)
    assert line_relerr(host(dd), ref.reshape(n, nlines), axis=0) <= TOL


@pytest.mark.parametrize("direction,method", [(1, 0), (2, 1), (0, 0)])
def test_refine_any_magnitude(T, ctx, orc, direction, method):
    """Each line's right-hand side is scaled by a power of two before the FP32
    solve, so lines whose values lie far outside FP32's range (here 1e-250 to
    1e250, a different magnitude on every line) still reach the exact solution."""
    n = {0: 2048, 1: 256, 2: 288}[direction]
    shape = {0: (5, 7, n), 1: (3, n, 130), 2: (n, 4, 70)}[direction]
    Nz, Ny, Nx = shape
    rng = np.random.default_rng(17)
    u = W.cfg_field(Nx, Ny, Nz, seed=17)
    mag = 10.0 ** rng.uniform(-250, 250, size={0: (Nz, Ny), 1: (Nz, Nx), 2: (Ny, Nx)}[direction])
    u = u * {0: mag[:, :, None], 1: mag[:, None, :], 2: mag[None]}[direction]
    a, b, c = {0: W.momentum_uniform, 1: W.momentum_stretched, 2: W.momentum_periodic}[direction](n)
    ref = _exact_sweep(orc, direction, u, a, b, c, direction == 2)
    du = dev(u)
    T.adi_sweep(ctx, direction, du, dev(a), dev(b), dev(c), {0: 8, 1: 4, 2: 4}[direction], periodic=direction == 2,
                method=method, prec=T.TRI_F32_REFINE)
    T.tri_sync_status(ctx)
    assert line_relerr(host(du), ref, axis=2 - direction) <= TOL


def test_refine_poisson_large_values(T, ctx, orc):
    Nx, Ny, Nz = 70, 64, 48
    phihat = W.cfg_poisson_rhs(Nx, Ny, Nz, seed=19) * 1e200
    ay, cy = W.poisson_metric(Ny)
    lam = W.modified_wavenumbers(Nz)
    ref = _poisson_exact(orc, phihat, ay, cy, lam)
    dphi = torch.as_tensor(phihat).cuda()
    T.poisson_wavenumber_solve(ctx, dphi, dev(ay), dev(cy), dev(lam), P=4, prec=T.TRI_F32_REFINE, fp64_kmax=2)
    T.tri_sync_status(ctx)
    assert line_relerr(host(dphi), ref, axis=1) <= TOL


def _cfg1(seed, rmax=None):
    n, nlines = 64, 4096
    r, dl = W.cfg_independent(nlines, n, seed=seed)
    if rmax is not None:
        r = 0.1 + (r - 0.1) * (rmax - 0.1) / 9.9
    d = np.ascontiguousarray(dl.T)                       # [j][line]
    return n, nlines, r, d


def _cfg1_exact(orc, n, nlines, r, d):
    ref = d.copy().ravel()
    orc.solve_batch(orc.EXACT_LD, ref, n, nlines, 1, nlines, 1, 0, -r, 1 + 2 * r, -r, cs_j=0, cs_b0=1, cs_b1=0)
    return ref.reshape(n, nlines)


def test_refine_independent_lines_ppt(T, ctx, orc):
    """Independent systems with their own coefficients (4096 x 64, r ~ U[0.1, 10],
    P = 4): FP32 blocks + FP64 refinement with the PPT inner solver reach the
    exact solution."""
    n, nlines, r, d = _cfg1(0)
    ref = _cfg1_exact(orc, n, nlines, r, d)
    dd = dev(d)
    info = T.tri_ppt_solve(ctx, dev(-r), dev(1 + 2 * r), dev(-r), dd, (n, nlines, 1, nlines, 1, 0),
                           coef_strides=(0, 1, 0), P=4, prec=T.TRI_F32_REFINE, info=True)
    T.tri_sync_status(ctx)
    assert line_relerr(host(dd), ref, axis=0) <= TOL
    assert 1 <= info["sweeps"] <= 3


def test_refine_independent_lines_pdd_inner(T, ctx, orc):
    """With the PDD inner solver the refinement converges to the exact solution
    where PDD's dropped entries are small (r <= 1: below 5e-8); on the full
    r range (dropped entries up to 3e-3) three refinements cannot reach the
    tolerance and the status says so."""
    n, nlines, r, d = _cfg1(1, rmax=1.0)
    ref = _cfg1_exact(orc, n, nlines, r, d)
    dd = dev(d)
    T.tri_pdd_solve(ctx, dev(-r), dev(1 + 2 * r), dev(-r), dd, (n, nlines, 1, nlines, 1, 0),
                    coef_strides=(0, 1, 0), P=4, prec=T.TRI_F32_REFINE)
    T.tri_sync_status(ctx)
    assert line_relerr(host(dd), ref, axis=0) <= TOL
    n, nlines, r, d = _cfg1(0)
    dd = dev(d)
    T.tri_pdd_solve(ctx, dev(-r), dev(1 + 2 * r), dev(-r), dd, (n, nlines, 1, nlines, 1, 0),
                    coef_strides=(0, 1, 0), P=4, prec=T.TRI_F32_REFINE)
    with pytest.raises(T.TriError) as e:
        T.tri_sync_status(ctx)
    assert e.value.status == T.TRI_E_NOT_CONVERGED


@pytest.mark.parametrize("periodic", [False, True])
@pytest.mark.parametrize("n,P", [(48, 4), (16, 2), (96, 8)])
def test_refine_general_per_element(T, ctx, orc, periodic, n, P):
    """Fully general rows (a, b, c per element), PPT inner solver.  Per-line
    periodic PPT takes P <= 4: at P = 8 the call is refused before any launch
    and the data is left as it was."""
    nlines = 130
    rng = np.random.default_rng(41 + n)
    A = np.empty((nlines, n)); B = np.empty((nlines, n)); C = np.empty((nlines, n))
    for s in range(nlines):
        A[s], B[s], C[s] = W.random_tridiag(n, rng, margin=0.5, periodic=periodic)
    D = rng.uniform(-1, 1, (n, nlines))
    At, Bt, Ct = (np.ascontiguousarray(X.T) for X in (A, B, C))
    ref = D.copy().ravel()
    orc.solve_batch(orc.EXACT_LD, ref, n, nlines, 1, s_j=nlines, s_b0=1, s_b1=0,
                    a=At.ravel(), b=Bt.ravel(), c=Ct.ravel(), cs_j=nlines, cs_b0=1, cs_b1=0, periodic=periodic)
    dd = dev(D)
    if periodic and P > 4:
        with pytest.raises(T.TriError) as e:
            T.tri_ppt_solve(ctx, dev(At), dev(Bt), dev(Ct), dd, (n, nlines, 1, nlines, 1, 0),
                            coef_strides=(nlines, 1, 0), P=P, periodic=periodic, prec=T.TRI_F32_REFINE)
        assert e.value.status == T.TRI_E_UNSUPPORTED
        T.tri_sync_status(ctx)
        assert np.array_equal(host(dd), D)
        return
    T.tri_ppt_solve(ctx, dev(At), dev(Bt), dev(Ct), dd, (n, nlines, 1, nlines, 1, 0), coef_strides=(nlines, 1, 0),
                    P=P, periodic=periodic, prec=T.TRI_F32_REFINE)
    T.tri_sync_status(ctx)
    assert line_relerr(host(dd), ref.reshape(n, nlines), axis=0) <= TOL


@pytest.mark.parametrize("kc", [2, 4, 8])
def test_refine_chunk_counts(T, ctx, orc, monkeypatch, kc):
    monkeypatch.setenv("TRI_FORCE_KC", str(kc))
    n, P = 128, 2
    Nz, Nx = 3, 100
    u = W.cfg_field(Nx, n, Nz, seed=kc)
    a, b, c = W.momentum_stretched(n)
    ref = _exact_sweep(orc, 1, u, a, b, c, False)
    du = dev(u)
    T.adi_sweep(ctx, 1, du, dev(a), dev(b), dev(c), P, method=1, prec=T.TRI_F32_REFINE)
    T.tri_sync_status(ctx)
    assert line_relerr(host(du), ref, axis=1) <= TOL


def test_refine_plan_and_graph(T, ctx, orc):
    Nz, Ny, Nx = 24, 64, 128
    u0 = W.cfg_field(Nx, Ny, Nz, seed=8)
    phi0 = W.cfg_poisson_rhs(Nx, Ny, Nz, seed=8)
    cyc, czc = W.momentum_stretched(Ny), W.momentum_periodic(Nz)
    ay, cy = W.poisson_metric(Ny)
    lam = W.modified_wavenumbers(Nz)
    u = dev(u0)
    phi = torch.as_tensor(phi0).cuda()
    gy = [dev(v) for v in cyc]
    gz = [dev(v) for v in czc]
    items = [dict(kind=T.TRI_ITEM_ADI_Y, field=u, Nx=Nx, Ny=Ny, Nz=Nz, a=gy[0], b=gy[1], c=gy[2], P=4, method=0),
             dict(kind=T.TRI_ITEM_ADI_Z, field=u, Nx=Nx, Ny=Ny, Nz=Nz, a=gz[0], b=gz[1], c=gz[2], P=4, periodic=1,
                  method=0),
             dict(kind=T.TRI_ITEM_POISSON, field=phi, Nx=Nx, Ny=Ny, Nz=Nz // 2 + 1, a=dev(ay), c=dev(cy),
                  lam=dev(lam), P=4, method=1)]
    plan = T.tri_plan_create(ctx, items, prec=T.TRI_F32_REFINE)
    try:
        ref = u0.copy()
        orc.adi_sweep(orc.EXACT_LD, 1, ref, *cyc, 1, False)
        orc.adi_sweep(orc.EXACT_LD, 2, ref, *czc, 1, True)
        pref = _poisson_exact(orc, phi0, ay, cy, lam)
        T.tri_plan_capture(plan)
        for rep in range(3):
            u.copy_(dev(u0)); phi.copy_(torch.as_tensor(phi0).cuda())
            torch.cuda.synchronize()
            T.tri_plan_graph_launch(plan)
            assert np.max(np.abs(host(u) - ref)) / np.max(np.abs(ref)) <= TOL, rep
            assert line_relerr(host(phi), pref, axis=1) <= TOL, rep
        T.tri_sync_status(ctx)
    finally:
        T.tri_plan_destroy(plan)
