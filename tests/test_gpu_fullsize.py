"""Parity at the benchmark's full shapes, in the launch configuration bench.py
times (plans with autotuned launch shapes), on sampled lines the oracle solves
one by one.  Each solve runs on the pristine input.

* ADI sweeps on 2048 x 256 x 288: x (PDD, P=8), y (PDD, P=4), periodic z (PDD, P=16 as
  in the benchmark, and P=4)
* Poisson wavenumber solves 145 x 256 x 2048 complex (PPT, P=4), k = 0 pinned
* independent systems 4096 x 64 (PDD, P=4, one r per line), all lines
* FP32 + FP64 refinement of the x, y, z sweeps and Poisson solves, against the exact solution
* shifted wall-normal solves of the 3-D pressure step, 145 x 256 x 2048 complex (PPT, P=8),
  one matrix per (k, i), the (0, 0) line pinned
"""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_helpers import TOL, dev, line_relerr

pytestmark = pytest.mark.gpu
NX, NY, NZ = 2048, 256, 288
NK = NZ // 2 + 1


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


@pytest.fixture(scope="module")
def field():
    return W.cfg_field(NX, NY, NZ, seed=0)


COEF = {0: lambda: W.momentum_uniform(NX), 1: lambda: W.momentum_stretched(NY), 2: lambda: W.momentum_periodic(NZ)}
PP = {0: 8, 1: 4, 2: 16}


def _sample_lines(u_dev, u0, direction, rng, nsamp):
    if direction == 0:
        j, k = rng.integers(0, NY, nsamp), rng.integers(0, NZ, nsamp)
        return u_dev[torch.as_tensor(k), torch.as_tensor(j), :].cpu().numpy(), u0[k, j, :]
    if direction == 1:
        i, k = rng.integers(0, NX, nsamp), rng.integers(0, NZ, nsamp)
        return u_dev[torch.as_tensor(k), :, torch.as_tensor(i)].cpu().numpy(), u0[k, :, i]
    i, j = rng.integers(0, NX, nsamp), rng.integers(0, NY, nsamp)
    return u_dev[:, torch.as_tensor(j), torch.as_tensor(i)].T.cpu().numpy(), u0[:, j, i].T


@pytest.mark.parametrize("prec", ["f64", "refine"])
@pytest.mark.parametrize("direction,P", [(0, 8), (1, 4), (2, 16), (2, 4)])
def test_fullsize_adi_sweep(T, ctx, orc, field, direction, P, prec):
    a, b, c = COEF[direction]()
    per = direction == 2
    u = dev(field)
    item = dict(kind=direction, field=u, Nx=NX, Ny=NY, Nz=NZ, a=dev(a), b=dev(b), c=dev(c), P=P,
                periodic=int(per), method=T.TRI_PDD)
    if prec == "refine" and P == 16:
        # the refinement kernel takes at most 8 wavefronts of more than 8 rows
        with pytest.raises(T.TriError) as e:
            T.tri_plan_create(ctx, [item], prec=T.TRI_F32_REFINE)
        assert e.value.status == T.TRI_E_UNSUPPORTED
        return
    plan = T.tri_plan_create(ctx, [item], prec=T.TRI_F64 if prec == "f64" else T.TRI_F32_REFINE)
    try:
        T.tri_plan_execute(plan)
        T.tri_sync_status(ctx)
    finally:
        T.tri_plan_destroy(plan)
    rng = np.random.default_rng(100 + direction)
    got, lines = _sample_lines(u, field, direction, rng, 96)
    for s in range(got.shape[0]):
        if prec == "f64":
            ref = orc.pdd(a, b, c, lines[s], P, per)
        else:
            ref = orc.exact_ld(a, b, c, lines[s], per)
        assert line_relerr(got[s], ref, axis=0) <= TOL, s


@pytest.mark.parametrize("prec", ["f64", "refine"])
def test_fullsize_poisson(T, ctx, orc, prec):
    phihat = W.cfg_poisson_rhs(NX, NY, NZ, seed=1)
    ay, cy = W.poisson_metric(NY)
    lam = W.modified_wavenumbers(NZ)
    phi = torch.as_tensor(phihat).cuda()
    item = dict(kind=T.TRI_ITEM_POISSON, field=phi, Nx=NX, Ny=NY, Nz=NK, a=dev(ay), c=dev(cy), lam=dev(lam),
                P=4, method=T.TRI_PPT)
    plan = T.tri_plan_create(ctx, [item], prec=T.TRI_F64 if prec == "f64" else T.TRI_F32_REFINE)
    try:
        T.tri_plan_execute(plan)
        T.tri_sync_status(ctx)
    finally:
        T.tri_plan_destroy(plan)
    rng = np.random.default_rng(7)
    ks = np.concatenate([[0, 1, 2, 3, NK - 1], rng.integers(0, NK, 43)])
    iis = rng.integers(0, NX, ks.size)
    got = phi[torch.as_tensor(ks), :, torch.as_tensor(iis)].cpu().numpy()
    assert np.all(got[0][0] == 0)
    for s, (k, i) in enumerate(zip(ks, iis)):
        b = -(ay + cy) - lam[k]
        c_ = cy.copy()
        rhs = phihat[k, :, i].copy()
        if lam[k] == 0.0:
            b = b.copy(); b[0] = 1.0; c_[0] = 0.0; rhs[0] = 0.0
        solve = (lambda v: orc.ppt(ay, b, c_, v, 4)) if (prec == "f64" or k <= 2) else \
                (lambda v: orc.exact_ld(ay, b, c_, v))
        ref = solve(rhs.real) + 1j * solve(rhs.imag)
        assert line_relerr(got[s], ref, axis=0) <= TOL, (s, k)



def test_fullsize_poisson_shifted(T, ctx, orc):
    phihat = W.cfg_poisson_rhs(NX, NY, NZ, seed=2)
    ay, cy = W.poisson_metric(NY)
    lamz = W.modified_wavenumbers(NZ)
    lamx = (4.0 * NX ** 2) * np.sin(np.pi * np.arange(NX) / (2 * NX)) ** 2
    phi = torch.as_tensor(phihat).cuda()
    T.poisson_shifted_solve(ctx, phi, dev(ay), dev(cy), dev(lamz), dev(lamx), P=8, method=T.TRI_PPT)
    T.tri_sync_status(ctx)
    rng = np.random.default_rng(8)
    ks = np.concatenate([[0, 0, 1, 2, NK - 1], rng.integers(0, NK, 43)])
    iis = np.concatenate([[0, 1, 0, 5, NX - 1], rng.integers(0, NX, 43)])
    got = phi[torch.as_tensor(ks), :, torch.as_tensor(iis)].cpu().numpy()
    assert np.all(got[0][0] == 0)
    for s, (k, i) in enumerate(zip(ks, iis)):
        sigma = lamz[k] + lamx[i]
        b = -(ay + cy) - sigma
        c_ = cy.copy()
        rhs = phihat[k, :, i].copy()
        if sigma == 0.0:
            b[0] = 1.0; c_[0] = 0.0; rhs[0] = 0.0
        ref = orc.ppt(ay, b, c_, rhs.real, 8) + 1j * orc.ppt(ay, b, c_, rhs.imag, 8)
        assert line_relerr(got[s], ref, axis=0) <= TOL, (s, k, i)

def test_fullsize_independent_lines(T, ctx, orc):
    n, nlines, P = 64, 4096, 4
    r, dl = W.cfg_independent(nlines, n, seed=0)
    a, b, c = -r, 1 + 2 * r, -r
    d = np.ascontiguousarray(dl.T)
    ref = d.copy().ravel()
    orc.solve_batch(orc.PDD, ref, n, nlines, 1, s_j=nlines, s_b0=1, s_b1=0, a=a, b=b, c=c,
                    cs_j=0, cs_b0=1, cs_b1=0, P=P)
    dd = dev(d)
    T.tri_pdd_solve(ctx, dev(a), dev(b), dev(c), dd, (n, nlines, 1, nlines, 1, 0), coef_strides=(0, 1, 0), P=P)
    T.tri_sync_status(ctx)
    torch.cuda.synchronize()
    assert line_relerr(dd.cpu().numpy(), ref.reshape(n, nlines), axis=0) <= TOL
