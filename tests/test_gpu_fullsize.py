"""Parity at the benchmark's full shapes, in the launch configuration bench.py
times (plans with autotuned launch shapes), on EVERY line: the oracle solves
the whole field (C, OpenMP over lines) and each line is held to 1e-12
relative error.  Each solve runs on the pristine input.

* ADI sweeps on 2048 x 256 x 288: x (PDD, P=8), y (PDD, P=4 as in the benchmark, and P=8),
  periodic z (PDD, P=16 as in the benchmark, P=4 and P=8), against the oracle's PDD at the same P
* Poisson wavenumber solves 145 x 256 x 2048 complex (PPT, P=4), k = 0 pinned
* independent systems 4096 x 64 (PDD, P=4, one r per line)
* FP32 + FP64 refinement of the x, y, z sweeps (y and z at P=8 as the benchmark times them)
  and Poisson solves, against the
  extended-precision exact solution (Poisson modes k <= 2 stay FP64: the oracle's PPT)
* shifted wall-normal solves of the 3-D pressure step, 145 x 256 x 2048 complex (PPT, P=8),
  one matrix per (k, i), the (0, 0) line pinned
* the ragged eight-sub-grid step in one launch per dependency level (x -> y -> z composed, Poisson)
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


def _every_line(got, ref, axis, what):
    """Assert every line's relative error <= 1e-12; print the worst."""
    err = line_relerr(got, ref, axis=axis)
    print(f"{what}: worst line relative error {err:.2e} over {got.size // got.shape[axis]} lines", flush=True)
    assert err <= TOL, (what, err)


@pytest.mark.parametrize("prec", ["f64", "refine"])
@pytest.mark.parametrize("direction,P", [(0, 8), (1, 4), (1, 8), (2, 16), (2, 4), (2, 8)])
def test_fullsize_adi_sweep(T, ctx, orc, field, direction, P, prec):
    a, b, c = COEF[direction]()
    per = direction == 2
    u = dev(field)
    item = dict(kind=direction, field=u, Nx=NX, Ny=NY, Nz=NZ, a=dev(a), b=dev(b), c=dev(c), P=P,
                periodic=int(per), method=T.TRI_PDD)
    if prec == "refine" and P == 16:
        # the refinement kernel takes at most 8 wavefronts of more than 16 rows
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
    got = u.cpu().numpy()
    ref = field.copy()
    orc.adi_sweep(orc.PDD if prec == "f64" else orc.EXACT_LD, direction, ref, a, b, c, P, per)
    _every_line(got, ref, 2 - direction, f"adi dir {direction} P={P} {prec}")


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
    got = phi.cpu().numpy()
    assert np.all(got[0, 0, :] == 0)
    ref = phihat.copy()
    orc.poisson(ref, ay, cy, lam, P=4)
    if prec == "refine":                    # modes k > 2 run FP32 + refinement: the exact solution
        ref_ld = phihat.copy()
        orc.poisson(ref_ld, ay, cy, lam, P=4, method=orc.EXACT_LD)
        ref[3:] = ref_ld[3:]
    _every_line(got, ref, 1, f"poisson {prec}")


def test_fullsize_poisson_shifted(T, ctx, orc):
    phihat = W.cfg_poisson_rhs(NX, NY, NZ, seed=2)
    ay, cy = W.poisson_metric(NY)
    lamz = W.modified_wavenumbers(NZ)
    lamx = (4.0 * NX ** 2) * np.sin(np.pi * np.arange(NX) / (2 * NX)) ** 2
    phi = torch.as_tensor(phihat).cuda()
    T.poisson_shifted_solve(ctx, phi, dev(ay), dev(cy), dev(lamz), dev(lamx), P=8, method=T.TRI_PPT)
    T.tri_sync_status(ctx)
    got = phi.cpu().numpy()
    assert np.all(got[0, 0, 0] == 0)
    ref = phihat.copy()
    orc.poisson_shifted_batch(ref, ay, cy, lamz, lamx, 8)
    _every_line(got, ref, 1, "shifted poisson P=8")


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


def test_fullsize_ragged_step_level_launches(T, ctx, orc, monkeypatch):
    """The ragged eight-sub-grid step at its full shapes in bench.py's
    configuration: one plan (partition counts from the shipped tuning table),
    every solve of a dependency level in one launch (three launches), each
    sub-grid's composed x -> y -> z sweep and Poisson solves against the
    oracle at the chosen partition counts, every line."""
    monkeypatch.delenv("TRI_BATCH", raising=False)
    grids, items, keep = [], [], []
    for s, (nx, ny, nz) in enumerate(W.RAGGED_SUBGRIDS):
        g = dict(shape=(nx, ny, nz), u0=W.cfg_field(nx, ny, nz, seed=200 + s),
                 phi0=W.cfg_poisson_rhs(nx, ny, nz, seed=300 + s),
                 coef=(W.momentum_uniform(nx), W.momentum_stretched(ny), W.momentum_periodic(nz)),
                 metric=W.poisson_metric(ny), lam=W.modified_wavenumbers(nz))
        g["u"], g["phi"] = dev(g["u0"]), torch.as_tensor(g["phi0"]).cuda()
        cf = [tuple(dev(v) for v in c) for c in g["coef"]]
        ay, cy = (dev(v) for v in g["metric"])
        lam = dev(g["lam"])
        keep += [cf, ay, cy, lam]
        for d in range(3):
            items.append(dict(kind=d, field=g["u"], Nx=nx, Ny=ny, Nz=nz, a=cf[d][0], b=cf[d][1], c=cf[d][2], P=0,
                              periodic=int(d == 2), method=T.TRI_PDD))
        items.append(dict(kind=T.TRI_ITEM_POISSON, field=g["phi"], Nx=nx, Ny=ny, Nz=nz // 2 + 1, a=ay, c=cy,
                          lam=lam, P=0, method=T.TRI_PPT))
        grids.append(g)
    plan = T.tri_plan_create(ctx, items)
    try:
        assert T.tri_plan_launch_count(plan) == 3
        Ps = [T.tri_plan_item_partitions(plan, i) for i in range(len(items))]
        print(f"ragged level plan P = {Ps}", flush=True)
        T.tri_plan_execute(plan)
        T.tri_sync_status(ctx)
    finally:
        T.tri_plan_destroy(plan)
    for s, g in enumerate(grids):
        ref = g["u0"].copy()
        for d in range(3):
            orc.adi_sweep(orc.PDD, d, ref, *g["coef"][d], Ps[4 * s + d], d == 2)
        _every_line(g["u"].cpu().numpy(), ref, 0, f"ragged {g['shape']} x->y->z")
        pref = g["phi0"].copy()
        orc.poisson(pref, *g["metric"], g["lam"], P=Ps[4 * s + 3])
        _every_line(g["phi"].cpu().numpy(), pref, 1, f"ragged {g['shape']} poisson")
        del g["u"], g["phi"]
