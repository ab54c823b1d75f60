"""Ragged batches through one plan: eight sub-grids of different shapes, each
with an x, y and periodic-z momentum sweep and a Poisson wavenumber solve.

* P = 0: the plan picks each item's partition count by timing, admitting PDD
  only where the reduced-system entries it drops are <= 1e-15 (beyond that
  PDD is not accurate, which is why the paper uses PPT for the Poisson
  systems); the results are compared with the oracle at the P the plan chose.
* Strided solves of one dependency level run as one batched launch; the
  whole step is also replayed as a HIP graph.
* FP32 + refinement plans are compared with the exact solution (x sweeps whose
  shape the contiguous refinement kernel does not take run in FP64).
"""
import numpy as np
import pytest
import torch

import workloads as W
from gpu_helpers import TOL, dev, host, line_relerr

pytestmark = pytest.mark.gpu

# the eight ragged sub-grids of the batched workload, halved in every direction
SMALL = [(nx // 2, ny // 2, nz // 2) for nx, ny, nz in W.RAGGED_SUBGRIDS]


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


def _inputs(shapes, seed=50):
    out = []
    for s, (nx, ny, nz) in enumerate(shapes):
        out.append(dict(
            shape=(nx, ny, nz),
            u0=W.cfg_field(nx, ny, nz, seed=seed + s),
            phi0=W.cfg_poisson_rhs(nx, ny, nz, seed=seed + 100 + s),
            coef=(W.momentum_uniform(nx), W.momentum_stretched(ny), W.momentum_periodic(nz)),
            metric=W.poisson_metric(ny),
            lam=W.modified_wavenumbers(nz)))
    return out


def _items(T, grids, P=0):
    """Per sub-grid x, y, z, Poisson (the plan reorders by dependency)."""
    items, keep = [], []
    for g in grids:
        nx, ny, nz = g["shape"]
        g["u"] = dev(g["u0"])
        g["phi"] = torch.as_tensor(g["phi0"]).cuda()
        cf = [tuple(dev(v) for v in c) for c in g["coef"]]
        ay, cy = (dev(v) for v in g["metric"])
        lam = dev(g["lam"])
        keep += [cf, ay, cy, lam]
        for d in range(3):
            items.append(dict(kind=d, field=g["u"], Nx=nx, Ny=ny, Nz=nz, a=cf[d][0], b=cf[d][1], c=cf[d][2],
                              P=P, periodic=int(d == 2), method=T.TRI_PDD))
        items.append(dict(kind=T.TRI_ITEM_POISSON, field=g["phi"], Nx=nx, Ny=ny, Nz=nz // 2 + 1, a=ay, c=cy,
                          lam=lam, P=P, method=T.TRI_PPT))
    return items, keep


def _oracle(orc, g, Ps, exact_strided=False, exact_x=False):
    ref = g["u0"].copy()
    for d in range(3):
        a, b, c = g["coef"][d]
        if exact_strided and (d > 0 or exact_x):
            orc.adi_sweep(orc.EXACT_LD, d, ref, a, b, c, 1, d == 2)
        else:
            orc.adi_sweep(orc.PDD, d, ref, a, b, c, Ps[d], d == 2)
    pref = g["phi0"].copy()
    if exact_strided:
        ay, cy = g["metric"]
        lam = g["lam"]
        nk, ny, nx = pref.shape
        for k in range(nk):
            b = -(ay + cy) - lam[k]
            c_ = cy.copy()
            rhs = pref[k].copy()
            if lam[k] == 0.0:
                b = b.copy(); b[0] = 1.0; c_[0] = 0.0; rhs[0] = 0.0
            parts = []
            for comp in (rhs.real, rhs.imag):
                v = np.ascontiguousarray(comp).ravel()
                if k <= 2:   # modes k <= 2 stay FP64 PPT in refinement plans
                    orc.solve_batch(orc.PPT, v, ny, nx, 1, nx, 1, 0, ay, b, c_, P=Ps[3])
                else:
                    orc.solve_batch(orc.EXACT_LD, v, ny, nx, 1, nx, 1, 0, ay, b, c_)
                parts.append(v.reshape(ny, nx))
            pref[k] = parts[0] + 1j * parts[1]
    else:
        orc.poisson(pref, *g["metric"], g["lam"], P=Ps[3])
    return ref, pref


def _check_grid(orc, g, Ps, exact_strided=False, exact_x=False):
    ref, pref = _oracle(orc, g, Ps, exact_strided, exact_x)
    got = host(g["u"])
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) <= TOL, g["shape"]
    assert line_relerr(host(g["phi"]), pref, axis=1) <= TOL, g["shape"]


def test_ragged_plan_fp64_batched_and_graph(T, ctx, orc):
    grids = _inputs(SMALL)
    items, keep = _items(T, grids)
    plan = T.tri_plan_create(ctx, items)
    try:
        descr = [T.tri_plan_item_describe(plan, i) for i in range(len(items))]
        assert sum("batch=" in d for d in descr) >= 2, descr       # some strided solves share a launch
        Ps = [T.tri_plan_item_partitions(plan, i) for i in range(len(items))]
        assert all(p in (1, 2, 4, 8, 16) for p in Ps)
        T.tri_plan_execute(plan)
        T.tri_sync_status(ctx)
        eager = [(host(g["u"]), host(g["phi"])) for g in grids]
        for s, g in enumerate(grids):
            _check_grid(orc, g, Ps[4 * s:4 * s + 4])
        T.tri_plan_capture(plan)
        for rep in range(2):
            for g in grids:
                g["u"].copy_(dev(g["u0"]))
                g["phi"].copy_(torch.as_tensor(g["phi0"]).cuda())
            torch.cuda.synchronize()
            T.tri_plan_graph_launch(plan)
            _ = sum(float(g["u"].sum()) for g in grids)      # unrelated eager work between replays
            for g, (ue, pe) in zip(grids, eager):
                assert np.array_equal(host(g["u"]), ue), (rep, g["shape"])
                assert np.array_equal(host(g["phi"]), pe), (rep, g["shape"])
    finally:
        T.tri_plan_destroy(plan)


def test_ragged_plan_batched_matches_unbatched(T, ctx, orc, monkeypatch):
    """A batch only joins solves that run the same kernel instance, so with
    fixed shapes (P = 4, no tuning) the batched plan equals the plan with
    batching switched off bit for bit, and both match the oracle."""
    monkeypatch.setenv("TRI_AUTOTUNE", "0")
    grids = _inputs(SMALL, seed=70)
    items, keep = _items(T, grids, P=4)
    plan = T.tri_plan_create(ctx, items)
    try:
        descr = [T.tri_plan_item_describe(plan, i) for i in range(len(items))]
        assert sum("batch=" in d for d in descr) >= 12, descr
        T.tri_plan_execute(plan)
        T.tri_sync_status(ctx)
        batched = [(host(g["u"]), host(g["phi"])) for g in grids]
    finally:
        T.tri_plan_destroy(plan)
    for s, g in enumerate(grids):
        _check_grid(orc, g, [4, 4, 4, 4])
    monkeypatch.setenv("TRI_BATCH", "0")
    items, keep2 = _items(T, grids, P=4)
    plan = T.tri_plan_create(ctx, items)
    try:
        assert not any("batch=" in T.tri_plan_item_describe(plan, i) for i in range(len(items)))
        T.tri_plan_execute(plan)
        T.tri_sync_status(ctx)
        for g, (ub, pb) in zip(grids, batched):
            assert np.array_equal(host(g["u"]), ub), g["shape"]
            assert np.array_equal(host(g["phi"]), pb), g["shape"]
    finally:
        T.tri_plan_destroy(plan)


def test_ragged_plan_refine(T, ctx, orc):
    grids = _inputs(SMALL, seed=90)
    items, keep = _items(T, grids)
    plan = T.tri_plan_create(ctx, items, prec=T.TRI_F32_REFINE)
    try:
        Ps = [T.tri_plan_item_partitions(plan, i) for i in range(len(items))]
        descr = [T.tri_plan_item_describe(plan, i) for i in range(len(items))]
        assert all("refine" in descr[4 * s + 1] for s in range(len(grids))), descr
        T.tri_plan_execute(plan)
        T.tri_sync_status(ctx)
        assert any("contiguous-refine" in descr[4 * s] for s in range(len(grids))), descr
        for s, g in enumerate(grids):
            _check_grid(orc, g, Ps[4 * s:4 * s + 4], exact_strided=True,
                        exact_x="contiguous-refine" in descr[4 * s])
    finally:
        T.tri_plan_destroy(plan)


def test_partition_choice_respects_pdd_accuracy(T, ctx, orc):
    """Stretched wall-normal momentum lines of 256: PDD's dropped entries grow
    with P (about 1e-16 at P = 4, 1e-11 at P = 8, 1e-4 at P = 16), so the plan
    may only pick a P whose PDD result equals the exact solution to round-off."""
    Nx, Ny, Nz = 300, 256, 5
    u0 = W.cfg_field(Nx, Ny, Nz, seed=12)
    a, b, c = W.momentum_stretched(Ny)
    u = dev(u0)
    plan = T.tri_plan_create(ctx, [dict(kind=T.TRI_ITEM_ADI_Y, field=u, Nx=Nx, Ny=Ny, Nz=Nz, a=dev(a), b=dev(b),
                                        c=dev(c), P=0, periodic=0, method=T.TRI_PDD)])
    try:
        P = T.tri_plan_item_partitions(plan, 0)
        assert P in (1, 2, 4), P
        T.tri_plan_execute(plan)
        T.tri_sync_status(ctx)
    finally:
        T.tri_plan_destroy(plan)
    got = host(u)
    ref = u0.copy()
    orc.adi_sweep(orc.PDD, 1, ref, a, b, c, P, False)
    assert line_relerr(got, ref, axis=1) <= TOL
    exact = u0.copy()
    orc.adi_sweep(orc.EXACT_LD, 1, exact, a, b, c, 1, False)
    assert line_relerr(got, exact, axis=1) <= 1e-13
