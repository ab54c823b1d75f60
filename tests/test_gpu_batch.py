"""Ragged batches through one plan: eight sub-grids of different shapes, each
with an x, y and periodic-z momentum sweep and a Poisson wavenumber solve.

* P = 0: the plan picks each item's partition count by timing, admitting PDD
  only where the reduced-system entries it drops are <= 1e-15 (beyond that
  PDD is not accurate, which is why the paper uses PPT for the Poisson
  systems); the results are compared with the oracle at the P the plan chose.
* Every solve of one dependency level runs in one launch of the level kernel
  (the default for plans of several FP64 items), or, with TRI_BATCH=1, the
  strided solves of one kernel instance share a batched launch; the whole
  step is also replayed as a HIP graph.
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


def test_ragged_plan_fp64_batched_and_graph(T, ctx, orc, monkeypatch):
    """TRI_BATCH=1: strided solves of one kernel instance share a launch."""
    monkeypatch.setenv("TRI_BATCH", "1")
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
    monkeypatch.setenv("TRI_BATCH", "1")
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


def _independent_items(T, grids, Px, Py, Pz, Pp):
    """x, y and z sweeps of each sub-grid on three separate fields and its
    Poisson solve: no item depends on another, so a plan runs them all in one
    dependency level."""
    items, keep = [], []
    for s, g in enumerate(grids):
        nx, ny, nz = g["shape"]
        g["uu"] = [dev(g["u0"]) for _ in range(3)]
        g["phi"] = torch.as_tensor(g["phi0"]).cuda()
        cf = [tuple(dev(v) for v in c) for c in g["coef"]]
        ay, cy = (dev(v) for v in g["metric"])
        lam = dev(g["lam"])
        keep += [cf, ay, cy, lam]
        for d, P in enumerate((Px[s], Py[s], Pz[s])):
            items.append(dict(kind=d, field=g["uu"][d], Nx=nx, Ny=ny, Nz=nz, a=cf[d][0], b=cf[d][1], c=cf[d][2],
                              P=P, periodic=int(d == 2), method=T.TRI_PDD))
        items.append(dict(kind=T.TRI_ITEM_POISSON, field=g["phi"], Nx=nx, Ny=ny, Nz=nz // 2 + 1, a=ay, c=cy,
                          lam=lam, P=Pp[s], method=T.TRI_PPT))
    return items, keep


def test_level_launch_runs_a_ragged_batch_in_one_launch(T, ctx, orc, monkeypatch):
    """TRI_BATCH=2 with every solve independent: the 32 solves of the eight
    sub-grids -- contiguous x sweeps (P up to 16), strided y sweeps (chunked at
    P = 1), periodic z sweeps at partition counts whose wavefronts do not
    divide the 512-lane workgroup (P = 3 in two chunks, 6) or fill it (8),
    Poisson modes by PPT -- run as ONE launch.  The strided solves equal the one-launch-per-solve plan
    bit for bit (the level kernel runs each with its own kernel body); the x
    sweeps, which run the plain contiguous body there, match the oracle."""
    monkeypatch.setenv("TRI_AUTOTUNE", "0")
    Px = [8, 4, 4, 2, 8, 4, 16, 8]
    Py = [2, 4, 1, 8, 2, 4, 8, 2]
    Pz = [4, 8, 3, 6, 2, 3, 4, 6]         # 144 / 4: one 36-row chunk a partition (the 40-row instance)
    Pp = [2, 4, 8, 8, 1, 2, 4, 8]
    grids = _inputs(SMALL, seed=130)
    monkeypatch.setenv("TRI_BATCH", "2")
    items, keep = _independent_items(T, grids, Px, Py, Pz, Pp)
    plan = T.tri_plan_create(ctx, items)
    try:
        descr = [T.tri_plan_item_describe(plan, i) for i in range(len(items))]
        assert all("level=" in d for d in descr), descr
        assert T.tri_plan_launch_count(plan) == 1
        T.tri_plan_execute(plan)
        T.tri_sync_status(ctx)
        level = [([host(u) for u in g["uu"]], host(g["phi"])) for g in grids]
    finally:
        T.tri_plan_destroy(plan)
    for s, g in enumerate(grids):
        a, b, c = g["coef"][0]
        ref = g["u0"].copy()
        orc.adi_sweep(orc.PDD, 0, ref, a, b, c, Px[s], False)
        assert line_relerr(level[s][0][0], ref, axis=2) <= TOL, g["shape"]
    monkeypatch.setenv("TRI_BATCH", "0")
    items, keep2 = _independent_items(T, grids, Px, Py, Pz, Pp)
    plan = T.tri_plan_create(ctx, items)
    try:
        assert T.tri_plan_launch_count(plan) == len(items)
        T.tri_plan_execute(plan)
        T.tri_sync_status(ctx)
        for g, (uu, phi) in zip(grids, level):
            for d in (1, 2):
                assert np.array_equal(host(g["uu"][d]), uu[d]), (g["shape"], d)
            assert np.array_equal(host(g["phi"]), phi), g["shape"]
    finally:
        T.tri_plan_destroy(plan)
    for s, g in enumerate(grids):
        for d, P in ((1, Py[s]), (2, Pz[s])):
            a, b, c = g["coef"][d]
            ref = g["u0"].copy()
            orc.adi_sweep(orc.PDD, d, ref, a, b, c, P, d == 2)
            assert line_relerr(level[s][0][d], ref, axis=2 - d) <= TOL, (g["shape"], d)
        pref = g["phi0"].copy()
        orc.poisson(pref, *g["metric"], g["lam"], P=Pp[s])
        assert line_relerr(level[s][1], pref, axis=1) <= TOL, g["shape"]


@pytest.mark.parametrize("method", ["PDD", "PPT"])
def test_level_launch_two_lines_per_lane(T, ctx, orc, monkeypatch, method):
    """The level kernel's two-lines-per-lane body (periodic z sweeps with
    16-byte lane accesses, PDD and PPT reduced systems) equals that kernel's
    own launch bit for bit."""
    meth = getattr(T, "TRI_" + method)
    monkeypatch.setenv("TRI_AUTOTUNE", "0")
    monkeypatch.setenv("TRI_LPL", "2")
    grids = _inputs(SMALL[:4], seed=150)
    Pz = [4, 8, 6, 2]

    def run(mode):
        monkeypatch.setenv("TRI_BATCH", mode)
        items, keep = [], []
        for s, g in enumerate(grids):
            nx, ny, nz = g["shape"]
            g["u"] = dev(g["u0"])
            a, b, c = (dev(v) for v in g["coef"][2])
            keep += [a, b, c]
            items.append(dict(kind=T.TRI_ITEM_ADI_Z, field=g["u"], Nx=nx, Ny=ny, Nz=nz, a=a, b=b, c=c, P=Pz[s],
                              periodic=1, method=meth))
        plan = T.tri_plan_create(ctx, items)
        try:
            n = T.tri_plan_launch_count(plan)
            T.tri_plan_execute(plan)
            T.tri_sync_status(ctx)
            return n, [host(g["u"]) for g in grids]
        finally:
            T.tri_plan_destroy(plan)

    n2, level = run("2")
    n0, single = run("0")
    assert (n2, n0) == (1, len(grids))
    for s, g in enumerate(grids):
        assert np.array_equal(level[s], single[s]), g["shape"]
        a, b, c = g["coef"][2]
        ref = g["u0"].copy()
        orc.adi_sweep(getattr(orc, method), 2, ref, a, b, c, Pz[s], True)
        assert line_relerr(level[s], ref, axis=0) <= TOL, g["shape"]


def test_ragged_step_level_launches_and_graph(T, ctx, orc, monkeypatch):
    """The default plan of the dependent step (x -> y -> z on one field per
    sub-grid, Poisson alongside), partition counts chosen by the plan: one
    launch per dependency level (three), oracle parity at the chosen P, and
    HIP graph replays equal to the eager run bit for bit."""
    monkeypatch.delenv("TRI_BATCH", raising=False)
    grids = _inputs(SMALL, seed=170)
    items, keep = _items(T, grids)
    plan = T.tri_plan_create(ctx, items)
    try:
        descr = [T.tri_plan_item_describe(plan, i) for i in range(len(items))]
        assert all("level=" in d for d in descr), descr
        assert T.tri_plan_launch_count(plan) == 3
        Ps = [T.tri_plan_item_partitions(plan, i) for i in range(len(items))]
        T.tri_plan_execute(plan)
        T.tri_sync_status(ctx)
        eager = [(host(g["u"]), host(g["phi"])) for g in grids]
        for s, g in enumerate(grids):
            _check_grid(orc, g, Ps[4 * s:4 * s + 4])
        T.tri_plan_capture(plan)
        for rep in range(3):
            for g in grids:
                g["u"].copy_(dev(g["u0"]))
                g["phi"].copy_(torch.as_tensor(g["phi0"]).cuda())
            torch.cuda.synchronize()
            T.tri_plan_graph_launch(plan)
            _ = sum(float(g["u"].sum()) for g in grids)
            for g, (ue, pe) in zip(grids, eager):
                assert np.array_equal(host(g["u"]), ue), (rep, g["shape"])
                assert np.array_equal(host(g["phi"]), pe), (rep, g["shape"])
    finally:
        T.tri_plan_destroy(plan)


@pytest.mark.parametrize("method,periodic", [("PDD", 0), ("PPT", 0), ("PDD", 1), ("PPT", 1)])
def test_level_launch_register_factor_body(T, ctx, orc, monkeypatch, method, periodic):
    """Contiguous x sweeps in the level kernel's register-factor body (4 rows
    per lane, a run of consecutive lines per block), PDD and PPT reduced
    systems, plain and periodic lines: line counts that leave a short last run
    and ghost blocks in the last workgroup.  Equal bit for bit to the
    register-factor kernel's own launch with 4 rows per lane, and to the
    oracle."""
    meth = getattr(T, "TRI_" + method)
    monkeypatch.setenv("TRI_AUTOTUNE", "0")
    shapes = [(1024, 4999, 1, 4), (512, 16411, 1, 4)]    # (Nx, Ny, Nz, P): 256 / 128 lanes a line
    rng = np.random.default_rng(190)
    fields = [rng.standard_normal((nz, ny, nx)) for nx, ny, nz, _ in shapes]
    coefs = [W.momentum_uniform(nx) for nx, _, _, _ in shapes]

    def run(mode, force_c=None):
        monkeypatch.setenv("TRI_BATCH", mode)
        if force_c:
            monkeypatch.setenv("TRI_FORCE_C", force_c)
        else:
            monkeypatch.delenv("TRI_FORCE_C", raising=False)
        us = [dev(f) for f in fields]
        cf = [tuple(dev(v) for v in c) for c in coefs]
        items = [dict(kind=T.TRI_ITEM_ADI_X, field=u, Nx=nx, Ny=ny, Nz=nz, a=c[0], b=c[1], c=c[2], P=P,
                      periodic=periodic, method=meth) for u, c, (nx, ny, nz, P) in zip(us, cf, shapes)]
        plan = T.tri_plan_create(ctx, items)
        try:
            n = T.tri_plan_launch_count(plan)
            T.tri_plan_execute(plan)
            T.tri_sync_status(ctx)
            return n, [host(u) for u in us]
        finally:
            T.tri_plan_destroy(plan)

    n2, level = run("2")
    n0, single = run("0", force_c="104")
    assert (n2, n0) == (1, 2)
    for s, (nx, ny, nz, P) in enumerate(shapes):
        assert np.array_equal(level[s], single[s]), shapes[s]
        a, b, c = coefs[s]
        ref = fields[s].copy()
        orc.adi_sweep(getattr(orc, method), 0, ref, a, b, c, P, bool(periodic))
        assert line_relerr(level[s], ref, axis=2) <= TOL, shapes[s]


def test_level_launch_keeps_solves_whose_lds_does_not_fit_apart(T, ctx, orc, monkeypatch):
    """A contiguous solve whose register-factor blocks would take more than the
    level workgroup's 64 KB of LDS (256 rows at P = 16: eight 64-lane blocks
    with the 16 x 16 reduced-system rows each) keeps a launch of its own; the
    other two share the level launch.  All three match the oracle."""
    monkeypatch.setenv("TRI_AUTOTUNE", "0")
    monkeypatch.delenv("TRI_BATCH", raising=False)
    shapes = [(256, 40, 3, 16), (512, 40, 3, 4), (1024, 24, 5, 8)]
    rng = np.random.default_rng(210)
    fields = [rng.standard_normal((nz, ny, nx)) for nx, ny, nz, _ in shapes]
    coefs = [W.momentum_uniform(nx) for nx, _, _, _ in shapes]
    us = [dev(f) for f in fields]
    cf = [tuple(dev(v) for v in c) for c in coefs]
    items = [dict(kind=T.TRI_ITEM_ADI_X, field=u, Nx=nx, Ny=ny, Nz=nz, a=c[0], b=c[1], c=c[2], P=P, periodic=0,
                  method=T.TRI_PDD) for u, c, (nx, ny, nz, P) in zip(us, cf, shapes)]
    plan = T.tri_plan_create(ctx, items)
    try:
        descr = [T.tri_plan_item_describe(plan, i) for i in range(3)]
        assert "level=" not in descr[0] and all("level=" in d for d in descr[1:]), descr
        assert T.tri_plan_launch_count(plan) == 2
        T.tri_plan_execute(plan)
        T.tri_sync_status(ctx)
    finally:
        T.tri_plan_destroy(plan)
    for s, (nx, ny, nz, P) in enumerate(shapes):
        a, b, c = coefs[s]
        ref = fields[s].copy()
        orc.adi_sweep(orc.PDD, 0, ref, a, b, c, P, False)
        assert line_relerr(host(us[s]), ref, axis=2) <= TOL, shapes[s]


@pytest.mark.parametrize("method,periodic", [("PDD", 1), ("PPT", 0), ("PPT", 1)])
def test_level_launch_plain_contiguous_body(T, ctx, orc, monkeypatch, method, periodic):
    """Contiguous lines whose partitions do not split into 4-row lanes of whole
    wavefronts (128 rows at P = 8 and 4: 32-lane lines) run the level kernel's
    plain contiguous body, many lines a workgroup; PDD and PPT, plain and
    periodic lines, against the oracle."""
    meth = getattr(T, "TRI_" + method)
    monkeypatch.setenv("TRI_AUTOTUNE", "0")
    monkeypatch.delenv("TRI_BATCH", raising=False)
    shapes = [(128, 37, 5, 8), (128, 29, 3, 4)]
    rng = np.random.default_rng(230)
    fields = [rng.standard_normal((nz, ny, nx)) for nx, ny, nz, _ in shapes]
    coefs = [W.momentum_uniform(nx) for nx, _, _, _ in shapes]
    us = [dev(f) for f in fields]
    cf = [tuple(dev(v) for v in c) for c in coefs]
    items = [dict(kind=T.TRI_ITEM_ADI_X, field=u, Nx=nx, Ny=ny, Nz=nz, a=c[0], b=c[1], c=c[2], P=P,
                  periodic=periodic, method=meth) for u, c, (nx, ny, nz, P) in zip(us, cf, shapes)]
    plan = T.tri_plan_create(ctx, items)
    try:
        assert all("level=" in T.tri_plan_item_describe(plan, i) for i in range(2))
        assert T.tri_plan_launch_count(plan) == 1
        T.tri_plan_execute(plan)
        T.tri_sync_status(ctx)
    finally:
        T.tri_plan_destroy(plan)
    for s, (nx, ny, nz, P) in enumerate(shapes):
        a, b, c = coefs[s]
        ref = fields[s].copy()
        orc.adi_sweep(getattr(orc, method), 0, ref, a, b, c, P, bool(periodic))
        assert line_relerr(host(us[s]), ref, axis=2) <= TOL, shapes[s]
