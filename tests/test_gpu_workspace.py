"""One-shot solves allocate nothing and never wait: the context workspace is
sized by tri_create (and tri_reserve), so

* the first one-shot calls on a fresh context record into a HIP graph, and
  three replays (with eager restores and synchronisations between them)
  reproduce the eager result bit for bit;
* a call whose factor tables do not fit the workspace is refused with
  TRI_E_NOMEM before any launch (the data is left exactly as it was), and
  runs after tri_reserve, matching the oracle.
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


def test_first_one_shot_calls_record_into_a_graph(T, orc):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    Nx, Ny, Nz = 96, 64, 48
    u0 = W.cfg_field(Nx, Ny, Nz, seed=7)
    phi0 = W.cfg_poisson_rhs(Nx, Ny, Nz, seed=8)
    coef = [W.momentum_uniform(Nx), W.momentum_stretched(Ny), W.momentum_periodic(Nz)]
    dcoef = [tuple(dev(v) for v in c) for c in coef]
    ay, cy = W.poisson_metric(Ny)
    lam = W.modified_wavenumbers(Nz)
    day, dcy, dlam = dev(ay), dev(cy), dev(lam)
    Ps = [8, 4, 4]
    u, phi = dev(u0), torch.as_tensor(phi0).cuda()

    side = torch.cuda.Stream()
    ctx = T.tri_create(0, side.cuda_stream)        # fresh: nothing solved on it yet
    try:
        def step():
            for d in range(3):
                T.adi_sweep(ctx, d, u, *dcoef[d], Ps[d], periodic=d == 2, method=T.TRI_PDD)
            T.poisson_wavenumber_solve(ctx, phi, day, dcy, dlam, P=4)

        g = torch.cuda.CUDAGraph()
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=side):
            step()
        # eager reference on the same context, after the capture
        u.copy_(dev(u0)); phi.copy_(torch.as_tensor(phi0).cuda())
        torch.cuda.synchronize()
        step()
        T.tri_sync_status(ctx)
        ref_u, ref_phi = u.clone(), phi.clone()
        want_u = u0.copy()
        for d in range(3):
            orc.adi_sweep(orc.PDD, d, want_u, *coef[d], Ps[d], d == 2)
        want_phi = phi0.copy()
        orc.poisson(want_phi, ay, cy, lam, P=4)
        assert np.max(np.abs(host(ref_u) - want_u)) / np.max(np.abs(want_u)) <= TOL
        assert line_relerr(host(ref_phi), want_phi, axis=1) <= TOL
        for rep in range(3):
            u.copy_(dev(u0)); phi.copy_(torch.as_tensor(phi0).cuda())
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(u, ref_u), rep
            assert torch.equal(phi, ref_phi), rep
        T.tri_sync_status(ctx)
    finally:
        torch.cuda.synchronize()
        T.tri_destroy(ctx)


def test_short_workspace_is_refused_then_reserved(T, orc):
    """4096 Poisson matrices of 256 rows need ~90 MB of factor tables, more than the
    64 MiB a context starts with."""
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    Nx, Ny, Nk, P = 2, 256, 4096, 4
    lam = W.modified_wavenumbers(2 * (Nk - 1))
    assert lam.size == Nk
    ay, cy = W.poisson_metric(Ny)
    rng = np.random.default_rng(11)
    phi0 = rng.standard_normal((Nk, Ny, Nx)) + 1j * rng.standard_normal((Nk, Ny, Nx))
    ctx = T.tri_create(0, torch.cuda.current_stream().cuda_stream)
    try:
        phi = torch.as_tensor(phi0).cuda()
        day, dcy, dlam = dev(ay), dev(cy), dev(lam)
        L = T.lib()
        st = L.poisson_wavenumber_solve(ctx, phi.data_ptr(), Nx, Ny, Nk, day.data_ptr(), dcy.data_ptr(),
                                        dlam.data_ptr(), P, T.TRI_F64, -1, None)
        assert st == T.TRI_E_NOMEM, st
        assert "tri_reserve" in T.tri_last_error(ctx)
        T.tri_sync_status(ctx)
        assert torch.equal(phi, torch.as_tensor(phi0).cuda())
        T.tri_reserve(ctx, Ny, P, Nk)
        T.poisson_wavenumber_solve(ctx, phi, day, dcy, dlam, P=P)
        T.tri_sync_status(ctx)
        want = phi0.copy()
        orc.poisson(want, ay, cy, lam, P=P)
        assert line_relerr(host(phi), want, axis=1) <= TOL
        with pytest.raises(T.TriError):
            T.tri_reserve(ctx, 0, P, 1)
    finally:
        T.tri_destroy(ctx)
