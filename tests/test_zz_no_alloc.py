"""The allocation-free sweep adi_sweep_noalloc (factor tables in the library's
static device scratch) against adi_sweep, through the C ABI: two calls in a
row on one context, the second on a smaller field, each direction; results
bit for bit those of adi_sweep (same kernels, same tables) and within 1e-12
of the oracle's PDD.  A sweep whose tables exceed the scratch is refused
before any launch with the field untouched."""
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


@pytest.mark.parametrize("prec", ["f64", "refine"])
def test_noalloc_sweeps_match_adi_sweep(T, ctx, orc, prec):
    p = T.TRI_F64 if prec == "f64" else T.TRI_F32_REFINE
    for call, (nx, ny, nz) in enumerate([(512, 128, 96), (256, 64, 48)]):     # the second call is smaller
        u0 = W.cfg_field(nx, ny, nz, seed=40 + call)
        coef = [W.momentum_uniform(nx), W.momentum_stretched(ny), W.momentum_periodic(nz)]
        Ps = [8, 4, 4]
        got, want = dev(u0), dev(u0)
        ref = u0.copy()
        for d in range(3):
            a, b, c = (dev(v) for v in coef[d])
            print(f"adi_sweep_noalloc call {call} dir {d} grid {nx}x{ny}x{nz} P={Ps[d]} {prec}", flush=True)
            T.adi_sweep_noalloc(ctx, d, got, a, b, c, Ps[d], periodic=d == 2, method=T.TRI_PDD, prec=p)
            T.adi_sweep(ctx, d, want, a, b, c, Ps[d], periodic=d == 2, method=T.TRI_PDD, prec=p)
            orc.adi_sweep(orc.PDD if prec == "f64" else orc.EXACT_LD, d, ref, *coef[d], Ps[d], d == 2)
        T.tri_sync_status(ctx)
        g = host(got)
        assert np.array_equal(g, host(want))
        assert line_relerr(g, ref, axis=0) <= TOL


def test_noalloc_refuses_tables_beyond_the_scratch(T, ctx):
    n = 16384                                # about 1.4 MB of tables for 1 MiB of scratch
    a, b, c = (dev(v) for v in W.momentum_uniform(n))
    u0 = np.random.default_rng(3).standard_normal((1, 1, n))
    u = dev(u0)
    with pytest.raises(T.TriError) as e:
        T.adi_sweep_noalloc(ctx, 0, u, a, b, c, 8)
    assert e.value.status == T.TRI_E_NOMEM
    T.tri_sync_status(ctx)
    assert np.array_equal(host(u), u0)
