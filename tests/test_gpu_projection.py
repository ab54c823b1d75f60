"""The pressure step around the Poisson solves (Sec. 2.2) on the GPU, through
the C ABI, against the oracle's projection pieces:

* spanwise real FFT / inverse: every supported radix mix (4, 2, 3, 5), all
  three workgroup widths (M <= 144, <= 288, <= 512), line counts that leave
  a ragged last workgroup; per-line relative error <= 1e-12;
* divergence fused into the forward transform, inverse transform fused with
  the spanwise correction, wall-normal correction;
* the whole projection: same result as the oracle, and the corrected
  velocity divergence free to round-off (at the benchmark grid too);
* refusals (odd or unsupported Nz, overlapping arrays) leave data untouched.
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


def cdev(shape):
    return torch.empty(shape, dtype=torch.complex128, device="cuda")


@pytest.mark.parametrize("nz,lines", [(2, 5), (4, 33), (6, 64), (10, 31), (24, 100), (96, 65), (120, 257),
                                      (288, 1000), (200, 37), (576, 300), (640, 129), (1024, 95)])
def test_spanwise_rfft_matches_oracle(T, ctx, nz, lines):
    from oracle import projection
    rng = np.random.default_rng(nz * 7 + lines)
    x = rng.standard_normal((nz, lines))
    dx = dev(x)
    xh = cdev((nz // 2 + 1, lines))
    T.spanwise_rfft(ctx, dx, xh)
    T.tri_sync_status(ctx)
    ref = projection.spanwise_rfft(x)
    assert line_relerr(host(xh), ref, axis=0) <= TOL
    assert torch.equal(dx.cpu(), torch.as_tensor(x))   # input untouched


@pytest.mark.parametrize("nz,lines", [(2, 3), (6, 64), (24, 100), (288, 1000), (200, 37), (576, 300), (1024, 95)])
def test_spanwise_irfft_matches_oracle(T, ctx, nz, lines):
    from oracle import projection
    rng = np.random.default_rng(nz + 11 * lines)
    X = rng.standard_normal((nz // 2 + 1, lines)) + 1j * rng.standard_normal((nz // 2 + 1, lines))
    x = torch.empty((nz, lines), dtype=torch.float64, device="cuda")
    T.spanwise_irfft(ctx, dev(X, torch.complex128), x)
    T.tri_sync_status(ctx)
    ref = projection.spanwise_irfft(X, nz)     # imaginary parts of modes 0 and nz/2 ignored
    assert line_relerr(host(x), ref, axis=0) <= TOL


def test_spanwise_round_trip(T, ctx):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((288, 2049))
    xh = cdev((145, 2049))
    back = torch.empty((288, 2049), dtype=torch.float64, device="cuda")
    T.spanwise_rfft(ctx, dev(x), xh)
    T.spanwise_irfft(ctx, xh, back)
    T.tri_sync_status(ctx)
    assert line_relerr(host(back), x, axis=0) <= 1e-14


def grid(nx, ny, nz, seed):
    rng = np.random.default_rng(seed)
    dy = np.diff(W.tanh_faces(ny))
    dz = 1.0 / nz
    v = rng.standard_normal((nz, ny + 1, nx))
    v[:, 0, :] = 0.0
    v[:, ny, :] = 0.0
    w = rng.standard_normal((nz, ny, nx))
    return dy, dz, v, w


@pytest.mark.parametrize("nx,ny,nz", [(5, 32, 24), (33, 17, 96), (64, 16, 288), (7, 9, 10)])
def test_divergence_rfft_matches_oracle(T, ctx, nx, ny, nz):
    from oracle import projection
    dy, dz, v, w = grid(nx, ny, nz, 1)
    dh = cdev((nz // 2 + 1, ny, nx))
    T.projection_divergence_rfft(ctx, dev(v), dev(w), dev(dy), dz, dh)
    T.tri_sync_status(ctx)
    ref = projection.spanwise_rfft(projection.divergence(v, w, dy, dz))
    assert line_relerr(host(dh), ref, axis=0) <= TOL


@pytest.mark.parametrize("nx,ny,nz", [(5, 32, 24), (33, 17, 96), (64, 16, 288)])
def test_correct_matches_oracle(T, ctx, nx, ny, nz):
    from oracle import projection
    dy, dz, v, w = grid(nx, ny, nz, 2)
    rng = np.random.default_rng(4)
    ph = rng.standard_normal((nz // 2 + 1, ny, nx)) + 1j * rng.standard_normal((nz // 2 + 1, ny, nx))
    dv, dw = dev(v), dev(w)
    phi = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
    T.projection_correct(ctx, dev(ph, torch.complex128), phi, dv, dw, dev(dy), dz)
    T.tri_sync_status(ctx)
    v1, w1, phi1 = projection.correct(ph, v, w, dy, dz)
    assert line_relerr(host(phi), phi1, axis=0) <= TOL
    assert line_relerr(host(dw), w1, axis=0) <= TOL
    got_v = host(dv)
    assert line_relerr(got_v, v1, axis=0) <= TOL
    assert np.all(got_v[:, 0, :] == 0) and np.all(got_v[:, ny, :] == 0)   # walls untouched


@pytest.mark.parametrize("nx,ny,nz,P", [(5, 32, 24, 4), (33, 64, 96, 4), (16, 64, 288, 8)])
def test_projection_step_matches_oracle_and_is_divergence_free(T, ctx, orc, nx, ny, nz, P):
    from oracle import projection
    dy, dz, v, w = grid(nx, ny, nz, 3)
    ay, cy, lam = projection.metric(dy, nz, dz)
    dv, dw = dev(v), dev(w)
    ph = cdev((nz // 2 + 1, ny, nx))
    phi = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
    T.projection_step(ctx, dv, dw, dev(dy), dz, dev(ay), dev(cy), dev(lam), ph, phi, P=P)
    T.tri_sync_status(ctx)
    v1, w1, phi1 = projection.project(v, w, dy, dz, P=P, method=orc.PPT)
    gv, gw = host(dv), host(dw)
    assert line_relerr(host(phi), phi1, axis=0) <= TOL
    assert line_relerr(gv, v1, axis=0) <= TOL
    assert line_relerr(gw, w1, axis=0) <= TOL
    div0 = np.max(np.abs(projection.divergence(v, w, dy, dz)))
    assert np.max(np.abs(projection.divergence(gv, gw, dy, dz))) <= 1e-13 * div0


def test_refusals_touch_nothing(T, ctx):
    L = T.lib()
    x = torch.randn(14 * 8, dtype=torch.float64, device="cuda")
    xh = torch.zeros(2 * 8 * 8, dtype=torch.float64, device="cuda")
    assert L.spanwise_rfft(ctx, x.data_ptr(), xh.data_ptr(), 8, 13) == T.TRI_E_SHAPE        # odd
    assert L.spanwise_rfft(ctx, x.data_ptr(), xh.data_ptr(), 8, 14) == T.TRI_E_UNSUPPORTED  # 7 = prime > 5
    assert L.spanwise_rfft(ctx, x.data_ptr(), xh.data_ptr(), 1, 2048) == T.TRI_E_UNSUPPORTED  # M = 1024 > 512
    assert L.spanwise_rfft(ctx, x.data_ptr(), x.data_ptr() + 64, 4, 12) == T.TRI_E_ARG      # overlap
    assert L.spanwise_irfft(ctx, xh.data_ptr(), xh.data_ptr(), 4, 12) == T.TRI_E_ARG         # in place
    assert L.spanwise_rfft(ctx, x.data_ptr(), xh.data_ptr(), -1, 12) == T.TRI_E_ARG
    assert L.spanwise_rfft(ctx, x.data_ptr(), xh.data_ptr() + 8, 2, 12) == T.TRI_E_ARG      # spectrum not 16-B aligned
    assert L.spanwise_rfft(ctx, x.data_ptr(), xh.data_ptr(), 0, 12) == T.TRI_OK             # nothing to do
    T.tri_sync_status(ctx)
    assert torch.all(xh == 0)


def test_projection_at_benchmark_grid(T, ctx):
    """2048 x 256 x 288: the corrected velocity is divergence free to round-off
    (divergence of the GPU result formed with plain torch ops), and sampled
    stations of the transformed divergence match the oracle."""
    from oracle import projection
    nx, ny, nz = 2048, 256, 288
    dy = np.diff(W.tanh_faces(ny))
    dz = 1.0 / nz
    ay, cy, lam = projection.metric(dy, nz, dz)
    g = torch.Generator(device="cuda").manual_seed(0)
    v = torch.randn((nz, ny + 1, nx), dtype=torch.float64, device="cuda", generator=g)
    v[:, 0, :] = 0.0
    v[:, ny, :] = 0.0
    w = torch.randn((nz, ny, nx), dtype=torch.float64, device="cuda", generator=g)
    ddy = dev(dy)

    def div(vv, ww):
        return (vv[:, 1:, :] - vv[:, :-1, :]) / ddy[None, :, None] + (torch.roll(ww, -1, 0) - ww) / dz

    div0 = div(v, w).abs().max().item()
    ph = cdev((nz // 2 + 1, ny, nx))
    T.projection_divergence_rfft(ctx, v, w, ddy, dz, ph)
    T.tri_sync_status(ctx)
    rng = np.random.default_rng(0)
    js, iss = rng.integers(0, ny, 16), rng.integers(0, nx, 16)
    vs = v[:, :, torch.as_tensor(iss)].cpu().numpy()
    ws = w[:, :, torch.as_tensor(iss)].cpu().numpy()
    got = ph[:, torch.as_tensor(js), torch.as_tensor(iss)].cpu().numpy()
    for s in range(16):
        D = projection.divergence(vs[:, :, s:s + 1], ws[:, :, s:s + 1], dy, dz)[:, js[s], 0]
        ref = projection.spanwise_rfft(D[:, None])[:, 0]
        assert np.max(np.abs(got[:, s] - ref)) <= TOL * np.max(np.abs(ref))
    phi = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
    T.poisson_wavenumber_solve(ctx, ph, dev(ay), dev(cy), dev(lam), P=4)
    T.projection_correct(ctx, ph, phi, v, w, ddy, dz)
    T.tri_sync_status(ctx)
    assert div(v, w).abs().max().item() <= 1e-13 * div0


@pytest.mark.parametrize("width", ["8", "16", "32"])
def test_every_workgroup_width(T, ctx, width, monkeypatch):
    """The transform kernels at each lines-per-workgroup width (TRI_FFT_LINES)."""
    from oracle import projection
    monkeypatch.setenv("TRI_FFT_LINES", width)
    dy, dz, v, w = grid(37, 12, 288, 5)
    dh = cdev((145, 12, 37))
    T.projection_divergence_rfft(ctx, dev(v), dev(w), dev(dy), dz, dh)
    T.tri_sync_status(ctx)
    assert line_relerr(host(dh), projection.spanwise_rfft(projection.divergence(v, w, dy, dz)), axis=0) <= TOL
    ph = host(dh)
    dv, dw = dev(v), dev(w)
    phi = torch.empty((288, 12, 37), dtype=torch.float64, device="cuda")
    T.projection_correct(ctx, dh, phi, dv, dw, dev(dy), dz)
    T.tri_sync_status(ctx)
    v1, w1, phi1 = projection.correct(ph, v, w, dy, dz)
    assert line_relerr(host(phi), phi1, axis=0) <= TOL
    assert line_relerr(host(dw), w1, axis=0) <= TOL
    assert line_relerr(host(dv), v1, axis=0) <= TOL


def lam_x(nx):
    """Modified wavenumbers of the cell-centred Neumann second difference in x (cosine modes)."""
    return (4.0 * nx * nx) * np.sin(np.pi * np.arange(nx) / (2 * nx)) ** 2


@pytest.mark.parametrize("nk,ny,nx,P,method", [(7, 64, 37, 4, "PPT"), (13, 256, 33, 8, "PPT"), (7, 64, 20, 8, "PDD"),
                                               (5, 64, 70, 16, "PPT"), (4, 32, 5, 1, "PPT"),
                                               # partition counts that are not powers of two (the
                                               # reduction's step count and end guards), odd tails
                                               (3, 96, 41, 3, "PPT"), (5, 60, 19, 5, "PPT"), (4, 96, 23, 6, "PDD"),
                                               (6, 112, 17, 7, "PPT"), (3, 64, 9, 2, "PPT")])
def test_shifted_poisson_matches_oracle(T, ctx, orc, nk, ny, nx, P, method):
    """One matrix per (k, i) line, formed on the fly; the (0, 0) line is gauge pinned."""
    ay, cy = W.poisson_metric(ny)
    lamz = W.modified_wavenumbers(2 * (nk - 1))
    lamx = lam_x(nx)
    rng = np.random.default_rng(nk * ny + nx)
    ph = rng.standard_normal((nk, ny, nx)) + 1j * rng.standard_normal((nk, ny, nx))
    d = dev(ph, torch.complex128)
    T.poisson_shifted_solve(ctx, d, dev(ay), dev(cy), dev(lamz), dev(lamx), P=P, method=getattr(T, "TRI_" + method))
    T.tri_sync_status(ctx)
    ref = ph.copy()
    orc.poisson_shifted(ref, ay, cy, lamz, lamx, P, getattr(orc, method))
    got = host(d)
    assert line_relerr(got, ref, axis=1) <= TOL
    assert np.all(got[0, 0, 0] == 0)



def test_shifted_poisson_strict_pdd(T, ctx):
    """With a PDD tolerance set, the shifted solves report TRI_E_PDD_UNSAFE when
    PDD drops O(1) entries (the low modes at 8 rows per partition) and stay
    silent under PPT, which drops nothing."""
    nk, ny, nx, P = 7, 64, 20, 8
    ay, cy = W.poisson_metric(ny)
    args = (dev(ay), dev(cy), dev(W.modified_wavenumbers(2 * (nk - 1))), dev(lam_x(nx)))
    rng = np.random.default_rng(5)
    ph = rng.standard_normal((nk, ny, nx)) + 1j * rng.standard_normal((nk, ny, nx))
    T.tri_sync_status(ctx)
    try:
        T.tri_set_pdd_tolerance(ctx, 1e-12)
        T.poisson_shifted_solve(ctx, dev(ph, torch.complex128), *args, P=P, method=T.TRI_PPT)
        T.tri_sync_status(ctx)
        T.poisson_shifted_solve(ctx, dev(ph, torch.complex128), *args, P=P, method=T.TRI_PDD)
        with pytest.raises(T.TriError) as e:
            T.tri_sync_status(ctx)
        assert e.value.status == T.TRI_E_PDD_UNSAFE
    finally:
        T.tri_set_pdd_tolerance(ctx, 0.0)
    T.poisson_shifted_solve(ctx, dev(ph, torch.complex128), *args, P=P, method=T.TRI_PDD)
    T.tri_sync_status(ctx)

def test_shifted_poisson_refusals(T, ctx):
    L = T.lib()
    ph = torch.zeros((3, 256, 4), dtype=torch.complex128, device="cuda")
    z = torch.zeros(256, dtype=torch.float64, device="cuda")
    args = lambda ny, P, meth: (ctx, ph.data_ptr(), 4, ny, 3, z.data_ptr(), z.data_ptr(), z.data_ptr(), z.data_ptr(),
                                P, meth)
    assert L.poisson_shifted_solve(*args(256, 4, T.TRI_PPT)) == T.TRI_E_UNSUPPORTED   # 64 rows per partition
    assert L.poisson_shifted_solve(*args(256, 6, T.TRI_PPT)) == T.TRI_E_SHAPE         # 256 % 6
    assert L.poisson_shifted_solve(*args(256, 8, 7)) == T.TRI_E_ARG                    # method
    T.tri_sync_status(ctx)
    assert torch.all(ph == 0)


# ---- the 3-D step: cosine transform in x as well ----------------------------

@pytest.mark.parametrize("nx,rows", [(2, 5), (6, 9), (10, 3), (24, 100), (96, 33), (200, 7), (512, 17), (640, 5),
                                     (2048, 13), (4096, 3)])
def test_streamwise_dct_matches_oracle(T, ctx, nx, rows):
    from oracle import projection
    rng = np.random.default_rng(nx + rows)
    x = rng.standard_normal((rows, nx)) + 1j * rng.standard_normal((rows, nx))
    d = dev(x, torch.complex128)
    T.streamwise_dct(ctx, d)
    T.tri_sync_status(ctx)
    ref = projection.streamwise_dct(x)
    assert line_relerr(host(d), ref, axis=1) <= TOL
    T.streamwise_idct(ctx, d)
    T.tri_sync_status(ctx)
    assert line_relerr(host(d), x, axis=1) <= 1e-14
    X = rng.standard_normal((rows, nx)) + 1j * rng.standard_normal((rows, nx))
    d = dev(X, torch.complex128)
    T.streamwise_idct(ctx, d)
    T.tri_sync_status(ctx)
    assert line_relerr(host(d), projection.streamwise_idct(X), axis=1) <= TOL


def grid3(nx, ny, nz, seed):
    dy, dz, v, w = grid(nx, ny, nz, seed)
    rng = np.random.default_rng(seed + 100)
    u = rng.standard_normal((nz, ny, nx + 1))
    u[:, :, 0] = 0.0
    u[:, :, nx] = 0.0
    return 1.0 / nx, dy, dz, u, v, w


@pytest.mark.parametrize("nx,ny,nz", [(6, 32, 24), (34, 17, 96), (64, 16, 288)])
def test_divergence3d_and_correct3d_match_oracle(T, ctx, nx, ny, nz):
    from oracle import projection
    dx, dy, dz, u, v, w = grid3(nx, ny, nz, 7)
    dh = cdev((nz // 2 + 1, ny, nx))
    T.projection3d_divergence_rfft(ctx, dev(u), dev(v), dev(w), dx, dev(dy), dz, dh)
    T.tri_sync_status(ctx)
    ref = projection.spanwise_rfft(projection.divergence3d(u, v, w, dx, dy, dz))
    assert line_relerr(host(dh), ref, axis=0) <= TOL
    rng = np.random.default_rng(8)
    ph = rng.standard_normal((nz // 2 + 1, ny, nx)) + 1j * rng.standard_normal((nz // 2 + 1, ny, nx))
    du, dv, dw = dev(u), dev(v), dev(w)
    phi = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
    T.projection3d_correct(ctx, dev(ph, torch.complex128), phi, du, dv, dw, dx, dev(dy), dz)
    T.tri_sync_status(ctx)
    u1, v1, w1, phi1 = projection.correct3d(ph, u, v, w, dx, dy, dz)
    assert line_relerr(host(phi), phi1, axis=0) <= TOL
    gu = host(du)
    assert line_relerr(gu, u1, axis=2) <= TOL
    assert np.all(gu[:, :, 0] == 0) and np.all(gu[:, :, nx] == 0)
    assert line_relerr(host(dv), v1, axis=0) <= TOL
    assert line_relerr(host(dw), w1, axis=0) <= TOL


@pytest.mark.parametrize("nx,ny,nz,P", [(6, 32, 24, 4), (30, 64, 96, 8), (16, 64, 288, 8)])
def test_projection3d_step_matches_oracle_and_is_divergence_free(T, ctx, orc, nx, ny, nz, P):
    from oracle import projection
    dx, dy, dz, u, v, w = grid3(nx, ny, nz, 9)
    ay, cy, lamz = projection.metric(dy, nz, dz)
    lamx = projection.metric_x(nx, dx)
    du, dv, dw = dev(u), dev(v), dev(w)
    ph = cdev((nz // 2 + 1, ny, nx))
    phi = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
    T.projection3d_step(ctx, du, dv, dw, dx, dev(dy), dz, dev(ay), dev(cy), dev(lamz), dev(lamx), ph, phi, P=P)
    T.tri_sync_status(ctx)
    u1, v1, w1, phi1 = projection.project3d(u, v, w, dx, dy, dz, P=P, method=orc.PPT)
    gu, gv, gw = host(du), host(dv), host(dw)
    assert line_relerr(host(phi), phi1, axis=0) <= TOL
    assert line_relerr(gu, u1, axis=2) <= TOL
    assert line_relerr(gv, v1, axis=0) <= TOL
    assert line_relerr(gw, w1, axis=0) <= TOL
    div0 = np.max(np.abs(projection.divergence3d(u, v, w, dx, dy, dz)))
    assert np.max(np.abs(projection.divergence3d(gu, gv, gw, dx, dy, dz))) <= 1e-13 * div0


def test_dct_refusals_touch_nothing(T, ctx):
    L = T.lib()
    x = torch.zeros(2 * 64, dtype=torch.float64, device="cuda")
    assert L.streamwise_dct(ctx, x.data_ptr(), 13, 2) == T.TRI_E_SHAPE          # odd
    assert L.streamwise_dct(ctx, x.data_ptr(), 14, 2) == T.TRI_E_UNSUPPORTED    # 7 = prime > 5
    assert L.streamwise_idct(ctx, x.data_ptr(), 8192, 0) == T.TRI_E_UNSUPPORTED  # > 4096
    assert L.streamwise_dct(ctx, x.data_ptr() + 8, 4, 2) == T.TRI_E_ARG          # not 16-byte aligned
    assert L.streamwise_dct(ctx, x.data_ptr(), 4, -1) == T.TRI_E_ARG
    T.tri_sync_status(ctx)
    assert torch.all(x == 0)


def test_projection3d_at_benchmark_grid(T, ctx):
    """2048 x 256 x 288 with u on the x-faces: divergence free to round-off after the
    full 3-D step (divergence of the GPU result formed with plain torch ops)."""
    from oracle import projection
    nx, ny, nz = 2048, 256, 288
    dy = np.diff(W.tanh_faces(ny))
    dx, dz = 1.0 / nx, 1.0 / nz
    ay, cy, lamz = projection.metric(dy, nz, dz)
    lamx = projection.metric_x(nx, dx)
    g = torch.Generator(device="cuda").manual_seed(1)
    u = torch.randn((nz, ny, nx + 1), dtype=torch.float64, device="cuda", generator=g)
    u[:, :, 0] = 0.0
    u[:, :, nx] = 0.0
    v = torch.randn((nz, ny + 1, nx), dtype=torch.float64, device="cuda", generator=g)
    v[:, 0, :] = 0.0
    v[:, ny, :] = 0.0
    w = torch.randn((nz, ny, nx), dtype=torch.float64, device="cuda", generator=g)
    ddy = dev(dy)

    def div(uu, vv, ww):
        return ((uu[:, :, 1:] - uu[:, :, :-1]) / dx + ((vv[:, 1:, :] - vv[:, :-1, :]) / ddy[None, :, None]
                + (torch.roll(ww, -1, 0) - ww) / dz))

    div0 = div(u, v, w).abs().max().item()
    ph = cdev((nz // 2 + 1, ny, nx))
    phi = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
    T.projection3d_step(ctx, u, v, w, dx, ddy, dz, dev(ay), dev(cy), dev(lamz), dev(lamx), ph, phi, P=8)
    T.tri_sync_status(ctx)
    assert div(u, v, w).abs().max().item() <= 1e-13 * div0


@pytest.mark.parametrize("rows_per_group", ["1", "2", "8"])
def test_streamwise_dct_every_row_width(T, ctx, rows_per_group, monkeypatch):
    """The cosine transform at each rows-per-workgroup width (TRI_DCT_ROWS)."""
    from oracle import projection
    monkeypatch.setenv("TRI_DCT_ROWS", rows_per_group)
    rng = np.random.default_rng(17)
    for nx in (480, 2048):
        x = rng.standard_normal((7, nx)) + 1j * rng.standard_normal((7, nx))
        d = dev(x, torch.complex128)
        T.streamwise_dct(ctx, d)
        T.tri_sync_status(ctx)
        assert line_relerr(host(d), projection.streamwise_dct(x), axis=1) <= TOL
        T.streamwise_idct(ctx, d)
        T.tri_sync_status(ctx)
        assert line_relerr(host(d), x, axis=1) <= 1e-14


def test_pressure_steps_replay_from_hip_graphs(T, ctx, orc):
    """Both projections allocate nothing and never synchronise, so they record into a
    HIP graph: the 3-D step as one call, the spanwise-only step with its Poisson solve as
    a plan.  Each graph is replayed three times, with eager restores and synchronisations
    between the replays, and every replay is checked against the eager result."""
    from oracle import projection
    nx, ny, nz = 30, 64, 96
    dx, dy, dz, u0, v0, w0 = grid3(nx, ny, nz, 21)
    ay, cy, lamz = projection.metric(dy, nz, dz)
    lamx = projection.metric_x(nx, dx)
    dd = [dev(t) for t in (dy, ay, cy, lamz, lamx)]
    u, v, w = dev(u0), dev(v0), dev(w0)
    ph = cdev((nz // 2 + 1, ny, nx))
    phi = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
    # eager references
    T.projection3d_step(ctx, u, v, w, dx, dd[0], dz, dd[1], dd[2], dd[3], dd[4], ph, phi, P=8)
    T.tri_sync_status(ctx)
    ref3 = [t.clone() for t in (u, v, w, phi)]
    v.copy_(dev(v0)); w.copy_(dev(w0))
    plan = T.tri_plan_create(ctx, [dict(kind=T.TRI_ITEM_POISSON, field=ph, Nx=nx, Ny=ny, Nz=nz // 2 + 1, a=dd[1],
                                        c=dd[2], lam=dd[3], P=4, method=T.TRI_PPT)])
    try:
        def step2():
            T.projection_divergence_rfft(ctx, v, w, dd[0], dz, ph)
            T.tri_plan_execute(plan)
            T.projection_correct(ctx, ph, phi, v, w, dd[0], dz)
        step2()
        T.tri_sync_status(ctx)
        ref2 = [t.clone() for t in (v, w, phi)]
        graphs = []
        side = torch.cuda.Stream()
        for body in (lambda: T.projection3d_step(ctx, u, v, w, dx, dd[0], dz, dd[1], dd[2], dd[3], dd[4], ph, phi,
                                                 P=8), step2):
            g = torch.cuda.CUDAGraph()
            T.tri_set_stream(ctx, side.cuda_stream)
            with torch.cuda.graph(g, stream=side):
                body()
            T.tri_set_stream(ctx, torch.cuda.current_stream().cuda_stream)
            graphs.append(g)
        for rep in range(3):
            for g, ref, tensors in ((graphs[0], ref3, (u, v, w, phi)), (graphs[1], ref2, (v, w, phi))):
                u.copy_(dev(u0)); v.copy_(dev(v0)); w.copy_(dev(w0)); phi.zero_()
                torch.cuda.synchronize()
                g.replay()
                torch.cuda.synchronize()
                for got, want in zip(tensors, ref):
                    assert torch.equal(got, want), rep
        T.tri_sync_status(ctx)
    finally:
        T.tri_set_stream(ctx, torch.cuda.current_stream().cuda_stream)
        T.tri_plan_destroy(plan)


def test_projection_steps_refuse_before_any_launch(T, ctx):
    """Overlapping outputs, a misaligned spectrum or an unsupported shape are refused
    before the first kernel: the velocity is left exactly as it was."""
    from oracle import projection
    nx, ny, nz = 12, 32, 24
    dx, dy, dz, u0, v0, w0 = grid3(nx, ny, nz, 13)
    ay, cy, lamz = projection.metric(dy, nz, dz)
    lamx = projection.metric_x(nx, dx)
    dd = [dev(t) for t in (dy, ay, cy, lamz, lamx)]
    u, v, w = dev(u0), dev(v0), dev(w0)
    ph = cdev((nz // 2 + 1, ny, nx))
    phi = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
    L = T.lib()
    ptr = lambda t: t.data_ptr()

    def step3(phihat_p, phi_p, P=8, Nx=nx):
        return L.projection3d_step(ctx, ptr(u), ptr(v), ptr(w), dx, ptr(dd[0]), dz, ptr(dd[1]), ptr(dd[2]),
                                   ptr(dd[3]), ptr(dd[4]), phihat_p, phi_p, Nx, ny, nz, P)
    assert step3(ptr(ph), ptr(ph)) == T.TRI_E_ARG                 # phi inside phihat
    assert step3(ptr(ph) + 8, ptr(phi)) == T.TRI_E_ARG             # spectrum not 16-byte aligned
    assert step3(ptr(ph), ptr(u)) == T.TRI_E_ARG                   # phi over u
    assert step3(ptr(ph), ptr(phi), P=3) == T.TRI_E_SHAPE          # 32 rows do not split in 3
    assert step3(ptr(ph), ptr(phi), Nx=15) == T.TRI_E_SHAPE         # odd
    assert step3(ptr(ph), ptr(phi), Nx=14) == T.TRI_E_UNSUPPORTED  # 7 is not a supported factor
    assert L.projection_step(ctx, ptr(v), ptr(w), ptr(dd[0]), dz, ptr(dd[1]), ptr(dd[2]), ptr(dd[3]), ptr(ph),
                             ptr(ph), nx, ny, nz, 4) == T.TRI_E_ARG
    T.tri_sync_status(ctx)
    assert torch.equal(u, dev(u0)) and torch.equal(v, dev(v0)) and torch.equal(w, dev(w0))
