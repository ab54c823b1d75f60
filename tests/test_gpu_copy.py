"""The reference copy (tri_stream_copy): bit-exact for even, odd and tiny
lengths, in place, and the host-side refusals (misaligned, partially
overlapping, negative length) that leave the destination untouched."""
import pytest
import torch

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


@pytest.mark.parametrize("n", [0, 1, 2, 3, 511, 512, 513, 1_000_003])
def test_copy_is_bit_exact(T, ctx, n):
    g = torch.Generator(device="cpu").manual_seed(n)
    src = torch.randn(n + 2, generator=g, dtype=torch.float64).cuda()
    dst = torch.full((n + 2,), -7.0, dtype=torch.float64, device="cuda")
    T.tri_stream_copy(ctx, dst, src, n)
    T.tri_sync_status(ctx)
    assert torch.equal(dst[:n], src[:n])
    assert torch.all(dst[n:] == -7.0)      # nothing past n is written


def test_copy_in_place(T, ctx):
    x = torch.randn(4097, dtype=torch.float64, device="cuda")
    ref = x.clone()
    T.tri_stream_copy(ctx, x, x)
    T.tri_sync_status(ctx)
    assert torch.equal(x, ref)


def test_copy_refusals_touch_nothing(T, ctx):
    src = torch.randn(64, dtype=torch.float64, device="cuda")
    dst = torch.zeros(64, dtype=torch.float64, device="cuda")
    L = T.lib()
    # 8-byte offset: not 16-byte aligned
    assert L.tri_stream_copy(ctx, dst.data_ptr() + 8, src.data_ptr(), 8) == T.TRI_E_ARG
    # destination starts inside the source range
    assert L.tri_stream_copy(ctx, src.data_ptr() + 16, src.data_ptr(), 8) == T.TRI_E_ARG
    assert L.tri_stream_copy(ctx, dst.data_ptr(), src.data_ptr(), -1) == T.TRI_E_ARG
    assert L.tri_stream_copy(ctx, None, src.data_ptr(), 8) == T.TRI_E_ARG
    T.tri_sync_status(ctx)
    assert torch.all(dst == 0)
