"""The HBM streaming reference kernels (include/tlb_stream.h) compute what they state: copy and
add bit for bit against torch, the read mode's partial sums against an FP64 sum."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n16", [1, 1000, 262144 + 37, 3 * 2048 * 256 * 4 + 5])
def test_stream_kernels(torch_cuda, n16):
    torch = torch_cuda
    from paper_1904_10070_amd.binding import hbm_stream, STREAM_COPY, STREAM_ADD, STREAM_READ
    g = torch.Generator(device="cuda").manual_seed(n16)
    x = torch.rand(4 * n16, device="cuda", generator=g)
    y = torch.rand(4 * n16, device="cuda", generator=g)
    z = torch.empty_like(x)
    assert hbm_stream(STREAM_COPY, x, None, z) == 32 * n16
    torch.cuda.synchronize()
    assert torch.equal(z, x)
    assert hbm_stream(STREAM_ADD, x, y, z) == 48 * n16
    torch.cuda.synchronize()
    assert torch.equal(z, x + y)
    parts = torch.zeros(4 * 8192, device="cuda")
    assert hbm_stream(STREAM_READ, x, None, parts) == 16 * n16
    torch.cuda.synchronize()
    total = parts.double().sum().item()
    want = x.double().sum().item()
    assert abs(total - want) <= 1e-5 * want + 1e-6
