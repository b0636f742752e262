"""The streaming reference kernel (adi_stream_ceiling) computes what it
states, x = a - c b and y = b - a, over every element, and refuses
misaligned or odd-sized arrays."""
import torch

import pytest

from paper_2006_07583_amd import adi

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("n", [4, 1000, 4097 * 4097 + 3])
def test_stream_kernel_values(dtype, n):
    esz = torch.tensor([], dtype=dtype).element_size()
    n = n // (16 // esz) * (16 // esz)
    g = torch.Generator(device="cpu").manual_seed(n)
    a, b, c = (torch.rand(n, generator=g, dtype=dtype).to("cuda:0") for _ in range(3))
    x, y = torch.full_like(a, 7.0), torch.full_like(a, 7.0)
    adi.stream_ceiling(a, b, c, x, y)
    torch.cuda.synchronize()
    assert torch.allclose(x, a - c * b, rtol=0, atol=4 * torch.finfo(dtype).eps)
    assert torch.equal(y, b - a)


def test_stream_kernel_refusals():
    a = torch.zeros(8, dtype=torch.float32, device="cuda:0")
    with pytest.raises(adi.AdiError, match="16-byte aligned"):
        adi.stream_ceiling(*[t[1:5] for t in (a, a.clone(), a.clone(), a.clone(), a.clone())])
    with pytest.raises(adi.AdiError, match="multiple of 16"):
        adi.stream_ceiling(*[t[:6] for t in (a, a.clone(), a.clone(), a.clone(), a.clone())])
