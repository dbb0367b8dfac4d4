"""fd_stream_probe computes what it states, through the C ABI: kind 0
copies a into out, kind 1 rewrites out as a + b * out, element by element,
over lengths that fill whole blocks, end in a ragged block, are one float4
long, or are empty (nothing launched, out untouched).  The inputs are
multiples of 1/16 below 2^10 in magnitude, so a + b * out is exact in FP32
whichever way it is evaluated and the comparison is bit for bit."""
import pytest
import torch

from paper_2311_05038_amd import _abi

pytestmark = pytest.mark.gpu

# 256 threads x 4 float4 per block for kind 1, 256 x 1 for kind 0
LENGTHS = [0, 4, 4 * 1024 * 3, 4 * (1024 * 3 + 7), 4 * 256 * 5 + 4 * 13, 1 << 22]


def _dyadic(n, seed):
    g = torch.Generator().manual_seed(seed)
    return (torch.randint(-256, 257, (n,), generator=g).float() / 16).cuda()


@pytest.mark.parametrize("n", LENGTHS)
def test_copy(n):
    print(f"case copy n={n}", flush=True)
    a = _dyadic(n + 4, 1)[:n]
    out = torch.full((n + 4,), 7.0, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    _abi.fd_stream_probe(0, a.data_ptr(), None, out.data_ptr(), n, s)
    torch.cuda.synchronize()
    assert torch.equal(out[:n], a)
    assert torch.all(out[n:] == 7.0)          # nothing written past n


@pytest.mark.parametrize("n", LENGTHS)
def test_update_in_place(n):
    print(f"case update n={n}", flush=True)
    a, b, z = _dyadic(n + 4, 2)[:n], _dyadic(n + 4, 3)[:n], _dyadic(n + 4, 4)
    want = (a.double() + b.double() * z[:n].double()).float()
    s = torch.cuda.current_stream().cuda_stream
    tail = z[n:].clone()
    _abi.fd_stream_probe(1, a.data_ptr(), b.data_ptr(), z.data_ptr(), n, s)
    torch.cuda.synchronize()
    assert torch.equal(z[:n], want)
    assert torch.equal(z[n:], tail)
