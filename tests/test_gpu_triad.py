"""The streaming calibration kernel c = a + s b (jfnk_stream_triad): exact
for s = 0.5 (the product is exact, one rounding in the sum), within one
rounding of the FMA otherwise; odd lengths (the scalar tail), n = 0, and
the argument checks."""
import ctypes

import pytest

torch = pytest.importorskip('torch')
pytestmark = pytest.mark.gpu

from paper_2103_13890_amd import _lib, api


@pytest.mark.parametrize('n', [1, 2, 7, 4097, (1 << 22) + 3])
def test_triad_values(n):
    g = torch.Generator(device='cuda').manual_seed(n)
    a = torch.rand(n, dtype=torch.float64, device='cuda', generator=g)
    b = torch.rand(n, dtype=torch.float64, device='cuda', generator=g)
    c = torch.full_like(a, float('nan'))
    api.jfnk_stream_triad(a, b, c, 0.5)
    assert torch.equal(c, a + 0.5 * b)
    api.jfnk_stream_triad(a, b, c, 1.0 / 3.0)
    ref = (a.cpu() + (1.0 / 3.0) * b.cpu()).cuda()
    assert float(((c - ref).abs() / ref.abs()).max()) <= 2 * 2.0 ** -53


def test_triad_arguments():
    lib = _lib.load()
    a = torch.zeros(16, dtype=torch.float64, device='cuda')
    p = ctypes.c_void_p(a.data_ptr())
    assert lib.jfnk_stream_triad(p, p, p, 0, 1.0, None) == _lib.OK
    assert lib.jfnk_stream_triad(p, p, p, -1, 1.0, None) != _lib.OK
    assert lib.jfnk_stream_triad(None, p, p, 4, 1.0, None) != _lib.OK
    odd = ctypes.c_void_p(a.data_ptr() + 8)
    assert lib.jfnk_stream_triad(odd, p, p, 4, 1.0, None) != _lib.OK
