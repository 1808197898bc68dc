"""The library's copy probe (measurement support): every load/store form copies the bytes
exactly, including a length that is not a multiple of the 256-element block or of the
eight-deep unrolled loop."""
import pytest
import torch

from paper_2207_11567_amd.solver import copy_probe

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
@pytest.mark.parametrize("n", [1, 255, 256 * 8192 * 8 + 12345])
def test_copy_probe_exact(mode, n):
    print(f"copy probe mode {mode} n {n}", flush=True)
    g = torch.Generator(device="cuda:0").manual_seed(n + mode)
    src = torch.randn(n, device="cuda:0", generator=g)
    buf = torch.full((n + 1024,), 7.0, device="cuda:0")
    dst = buf[:n]                                     # the 1024 elements after it must stay
    copy_probe(src, dst, mode)
    torch.cuda.synchronize()
    assert torch.equal(src.view(torch.int32), dst.view(torch.int32))
    assert torch.all(buf[n:] == 7.0)
