"""lf_stream_copy, the benchmark's bandwidth reference: an exact copy of four
arrays, for sizes that leave a partly filled last block (one element per
lane, a grid that covers the arrays once)."""
import pytest
import torch

from _parity import log
from paper_0911_5692_amd import stream_copy

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [0, 4, 1028, 256 * 1024 + 12, 3 * 65536 * 256 * 4 + 4 * 37])
def test_stream_copy_is_exact(n):
    log(f"[stream_copy] n={n}")
    g = torch.Generator(device="cuda").manual_seed(n)
    src = [torch.randn(n, generator=g, device="cuda", dtype=torch.float32) for _ in range(4)]
    dst = [torch.full((n,), float("nan"), device="cuda", dtype=torch.float32) for _ in range(4)]
    stream_copy(src, dst)
    torch.cuda.synchronize()
    for a, b in zip(src, dst):
        assert torch.equal(a, b)
