"""GPU check of the memory-bandwidth probes: both patterns are exact copies
(every byte of dst equals src), including a flat copy whose element count
is not a multiple of the block and several grids of a band sweep."""

import pytest

from _helpers import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("pattern,n,nbytes,wpc", [
    (0, 0, 16 * 1000 + 16 * 37, 0),
    (1, 128, 5 * 128 * 128 * 8, 0),
    (1, 384, 2 * 384 * 384 * 8, 16),
    (1, 256, 3 * 256 * 256 * 8, 32),
])
def test_bandwidth_probes_copy_exactly(pattern, n, nbytes, wpc):
    import torch
    from paper_1612_00746_amd import bandwidth_probe
    say(f"case: bandwidth probe pattern={pattern} n={n} bytes={nbytes} waves/CU={wpc}")
    g = torch.Generator(device="cpu").manual_seed(5)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, generator=g).cuda()
    dst = torch.zeros_like(src)
    bandwidth_probe(src, dst, pattern, n=n or 1024, waves_per_cu=wpc)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
