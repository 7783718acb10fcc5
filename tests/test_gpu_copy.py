"""The copy kernel behind the bandwidth calibration (the copy experiment of Sec. 4.2).

Its measured rate is the practical DRAM ceiling the step kernels are compared with, and the
byte counts of the HBM traffic counters are scaled by what the counters read for it, so the
kernel must move exactly the bytes it is asked to: every byte of the range copied, nothing
written past its end, and sizes that are not a multiple of 16 refused.
"""
import pytest

from gpu_util import announce

pytestmark = pytest.mark.gpu

GUARD = 4096


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_13241_amd as m
    m.load()
    return m


def _random_bytes(n, seed):
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    return torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda", generator=g)


# 16 B: a single lane; 4 KiB + 16: a partial last workgroup; 1 GiB + 48: more 16-byte
# elements than the capped grid has threads, so the grid-stride loop takes a second lap.
@pytest.mark.parametrize("nbytes", [16, 4096 + 16, (1 << 30) + 48])
def test_copy_moves_exactly_the_range(lbm, nbytes):
    import torch
    announce(f"copy kernel {nbytes} bytes")
    src = _random_bytes(nbytes + GUARD, seed=nbytes % 1000)
    dst = torch.zeros(nbytes + GUARD, dtype=torch.uint8, device="cuda")
    # the guard region holds a known pattern that must survive the copy
    dst[nbytes:] = 0xA5
    lbm.copy_kernel(src, dst, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])
    assert bool((dst[nbytes:] == 0xA5).all())
    del src, dst


@pytest.mark.parametrize("nbytes", [8, 24, 4096 + 4])
def test_copy_refuses_sizes_not_multiple_of_16(lbm, nbytes):
    import torch
    announce(f"copy kernel refuses {nbytes} bytes")
    src = torch.ones(nbytes + 16, dtype=torch.uint8, device="cuda")
    dst = torch.zeros(nbytes + 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(lbm.LbmError):
        lbm.copy_kernel(src, dst, nbytes)
    torch.cuda.synchronize()
    assert int(dst.sum()) == 0
