"""The library's streaming copy kernel (mbt_stream_copy), used as the
achievable-bandwidth yardstick beside the HBM peak: every byte arrives, no
byte past the range is written, for sizes below one 16-byte element per
thread, with a ragged last workgroup, and large enough for many thousands of
workgroups (one element per thread, 4 KiB per workgroup)."""
import pytest
import torch

from paper_1809_00391_amd import tracker as tr

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 4096 * 16 + 48, (64 << 20) + 48])
def test_stream_copy_exact(cuda, nbytes):
    print(f"[gpu case] stream copy nbytes={nbytes}", flush=True)
    g = torch.Generator(device="cuda").manual_seed(nbytes)
    n = nbytes // 4
    src = torch.randint(-2**31, 2**31 - 1, (n,), dtype=torch.int32, device="cuda", generator=g)
    guard = 64  # elements on each side of the destination range
    dst = torch.full((n + 2 * guard,), 0x5A5A5A5A, dtype=torch.int32, device="cuda")
    tr.stream_copy(src, dst[guard:guard + n])
    torch.cuda.synchronize()
    assert torch.equal(dst[guard:guard + n], src)
    assert bool((dst[:guard] == 0x5A5A5A5A).all()) and bool((dst[guard + n:] == 0x5A5A5A5A).all())
