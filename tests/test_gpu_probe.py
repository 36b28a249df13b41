"""The memory-system reference kernels that price the table's kernels: the copy moves exactly the
source bytes (ragged sizes included) and each random gather reads the width-aligned unit its
published mixing function names (SplitMix64's output function of the access index xor salt)."""
import numpy as np
import pytest
import torch

from paper_2603_17168_amd import cskv

pytestmark = pytest.mark.gpu

M64 = (1 << 64) - 1


def mix(z: int) -> int:
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


@pytest.mark.parametrize("nbytes", [16, 4096, 4096 + 16, (1 << 20) + 48, 3 * (1 << 22) + 4080])
def test_probe_copy_exact(nbytes):
    dev = torch.device("cuda", 0)
    g = torch.Generator().manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, generator=g).to(dev)
    pad = torch.full((nbytes + 64,), 0xA5, dtype=torch.uint8, device=dev)
    dst = pad[:nbytes]
    cskv.probe_copy(src, dst)
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    assert bool((pad[nbytes:] == 0xA5).all().item()), "the copy wrote past the buffer"


def test_probe_copy_rejects_bad_arguments():
    dev = torch.device("cuda", 0)
    a = torch.zeros(64, dtype=torch.uint8, device=dev)
    b = torch.zeros(64, dtype=torch.uint8, device=dev)
    with pytest.raises(cskv.CskvError):
        cskv.probe_copy(a[:40], b[:40])  # not a multiple of 16
    with pytest.raises(cskv.CskvError):
        cskv.probe_copy(a[1:33], b[1:33])  # misaligned


@pytest.mark.parametrize("width", [8, 16, 32, 64, 128])
def test_probe_gather_reads_the_named_units(width):
    dev = torch.device("cuda", 0)
    src_bytes = 1 << 16
    g = torch.Generator().manual_seed(width)
    src = torch.randint(0, 256, (src_bytes,), dtype=torch.uint8, generator=g)
    n, salt = 1000, 12345
    out = torch.zeros(n * width, dtype=torch.uint8, device=dev)
    cskv.probe_gather(src.to(dev), width, n, salt, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(n, width)
    s = src.numpy()
    units = src_bytes // width
    for i in range(n):
        u = mix(i ^ salt) & (units - 1)
        assert np.array_equal(got[i], s[u * width:(u + 1) * width]), f"access {i}"
