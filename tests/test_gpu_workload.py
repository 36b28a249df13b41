"""The seeded generators give the same words on a GPU tensor as on the CPU (torch int64 wraps)."""
import pytest
import torch

from paper_2603_17168_amd.workload import keys, randint, uniform_u64, value_rows

pytestmark = pytest.mark.gpu


def test_generators_match_cpu():
    for stream, n, start in [(1, 1000, 0), (7, 4097, 123456789)]:
        assert torch.equal(keys(stream, n, start), keys(stream, n, start, device="cuda").cpu())
        assert torch.equal(uniform_u64(stream, n, start), uniform_u64(stream, n, start, device="cuda").cpu())
        assert torch.equal(randint(stream, n, 1 << 30, start), randint(stream, n, 1 << 30, start, device="cuda").cpu())
    v = keys(3, 777)
    a = value_rows(5, v, 32).view(torch.int32)
    b = value_rows(5, v.cuda(), 32).cpu().view(torch.int32)
    assert torch.equal(a, b)
