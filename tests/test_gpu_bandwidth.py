"""The Scale bandwidth kernel (b = s a) on the GPU: bitwise equal to the same
multiplication done by torch, in the 16-byte path (odd and even lengths,
several blocks and a ragged last block) and the 8-byte path (misaligned
arrays), nothing written past n, and the host-side refusals."""

import pytest
import torch

from paper_2403_08777_amd import api
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 1023, 1024, 1025, 2 * 1024 + 7, 4096 * 5 + 1, (1 << 20) + 1, (1 << 22) + 3]


def _call(a_ptr, b_ptr, n, s):
    return api.lib.nsasm_stream_scale(a_ptr, b_ptr, n, s, torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("offset", [0, 1], ids=["aligned", "misaligned"])
def test_scale_matches_torch(n, offset):
    g = torch.Generator(device="cuda").manual_seed(n)
    base = torch.randn(n + offset, dtype=torch.float64, device="cuda", generator=g)
    a = base[offset:]
    out = torch.full((n + 16,), 7.0, dtype=torch.float64, device="cuda")
    s = -1.7
    log(f"scale n={n} offset={offset}")
    assert _call(a.data_ptr(), out.data_ptr(), n, s) == 0
    torch.cuda.synchronize()
    assert torch.equal(out[:n], a * s)
    assert torch.equal(out[n:], torch.full((16,), 7.0, dtype=torch.float64, device="cuda"))


def test_binding_and_refusals():
    a = torch.arange(1000, dtype=torch.float64, device="cuda")
    assert torch.equal(api.stream_scale(a, 0.5), a * 0.5)
    assert api.stream_scale(a[:0], 2.0).numel() == 0
    # in place and partial overlap are refused before any launch
    assert _call(a.data_ptr(), a.data_ptr(), 1000, 2.0) == 1
    assert b"overlap" in api.lib.nsasm_last_error()
    assert _call(a.data_ptr(), a.data_ptr() + 8 * 999, 1000, 2.0) == 1
    # adjacent but disjoint halves are fine
    assert _call(a.data_ptr(), a.data_ptr() + 8 * 500, 500, 2.0) == 0
    torch.cuda.synchronize()
    assert torch.equal(a[500:], torch.arange(500, dtype=torch.float64, device="cuda") * 2.0)
    with pytest.raises(TypeError):
        api.stream_scale(a.float(), 2.0)
    with pytest.raises(ValueError):
        api.stream_scale(a.view(10, 100), 2.0)
