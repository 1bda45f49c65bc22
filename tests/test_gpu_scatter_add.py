"""The atomic-rate measurement kernel (nsasm_scatter_add) computes what it
claims: out[index[k], c] += value, entries outside the rows skipped; checked
against numpy's unbuffered add on the host (sums of equal small values are
exact in both precisions)."""

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_scatter_add_matches_host(dtype):
    from paper_2403_08777_amd import api

    rng = np.random.default_rng(3)
    rows, ncomp = 57, 3
    idx = rng.integers(-5, rows + 5, 5000).astype(np.int32)   # some entries out of range
    base = rng.integers(-4, 5, (rows, ncomp)).astype(np.float64)
    dev = torch.device("cuda")
    out = torch.from_numpy(base).to(dev, dtype)
    api.scatter_add(torch.from_numpy(idx).to(dev), out, value=0.5)
    torch.cuda.synchronize()
    ref = base.copy()
    keep = (idx >= 0) & (idx < rows)
    np.add.at(ref, idx[keep], 0.5)
    assert np.array_equal(out.double().cpu().numpy(), ref)


def test_scatter_add_arguments():
    from paper_2403_08777_amd import api

    dev = torch.device("cuda")
    out = torch.zeros((4, 2), dtype=torch.float64, device=dev)
    api.scatter_add(torch.empty(0, dtype=torch.int32, device=dev), out)   # nothing to do
    assert float(out.abs().sum()) == 0.0
    with pytest.raises(api.NsasmError):
        api.scatter_add(torch.zeros(3, dtype=torch.int32, device=dev), torch.zeros((4, 17), device=dev,
                                                                                  dtype=torch.float64))
