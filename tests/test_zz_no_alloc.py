"""nsasm_assemble_rhs_noalloc, the allocation-free variant of the forward
assembly: through the C ABI (the ctypes binding) its output must equal
nsasm_assemble_rhs's on the same mesh -- bit for bit with the gather scatter,
whose summation order is fixed and only the partial-sum buffer differs --
and the FP64 oracle's within the FP64 tolerance, over consecutive calls that
share the library's one scratch region (the second on a smaller mesh), and it
must refuse a mesh whose partial sums exceed the region."""

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_helpers import Case, Prepared, log

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
SCRATCH_BYTES = 64 << 20


def _noalloc(pr, dtype, accumulate_into=None):
    from paper_2403_08777_amd import api

    u, p, _ = pr.fields(dtype)
    out = torch.empty_like(u) if accumulate_into is None else accumulate_into.clone()
    api.assemble_rhs_noalloc(pr.mesh, u, p, pr.case.params(), out=out, accumulate=accumulate_into is not None)
    torch.cuda.synchronize()
    return out


def _regular(pr, dtype):
    from paper_2403_08777_amd import api

    u, p, _ = pr.fields(dtype)
    out = api.assemble_rhs(pr.mesh, u, p, pr.case.params())
    torch.cuda.synchronize()
    return out


def _check_case(pr, dtype):
    got = _noalloc(pr, dtype)
    ref = _regular(pr, dtype)
    assert torch.equal(got, ref), f"{pr.case.label()} {dtype}: differs from nsasm_assemble_rhs"
    if dtype == torch.float64:
        err = oracle.rel_l2(pr.mesh.from_mesh_order(got).cpu().numpy(), pr.oracle_rhs())
        log(f"[noalloc] {pr.case.label()}: rel L2 vs oracle {err:.2e}")
        assert err <= TOL64


def test_two_calls_in_a_row_second_smaller():
    big = Prepared(Case(16, jitter=True, permute=True, mu=1e-4, cs=0.1))
    small = Prepared(Case(5, jitter=True, permute=True, mu=1e-3))
    assert big.mesh.info["scatter"] == "patch_gather" and small.mesh.info["scatter"] == "patch_gather"
    assert small.mesh.info["patch_node_refs"] < big.mesh.info["patch_node_refs"]
    for dtype in (torch.float64, torch.float32):
        log(f"[noalloc] 16^3 then 5^3, {dtype}")
        _check_case(big, dtype)
        _check_case(small, dtype)   # the region still holds the larger call's sums
        _check_case(big, dtype)
    big.mesh.close()
    small.mesh.close()


def test_accumulate_and_atomic_scatter():
    pr = Prepared(Case(7, jitter=True, permute=True, mu=1e-4, cs=0.1))
    u, p, _ = pr.fields(torch.float64)
    base = torch.randn_like(u)
    got = _noalloc(pr, torch.float64, accumulate_into=base)
    assert torch.equal(got, base + _regular(pr, torch.float64))
    pr.mesh.close()
    # the atomic scatter uses no scratch memory: the same kernels as nsasm_assemble_rhs
    at = Prepared(Case(7, jitter=True, permute=True, mu=1e-4, cs=0.1), scatter="atomic")
    err = oracle.rel_l2(at.mesh.from_mesh_order(_noalloc(at, torch.float64)).cpu().numpy(), at.oracle_rhs())
    assert err <= TOL64
    at.mesh.close()


def test_full_size_96():
    """The 96^3 jittered relabelled cube (5,308,416 tets): its FP64 partial sums
    (57 MB) fit the region; the result equals nsasm_assemble_rhs bit for bit
    and matches the oracle at 64 sampled nodes' elements."""
    pr = Prepared(Case(96, jitter=True, permute=True, mu=1e-3))
    refs = pr.mesh.info["patch_node_refs"]
    assert 3 * refs * 8 <= SCRATCH_BYTES
    for dtype in (torch.float64, torch.float32):
        log(f"[noalloc] 96^3 {dtype}")
        got = _noalloc(pr, dtype)
        assert torch.equal(got, _regular(pr, dtype))
    got = pr.mesh.from_mesh_order(_noalloc(pr, torch.float64)).cpu().numpy()
    rng = np.random.default_rng(11)
    nodes = rng.choice(pr.m.n_nodes, 64, replace=False)
    touching = np.nonzero(np.isin(pr.m.conn, nodes).any(axis=1))[0]
    sub = pr.m.conn[touching]
    ref = oracle.rhs(pr.m.coords, sub, pr.u, pr.p, pr.case.oracle_params())
    err = oracle.rel_l2(got[nodes], ref[nodes])
    log(f"[noalloc] 96^3 sampled nodes: rel L2 vs oracle {err:.2e}")
    assert err <= TOL64
    pr.mesh.close()


def test_refuses_beyond_the_region():
    """112^3 cube (8.4 M tets): FP64 partial sums exceed 64 MiB and are refused
    with UNSUPPORTED; in mixed precision they fit and the call matches."""
    from paper_2403_08777_amd import api

    pr = Prepared(Case(112, jitter=False, permute=False))
    refs = pr.mesh.info["patch_node_refs"]
    assert 3 * refs * 8 > SCRATCH_BYTES >= 3 * refs * 4
    u, p, _ = pr.fields(torch.float64)
    with pytest.raises(api.NsasmError) as ei:
        api.assemble_rhs_noalloc(pr.mesh, u, p, pr.case.params(), out=torch.empty_like(u))
    assert ei.value.status_name == "UNSUPPORTED" and "at most" in str(ei.value)
    log("[noalloc] 112^3 mixed")
    assert torch.equal(_noalloc(pr, torch.float32), _regular(pr, torch.float32))
    pr.mesh.close()
