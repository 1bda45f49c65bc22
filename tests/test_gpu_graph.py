"""The assembly calls inside a captured HIP graph (torch.cuda.CUDAGraph): a
forward + VJP + explicit-update step is captured once and replayed several
times, with eager work and synchronisations between the replays; every
replay must reproduce the eager results bit for bit (gather scatter: fixed
summation order)."""

import pytest
import torch

from tests.gpu_helpers import Case, Prepared, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_graph_replay_matches_eager(dtype):
    from paper_2403_08777_amd import api

    case = Case(9, jitter=True, permute=True, mu=1e-4, cs=0.1, model="vreman", form="skew")
    pr = Prepared(case)
    u, p, lam = pr.fields(dtype)
    prm = case.params()
    rhs, grad, unew = torch.empty_like(u), torch.empty_like(u), torch.empty_like(u)

    def step():
        api.assemble_rhs(pr.mesh, u, p, prm, out=rhs)
        api.assemble_rhs_vjp(pr.mesh, u, lam, prm, out=grad)
        api.explicit_update(pr.mesh, u, p, prm, 1e-3, out=unew)

    step()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (rhs, grad, unew)]
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        step()
    for k in range(4):
        for t in (rhs, grad, unew):
            t.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ok = all(torch.equal(a, b) for a, b in zip((rhs, grad, unew), ref))
        log(f"graph replay {k} {dtype}: bitwise equal {ok}")
        assert ok
        # eager work between replays
        api.assemble_rhs(pr.mesh, u * 2, p, prm, out=rhs)
        torch.cuda.synchronize()
