"""Velocity VJP on the GPU: central finite differences of the GPU forward,
the oracle's complex-step dense Jacobian, and torch.autograd.gradcheck through
the autograd.Function."""

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_helpers import Case, Prepared, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("cs,mu,model", [(0.0, 1e-3, "smagorinsky"), (0.1, 1e-4, "smagorinsky"),
                                         (0.1, 1e-4, "vreman")])
def test_vjp_central_fd_16(cs, mu, model):
    from paper_2403_08777_amd import api

    case = Case(16, jitter=True, permute=True, mu=mu, cs=cs, model=model)
    log(f"fd {case.label()}")
    pr = Prepared(case)
    u, p, lam = pr.fields(torch.float64)
    d = pr.mesh.to_mesh_order(torch.from_numpy(np.random.default_rng(5).standard_normal(pr.u.shape)).to(pr.dev))
    h = 1e-6
    prm = case.params()
    rp = api.assemble_rhs(pr.mesh, u + h * d, p, prm)
    rm = api.assemble_rhs(pr.mesh, u - h * d, p, prm)
    fd = float((lam * rp).sum() - (lam * rm).sum()) / (2 * h)
    g = api.assemble_rhs_vjp(pr.mesh, u, lam, prm)
    gd = float((g * d).sum())
    log(f"  fd={fd:.12e} vjp.d={gd:.12e}")
    assert abs(fd - gd) <= 1e-6 * abs(gd)


@pytest.mark.parametrize("cs,model", [(0.0, "smagorinsky"), (0.1, "smagorinsky"), (0.1, "vreman")])
def test_vjp_dense_jacobian_2(cs, model):
    case = Case(2, jitter=True, permute=True, mu=1e-3, cs=cs, model=model)
    pr = Prepared(case)
    jac = oracle.dense_jacobian_complex_step(pr.m.coords, pr.m.conn, pr.u, pr.p, case.oracle_params())
    ref = (jac.T @ pr.lam.reshape(-1)).reshape(-1, 3)
    err = oracle.rel_l2(pr.vjp(), ref)
    log(f"dense jacobian cs={cs}: rel_l2={err:.3e}")
    assert err <= 1e-12


def test_autograd_function_gradcheck():
    from paper_2403_08777_amd import api

    case = Case(2, jitter=True, permute=True, mu=1e-2, cs=0.1)
    pr = Prepared(case)
    u, p, _ = pr.fields(torch.float64)
    u = u.clone().requires_grad_(True)
    prm = case.params()
    assert torch.autograd.gradcheck(lambda v: api.NSAssembleRHS.apply(v, p, pr.mesh, prm), (u,), eps=1e-6,
                                    atol=1e-8, rtol=1e-6)


def test_autograd_backward_matches_vjp():
    from paper_2403_08777_amd import api

    case = Case(8, jitter=True, permute=True, mu=1e-4, cs=0.1)
    pr = Prepared(case)
    u, p, lam = pr.fields(torch.float64)
    uu = u.clone().requires_grad_(True)
    rhs = api.NSAssembleRHS.apply(uu, p, pr.mesh, case.params())
    (rhs * lam).sum().backward()
    g = api.assemble_rhs_vjp(pr.mesh, u, lam, case.params())
    assert oracle.rel_l2(uu.grad.cpu().numpy(), g.cpu().numpy()) <= 1e-14
    with pytest.raises(NotImplementedError):
        api.NSAssembleRHS.apply(uu, p.clone().requires_grad_(True), pr.mesh, case.params())
