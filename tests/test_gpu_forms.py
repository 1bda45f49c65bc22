"""Convective forms (divergence, skew-symmetric, rotational, EMAC) on the GPU:
forward, velocity VJP and JVP against the oracle element by element, on
meshes spanning several patches with ragged tails, under every scatter
strategy; mixed precision; the kinetic-energy property at full size; and
autograd through the Function."""

import numpy as np
import pytest
import torch

import oracle
from paper_2403_08777_amd import synth
from tests.gpu_helpers import Case, Prepared, log

pytestmark = pytest.mark.gpu

FORMS = ["divergence", "skew", "rotational", "emac"]
CASES = [Case(7, jitter=True, permute=True, mu=1e-3, form=f) for f in FORMS] + [
    Case(9, jitter=True, permute=True, mu=1e-4, cs=0.1, form="skew"),
    Case(9, jitter=True, permute=True, mu=1e-4, cs=0.1, model="vreman", form="emac"),
    Case(5, jitter=False, permute=True, mu=1e-3, cs=0.1, form="rotational"),
]


def _jvp_dirs(pr):
    rng = np.random.default_rng(21)
    return rng.standard_normal(pr.u.shape), rng.standard_normal(pr.p.shape)


@pytest.mark.parametrize("scatter", ["atomic", "patch", "patch_gather"])
@pytest.mark.parametrize("case", CASES, ids=[c.label() for c in CASES])
def test_forms_fp64_parity(case, scatter):
    from paper_2403_08777_amd import api

    log(f"forms fp64 {case.label()} {scatter}")
    pr = Prepared(case, scatter=scatter)
    e1 = oracle.rel_l2(pr.rhs(), pr.oracle_rhs())
    e2 = oracle.rel_l2(pr.vjp(), pr.oracle_vjp())
    du, dp = _jvp_dirs(pr)
    u, _, _ = pr.fields(torch.float64)
    tm = lambda a: pr.mesh.to_mesh_order(torch.from_numpy(np.ascontiguousarray(a)).to(pr.dev))
    got = pr.mesh.from_mesh_order(api.assemble_rhs_jvp(pr.mesh, u, tm(du), tm(dp), case.params())).cpu().numpy()
    e3 = oracle.rel_l2(got, oracle.jvp(pr.m.coords, pr.m.conn, pr.u, pr.p, du, dp, case.oracle_params()))
    log(f"  rhs {e1:.2e} vjp {e2:.2e} jvp {e3:.2e}")
    assert e1 <= 1e-12 and e2 <= 1e-12 and e3 <= 1e-12


@pytest.mark.parametrize("form", FORMS)
def test_forms_mixed(form):
    case = Case(16, jitter=True, permute=True, mu=1e-4, cs=0.1, form=form)
    pr = Prepared(case)
    er = oracle.rel_l2(pr.rhs(torch.float32), pr.oracle_rhs())
    eg = oracle.rel_l2(pr.vjp(torch.float32), pr.oracle_vjp())
    log(f"forms mixed {case.label()}: rhs {er:.2e} vjp {eg:.2e}")
    assert er <= 1e-4 and eg <= 1e-4


def test_forms_vjp_dense_jacobian():
    """The kernel VJP of the EMAC form with Vreman against the oracle's
    complex-step Jacobian of the definition-based forward (2^3 mesh)."""
    case = Case(2, jitter=True, permute=True, mu=1e-3, cs=0.1, model="vreman", form="emac")
    pr = Prepared(case)
    jac = oracle.dense_jacobian_complex_step(pr.m.coords, pr.m.conn, pr.u, pr.p, case.oracle_params())
    ref = (jac.T @ pr.lam.reshape(-1)).reshape(-1, 3)
    assert oracle.rel_l2(pr.vjp(), ref) <= 1e-12


@pytest.mark.parametrize("form", ["skew", "rotational"])
def test_forms_energy_full_size(form):
    """96^3 jittered mesh in the benchmark's launch configuration, u zero on
    the boundary: the convective term's kinetic-energy exchange
    sum_n u_n . R_n vanishes to rounding for the energy-preserving forms
    (no oracle needed at this size), while the advective form's does not."""
    from paper_2403_08777_amd import api

    wl = synth.WORKLOADS["cube96_jit_perm"]
    m, u, p, _ = synth.build(wl)
    bnd = np.any((m.coords < 1e-12) | (m.coords > 1 - 1e-12), axis=1)
    u = u.copy()
    u[bnd] = 0.0
    dev = torch.device("cuda")
    mesh = api.Mesh(torch.from_numpy(m.coords).to(dev), torch.from_numpy(m.conn).to(dev))
    ut = mesh.to_mesh_order(torch.from_numpy(u).to(dev))
    pz = torch.zeros(m.n_nodes, dtype=torch.float64, device=dev)
    res = {}
    for f in (form, "advective"):
        prm = api.Params(wl.rho, 0.0, 0.0, (0.0, 0.0, 0.0), "smagorinsky", f)
        r = api.assemble_rhs(mesh, ut, pz, prm)
        res[f] = (float((ut * r).sum()), float((ut * r).abs().sum()))
    log(f"energy 96^3 {form}: {res[form][0]:.3e} / {res[form][1]:.3e}; advective {res['advective'][0]:.3e}")
    assert abs(res[form][0]) <= 1e-13 * res[form][1]
    assert abs(res["advective"][0]) > 1e-8 * res["advective"][1]


def test_forms_full_size_parity():
    """The skew-symmetric form with Vreman on the 96^3 jittered benchmark
    mesh, FP64 forward and VJP against the full oracle."""
    from paper_2403_08777_amd import api

    wl = synth.WORKLOADS["cube96_jit_perm"]
    m, u, p, lam = synth.build(wl)
    dev = torch.device("cuda")
    mesh = api.Mesh(torch.from_numpy(m.coords).to(dev), torch.from_numpy(m.conn).to(dev))
    prm = api.Params(wl.rho, wl.mu, 0.1, wl.body_force, "vreman", "skew")
    oprm = oracle.Params(wl.rho, wl.mu, 0.1, wl.body_force, model="vreman", form="skew")
    tm = lambda a: mesh.to_mesh_order(torch.from_numpy(np.ascontiguousarray(a)).to(dev))
    r = mesh.from_mesh_order(api.assemble_rhs(mesh, tm(u), tm(p), prm)).cpu().numpy()
    g = mesh.from_mesh_order(api.assemble_rhs_vjp(mesh, tm(u), tm(lam), prm)).cpu().numpy()
    er = oracle.rel_l2(r, oracle.rhs(m.coords, m.conn, u, p, oprm))
    eg = oracle.rel_l2(g, oracle.vjp(m.coords, m.conn, u, lam, oprm))
    log(f"96^3 skew+vreman fp64: rhs {er:.2e} vjp {eg:.2e}")
    assert er <= 1e-12 and eg <= 1e-12


def test_forms_autograd():
    from paper_2403_08777_amd import api

    case = Case(3, jitter=True, permute=True, mu=1e-2, cs=0.1, form="emac")
    pr = Prepared(case)
    u, p, _ = pr.fields(torch.float64)
    prm = case.params()
    uu = u.clone().requires_grad_(True)
    pp = p.clone().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: api.NSAssembleRHS.apply(a, b, pr.mesh, prm), (uu, pp),
                                    eps=1e-6, atol=1e-8, rtol=1e-6)
