"""Parity on an unstructured mesh: the Delaunay tetrahedralisation of 40,000
seeded random points in the unit cube (synth.delaunay_mesh) (268 K tetrahedra, node valence up to
86, random node ids, slivers with |det J| / (|d1||d2||d3|) down to 3e-6).
The cube meshes of the other tests are lattices; this one exercises the
mesh preprocessing (Hilbert order, first-touch numbering, patch runs up to the
highest valence, bank-aware run placement and node colouring) on the kind of
irregular topology an LES mesh has.  FP64 forward, velocity and pressure VJPs
and JVP against the oracle in every scatter strategy, with no eddy viscosity,
Smagorinsky and Vreman; the other convective forms; the lumped volume and the
explicit update with a Dirichlet mask; mixed precision on the mesh without
its worst slivers."""

import numpy as np
import pytest
import torch

import oracle
from paper_2403_08777_amd import synth
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
# Vreman on every element, slivers included: the oracle's rounding on the
# worst-conditioned elements (see _vreman_conditioned), not the kernel's
VREMAN_ILL = 1e-8  # measured 3.2e-9 (VJP)
TOL_MIXED = 3e-6  # about ten times the measured 3.7e-7 (Smagorinsky forward)
_MESH = {}


def _delaunay():
    if "m" not in _MESH:
        pts, conn = synth.delaunay_mesh(40000, seed=23)
        _MESH["m"] = (pts, conn, *synth.unstructured_fields(pts, seed=24))
    return _MESH["m"]


def _quality(coords, conn):
    d = coords[conn[:, 1:]] - coords[conn[:, :1]]
    det = np.einsum("ij,ij->i", d[:, 0], np.cross(d[:, 1], d[:, 2]))
    return np.abs(det) / np.linalg.norm(d, axis=2).prod(axis=1)


def _vreman_conditioned(coords, conn, u, floor=1e-6):
    """Elements whose Vreman invariant B = |cof G|^2 is at least `floor` A^2,
    A = |G|^2.  Below that, B written as 2x2 minors of beta = G^T G (the model's
    definition, which the oracle keeps) cancels to a relative error of about
    eps A^2 / B; the worst sliver here (B / A^2 = 4.5e-12) loses 4e-6 of its eddy
    viscosity that way."""
    vol, gn = oracle.geometry(coords, conn)
    g = np.einsum("eai,eaj->eij", gn, u[conn])
    cof = np.stack([np.cross(g[:, (i + 1) % 3], g[:, (i + 2) % 3]) for i in range(3)], axis=1)
    b, a = np.sum(cof * cof, axis=(1, 2)), np.sum(g * g, axis=(1, 2))
    return conn[b >= floor * a * a]


def _errors(conn, scatter, prm, oprm, log_prefix):
    from paper_2403_08777_amd import api

    pts, _, u, p, lam, du, dp = _delaunay()
    dev = torch.device("cuda")
    mesh = api.Mesh(torch.from_numpy(pts).to(dev), torch.from_numpy(conn).to(dev), scatter=scatter)
    log(f"{log_prefix}: {conn.shape[0]} tets, {mesh.info}")
    tm = lambda a: mesh.to_mesh_order(torch.from_numpy(np.ascontiguousarray(a)).to(dev))
    back = lambda t: mesh.from_mesh_order(t).cpu().numpy()
    ut, pt, lt = tm(u), tm(p), tm(lam)
    r = back(api.assemble_rhs(mesh, ut, pt, prm))
    g = back(api.assemble_rhs_vjp(mesh, ut, lt, prm))
    gp = back(api.assemble_rhs_vjp_p(mesh, lt, prm))
    jv = back(api.assemble_rhs_jvp(mesh, ut, tm(du), tm(dp), prm))
    errs = {"rhs": oracle.rel_l2(r, oracle.rhs(pts, conn, u, p, oprm)),
            "vjp": oracle.rel_l2(g, oracle.vjp(pts, conn, u, lam, oprm)),
            "vjp_p": oracle.rel_l2(gp, oracle.vjp_p(pts, conn, lam)),
            "jvp": oracle.rel_l2(jv, oracle.jvp(pts, conn, u, p, du, dp, oprm))}
    log("  " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    if mesh.info["scatter"] == "patch_gather":
        # the fixed summation order gives the same bits on every call
        assert np.array_equal(back(api.assemble_rhs(mesh, ut, pt, prm)), r)
        assert np.array_equal(back(api.assemble_rhs_vjp(mesh, ut, lt, prm)), g)
    mesh.close()
    return errs


@pytest.mark.parametrize("scatter", ["auto", "patch", "atomic"])
@pytest.mark.parametrize("cs,model", [(0.0, "smagorinsky"), (0.1, "smagorinsky"), (0.1, "vreman")])
def test_unstructured_fp64(scatter, cs, model):
    from paper_2403_08777_amd import api

    pts, conn, u = _delaunay()[:3]
    prm = api.Params(1.0, 1e-3, cs, synth.BODY_FORCE, model)
    oprm = oracle.Params(1.0, 1e-3, cs, synth.BODY_FORCE, model)
    if model == "vreman":
        full = _errors(conn, scatter, prm, oprm, f"delaunay ({scatter}, {model}, all elements)")
        assert all(v <= VREMAN_ILL for v in full.values())
        conn = _vreman_conditioned(pts, conn, u)
    errs = _errors(conn, scatter, prm, oprm, f"delaunay ({scatter}, {model}, cs={cs})")
    assert all(v <= TOL64 for v in errs.values())


@pytest.mark.parametrize("model", ["smagorinsky", "vreman"])
def test_unstructured_mixed(model):
    """Mixed precision (FP64 geometry, FP32 fields and arithmetic) on the same
    mesh without the 0.1 % of elements whose quality is below 1e-3: on the
    slivers the gradients reach 1e5 times the mesh's typical ones and the
    FP32 rounding of the element terms, not the method, decides the error."""
    from paper_2403_08777_amd import api

    pts, conn, u, p, lam, du, dp = _delaunay()
    conn = conn[_quality(pts, conn) >= 1e-3]
    if model == "vreman":
        conn = _vreman_conditioned(pts, conn, u)
    dev = torch.device("cuda")
    mesh = api.Mesh(torch.from_numpy(pts).to(dev), torch.from_numpy(conn).to(dev))
    prm = api.Params(1.0, 1e-3, 0.1, synth.BODY_FORCE, model)
    oprm = oracle.Params(1.0, 1e-3, 0.1, synth.BODY_FORCE, model)
    tm = lambda a: mesh.to_mesh_order(torch.from_numpy(np.ascontiguousarray(a)).to(dev, torch.float32))
    back = lambda t: mesh.from_mesh_order(t).double().cpu().numpy()
    r = back(api.assemble_rhs(mesh, tm(u), tm(p), prm))
    g = back(api.assemble_rhs_vjp(mesh, tm(u), tm(lam), prm))
    er = oracle.rel_l2(r, oracle.rhs(pts, conn, u, p, oprm))
    eg = oracle.rel_l2(g, oracle.vjp(pts, conn, u, lam, oprm))
    log(f"delaunay mixed {model} ({conn.shape[0]} tets): rhs {er:.2e}, grad {eg:.2e}")
    assert er <= TOL_MIXED and eg <= TOL_MIXED
    mesh.close()


@pytest.mark.parametrize("form", ["divergence", "skew", "rotational", "emac"])
def test_unstructured_forms(form):
    """The convective forms other than the advective one, FP64 forward, VJP and
    JVP, with Smagorinsky, on every element."""
    from paper_2403_08777_amd import api

    conn = _delaunay()[1]
    prm = api.Params(1.0, 1e-3, 0.1, synth.BODY_FORCE, "smagorinsky", form)
    oprm = oracle.Params(1.0, 1e-3, 0.1, synth.BODY_FORCE, "smagorinsky", form)
    errs = _errors(conn, "auto", prm, oprm, f"delaunay ({form})")
    assert all(v <= TOL64 for v in errs.values())


def test_unstructured_update():
    """Lumped volume and one explicit stage with a random Dirichlet mask, in
    place and out of place, FP64."""
    from paper_2403_08777_amd import api

    pts, conn, u, p = _delaunay()[:4]
    dev = torch.device("cuda")
    dt = 1e-4
    mesh = api.Mesh(torch.from_numpy(pts).to(dev), torch.from_numpy(conn).to(dev))
    prm = api.Params(1.0, 1e-3, 0.1, synth.BODY_FORCE)
    oprm = oracle.Params(1.0, 1e-3, 0.1, synth.BODY_FORCE)
    back = lambda t: mesh.from_mesh_order(t).cpu().numpy()
    vl = back(mesh.lumped_volume())
    vref = oracle.lumped_volume(pts, conn)
    e_vol = float(np.max(np.abs(vl - vref) / vref))
    mask_np = np.random.default_rng(5).integers(0, 8, pts.shape[0]).astype(np.uint8)
    mask = mesh.to_mesh_order(torch.from_numpy(mask_np.astype(np.float64)).to(dev)).to(torch.uint8)
    ut, pt = mesh.to_mesh_order(torch.from_numpy(u).to(dev)), mesh.to_mesh_order(torch.from_numpy(p).to(dev))
    rhs = torch.empty_like(ut)
    un = back(api.explicit_update(mesh, ut, pt, prm, dt, mask, rhs=rhs))
    ref, ref_r = oracle.explicit_update(pts, conn, u, p, oprm, dt, mask_np)
    fixed = np.stack([(mask_np >> i) & 1 for i in range(3)], axis=1).astype(bool)
    assert np.array_equal(un[fixed], u[fixed])
    e_inc = oracle.rel_l2(un - u, ref - u)
    e_rhs = oracle.rel_l2(back(rhs), ref_r)
    uu = ut.clone()
    api.explicit_update(mesh, uu, pt, prm, dt, out=uu)
    ref0, _ = oracle.explicit_update(pts, conn, u, p, oprm, dt)
    e_inp = oracle.rel_l2(back(uu) - u, ref0 - u)
    log(f"delaunay update: lumped max rel {e_vol:.2e}, increment {e_inc:.2e}, rhs {e_rhs:.2e}, in place {e_inp:.2e}")
    assert e_vol <= 1e-14 and e_inc <= TOL64 and e_rhs <= TOL64 and e_inp <= TOL64
    mesh.close()


def test_unstructured_mixed_tangents():
    """Mixed-precision JVP and pressure VJP on the sliver-filtered mesh."""
    from paper_2403_08777_amd import api

    pts, conn, u, p, lam, du, dp = _delaunay()
    conn = conn[_quality(pts, conn) >= 1e-3]
    dev = torch.device("cuda")
    mesh = api.Mesh(torch.from_numpy(pts).to(dev), torch.from_numpy(conn).to(dev))
    prm = api.Params(1.0, 1e-3, 0.1, synth.BODY_FORCE)
    oprm = oracle.Params(1.0, 1e-3, 0.1, synth.BODY_FORCE)
    tm = lambda a: mesh.to_mesh_order(torch.from_numpy(np.ascontiguousarray(a)).to(dev, torch.float32))
    back = lambda t: mesh.from_mesh_order(t).double().cpu().numpy()
    jv = back(api.assemble_rhs_jvp(mesh, tm(u), tm(du), tm(dp), prm))
    gp = back(api.assemble_rhs_vjp_p(mesh, tm(lam), prm))
    ej = oracle.rel_l2(jv, oracle.jvp(pts, conn, u, p, du, dp, oprm))
    ep = oracle.rel_l2(gp, oracle.vjp_p(pts, conn, lam))
    log(f"delaunay mixed tangents ({conn.shape[0]} tets): jvp {ej:.2e}, vjp_p {ep:.2e}")
    assert ej <= TOL_MIXED and ep <= TOL_MIXED
    mesh.close()
