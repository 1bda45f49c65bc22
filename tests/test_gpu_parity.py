"""Parity of the HIP assembly with the CPU oracle, element by element (nodal
values), on seeded synthetic meshes.  FP64: relative L2 <= 1e-12 (atomic
summation order is the only difference besides FMA contraction and the
kernel's exact collapse of the Gauss sums).  Mixed precision: the error is
bounded loosely (catches bugs) and printed."""

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_helpers import Case, Prepared, log

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL_MIXED = 1e-4

SMALL = [
    Case(2),
    Case(2, jitter=True, permute=True, mu=1e-4, cs=0.1),
    Case(3, jitter=True, permute=True),           # ragged patches (162 elements)
    Case(4, jitter=True, permute=True, mu=1e-4, cs=0.1),
    Case(7, jitter=True, permute=True, mu=1e-4, cs=0.1),  # 2058 elements
    Case(16),                                     # 16^3 natural order, FP64 forward case
    Case(16, jitter=True, permute=True, mu=1e-4, cs=0.1),
]
MODES = [dict(scatter="atomic", renumber=False), dict(scatter="atomic", renumber=True),
         dict(scatter="patch", renumber=True), dict(scatter="patch_gather", renumber=True),
         dict(scatter="auto", renumber=True, patch_elems=64)]


def _ids(cases):
    return [c.label() for c in cases]


@pytest.mark.parametrize("mode", MODES, ids=lambda m: "-".join(f"{k}={v}" for k, v in m.items()))
@pytest.mark.parametrize("case", SMALL, ids=_ids(SMALL))
def test_forward_fp64(case, mode):
    log(f"forward fp64 {case.label()} {mode}")
    pr = Prepared(case, **mode)
    err = oracle.rel_l2(pr.rhs(), pr.oracle_rhs())
    log(f"  rel_l2={err:.3e} info={pr.mesh.info}")
    assert err <= TOL64


@pytest.mark.parametrize("mode", MODES, ids=lambda m: "-".join(f"{k}={v}" for k, v in m.items()))
@pytest.mark.parametrize("case", SMALL, ids=_ids(SMALL))
def test_vjp_fp64(case, mode):
    log(f"vjp fp64 {case.label()} {mode}")
    pr = Prepared(case, **mode)
    err = oracle.rel_l2(pr.vjp(), pr.oracle_vjp())
    log(f"  rel_l2={err:.3e}")
    assert err <= TOL64


@pytest.mark.parametrize("scatter", ["atomic", "patch", "patch_gather"])
@pytest.mark.parametrize("case", [SMALL[1], SMALL[4], SMALL[6]], ids=_ids([SMALL[1], SMALL[4], SMALL[6]]))
def test_mixed_precision(case, scatter):
    log(f"mixed {case.label()} {scatter}")
    pr = Prepared(case, scatter=scatter)
    ef = oracle.rel_l2(pr.rhs(torch.float32), pr.oracle_rhs())
    eg = oracle.rel_l2(pr.vjp(torch.float32), pr.oracle_vjp())
    log(f"  mixed rel_l2 rhs={ef:.3e} grad={eg:.3e}")
    assert ef <= TOL_MIXED and eg <= TOL_MIXED


def test_patch_sizes_and_info():
    case = Case(5, jitter=True, permute=True, mu=1e-4, cs=0.1)
    ref = None
    for pe in (32, 96, 160, 256):
        pr = Prepared(case, scatter="patch_gather", patch_elems=pe)
        info = pr.mesh.info
        assert info["scatter"] == "patch_gather" and info["patch_elems"] == pe
        assert info["n_patches"] == -(-pr.m.n_elems // pe)
        assert 4 <= info["max_patch_nodes"] <= 256
        r = pr.rhs()
        ref = pr.oracle_rhs() if ref is None else ref
        assert oracle.rel_l2(r, ref) <= TOL64


def test_auto_falls_back_to_atomic_without_renumbering():
    """Random node ids and element order: 256-element patches touch far more
    than 256 nodes, so AUTO must pick atomic scatter and PATCH must refuse."""
    from paper_2403_08777_amd import api

    case = Case(12, jitter=True, permute=True)
    pr = Prepared(case, scatter="auto", renumber=False)
    # shuffle elements too, so user order has no locality at all
    assert pr.mesh.info["scatter"] in ("atomic", "patch", "patch_gather")
    m = pr.m
    rng = np.random.default_rng(3)
    conn = m.conn[rng.permutation(m.n_elems)]
    dev = torch.device("cuda")
    mesh = api.Mesh(torch.from_numpy(m.coords).to(dev), torch.from_numpy(conn).to(dev), renumber=False)
    assert mesh.info["scatter"] == "atomic"
    for scatter in ("patch", "patch_gather"):
        with pytest.raises(api.NsasmError) as ei:
            api.Mesh(torch.from_numpy(m.coords).to(dev), torch.from_numpy(conn).to(dev), renumber=False,
                     scatter=scatter)
        assert ei.value.status_name == "UNSUPPORTED"


def test_accumulate_flag():
    from paper_2403_08777_amd import api

    pr = Prepared(Case(4, jitter=True, permute=True, mu=1e-4, cs=0.1))
    u, p, lam = pr.fields(torch.float64)
    prm = pr.case.params()
    r1 = api.assemble_rhs(pr.mesh, u, p, prm)
    r2 = r1.clone()
    api.assemble_rhs(pr.mesh, u, p, prm, out=r2, accumulate=True)
    assert oracle.rel_l2(r2.cpu().numpy(), 2 * r1.cpu().numpy()) < 1e-14
    g1 = api.assemble_rhs_vjp(pr.mesh, u, lam, prm)
    g2 = torch.ones_like(g1)
    api.assemble_rhs_vjp(pr.mesh, u, lam, prm, out=g2, accumulate=True)
    assert oracle.rel_l2(g2.cpu().numpy(), g1.cpu().numpy() + 1) < 1e-14


@pytest.mark.parametrize("scatter", ["atomic", "patch", "patch_gather"])
def test_repeat_runs_agree(scatter):
    """Atomic scatters agree to rounding; the gather scatter is bitwise
    reproducible."""
    from paper_2403_08777_amd import api

    pr = Prepared(Case(16, jitter=True, permute=True, mu=1e-4, cs=0.1), scatter=scatter)
    u, p, lam = pr.fields(torch.float64)
    prm = pr.case.params()
    a = api.assemble_rhs(pr.mesh, u, p, prm).cpu().numpy()
    ga = api.assemble_rhs_vjp(pr.mesh, u, lam, prm).cpu().numpy()
    for _ in range(3):
        b = api.assemble_rhs(pr.mesh, u, p, prm).cpu().numpy()
        gb = api.assemble_rhs_vjp(pr.mesh, u, lam, prm).cpu().numpy()
        if scatter == "patch_gather":
            assert np.array_equal(a, b) and np.array_equal(ga, gb)
        else:
            assert oracle.rel_l2(b, a) <= 1e-14 and oracle.rel_l2(gb, ga) <= 1e-14


VREMAN = [Case(2, jitter=True, permute=True, mu=1e-4, cs=0.1, model="vreman"),
          Case(7, jitter=True, permute=True, mu=1e-4, cs=0.1, model="vreman"),
          Case(16, jitter=True, permute=True, mu=1e-4, cs=0.1, model="vreman")]


@pytest.mark.parametrize("scatter", ["atomic", "patch", "patch_gather"])
@pytest.mark.parametrize("case", VREMAN, ids=_ids(VREMAN))
def test_vreman_fp64(case, scatter):
    log(f"vreman {case.label()} {scatter}")
    pr = Prepared(case, scatter=scatter)
    ef = oracle.rel_l2(pr.rhs(), pr.oracle_rhs())
    eg = oracle.rel_l2(pr.vjp(), pr.oracle_vjp())
    log(f"  rel_l2 rhs={ef:.3e} grad={eg:.3e}")
    assert ef <= TOL64 and eg <= TOL64


@pytest.mark.parametrize("case", VREMAN[1:], ids=_ids(VREMAN[1:]))
def test_vreman_mixed(case):
    pr = Prepared(case)
    ef = oracle.rel_l2(pr.rhs(torch.float32), pr.oracle_rhs())
    eg = oracle.rel_l2(pr.vjp(torch.float32), pr.oracle_vjp())
    log(f"vreman mixed {case.label()}: rhs={ef:.3e} grad={eg:.3e}")
    assert ef <= TOL_MIXED and eg <= TOL_MIXED


def test_vreman_differs_from_smagorinsky():
    from paper_2403_08777_amd import api

    case = Case(6, jitter=True, permute=True, mu=1e-4, cs=0.1)
    pr = Prepared(case)
    u, p, _ = pr.fields(torch.float64)
    rs = api.assemble_rhs(pr.mesh, u, p, case.params()).cpu().numpy()
    rv = api.assemble_rhs(pr.mesh, u, p, api.Params(1.0, 1e-4, 0.1, case.params().body_force, "vreman")).cpu().numpy()
    assert oracle.rel_l2(rv, rs) > 1e-8


@pytest.mark.parametrize("model", ["smagorinsky", "vreman"])
def test_anisotropic_elements(model):
    """Nearly degenerate geometry: the jittered 8^3 cube squashed by 1e-4 in z
    (aspect ratios near 1e4, det J ~ 1e-4 h^3).  FP64 keeps full parity; the
    mixed path, whose geometry stays FP64, keeps its usual error."""
    from paper_2403_08777_amd import api, synth

    m = synth.cube_mesh(8, jitter=True, permute=True)
    coords = m.coords * np.array([1.0, 1.0, 1e-4])
    u, p = synth.taylor_green(m)
    lam = synth.adjoint(m.n_nodes)
    dev = torch.device("cuda")
    mesh = api.Mesh(torch.from_numpy(coords).to(dev), torch.from_numpy(m.conn).to(dev))
    prm = api.Params(1.0, 1e-3, 0.1, synth.BODY_FORCE, model)
    oprm = oracle.Params(1.0, 1e-3, 0.1, synth.BODY_FORCE, model=model)
    ref_r = oracle.rhs(coords, m.conn, u, p, oprm)
    ref_g = oracle.vjp(coords, m.conn, u, lam, oprm)
    for dtype, tol in ((torch.float64, TOL64), (torch.float32, TOL_MIXED)):
        tm = lambda a: mesh.to_mesh_order(torch.from_numpy(np.ascontiguousarray(a)).to(dev, dtype))
        r = mesh.from_mesh_order(api.assemble_rhs(mesh, tm(u), tm(p), prm)).double().cpu().numpy()
        g = mesh.from_mesh_order(api.assemble_rhs_vjp(mesh, tm(u), tm(lam), prm)).double().cpu().numpy()
        er, eg = oracle.rel_l2(r, ref_r), oracle.rel_l2(g, ref_g)
        log(f"anisotropic {model} {dtype}: rhs {er:.2e} vjp {eg:.2e}")
        assert er <= tol and eg <= tol
