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


def test_anisotropic_elements_smagorinsky():
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
    prm = api.Params(1.0, 1e-3, 0.1, synth.BODY_FORCE)
    oprm = oracle.Params(1.0, 1e-3, 0.1, synth.BODY_FORCE)
    ref_r = oracle.rhs(coords, m.conn, u, p, oprm)
    ref_g = oracle.vjp(coords, m.conn, u, lam, oprm)
    for dtype, tol in ((torch.float64, TOL64), (torch.float32, TOL_MIXED)):
        tm = lambda a: mesh.to_mesh_order(torch.from_numpy(np.ascontiguousarray(a)).to(dev, dtype))
        r = mesh.from_mesh_order(api.assemble_rhs(mesh, tm(u), tm(p), prm)).double().cpu().numpy()
        g = mesh.from_mesh_order(api.assemble_rhs_vjp(mesh, tm(u), tm(lam), prm)).double().cpu().numpy()
        er, eg = oracle.rel_l2(r, ref_r), oracle.rel_l2(g, ref_g)
        log(f"anisotropic smagorinsky {dtype}: rhs {er:.2e} vjp {eg:.2e}")
        assert er <= tol and eg <= tol


@pytest.mark.parametrize("model", ["smagorinsky", "vreman"])
@pytest.mark.parametrize("scale", [2.0 ** -200, 2.0 ** -60, 2.0 ** 60, 2.0 ** 200], ids=["2^-200", "2^-60", "2^60", "2^200"])
def test_eddy_model_at_extreme_length_scales(model, scale):
    """The jittered, relabelled 6^3 cube with its coordinates scaled by L, no
    molecular viscosity, no body force and a model constant of 1, so that
    every term of the RHS scales as L^2 and the eddy viscosity (about
    c V^(2/3) |grad u| ~ L) makes about 60 % of it.  V ~ L^3 and
    |S|^2 ~ L^-2 then lie far outside the single-precision range in which
    the FP64 kernels estimate V^(-1/3) and 1/|S| before refining them, so
    this checks their rescaling by exact powers of two.  FP64 forward and
    VJP against the oracle."""
    from paper_2403_08777_amd import api, synth

    m = synth.cube_mesh(6, jitter=True, permute=True)
    coords = m.coords * scale
    u, p = synth.taylor_green(m)
    lam = synth.adjoint(m.n_nodes)
    dev = torch.device("cuda")
    mesh = api.Mesh(torch.from_numpy(coords).to(dev), torch.from_numpy(m.conn).to(dev))
    prm = api.Params(1.0, 0.0, 1.0, (0.0, 0.0, 0.0), model)
    oprm = oracle.Params(1.0, 0.0, 1.0, (0.0, 0.0, 0.0), model=model)
    tm = lambda a: mesh.to_mesh_order(torch.from_numpy(np.ascontiguousarray(a)).to(dev))
    r = mesh.from_mesh_order(api.assemble_rhs(mesh, tm(u), tm(p), prm)).cpu().numpy()
    g = mesh.from_mesh_order(api.assemble_rhs_vjp(mesh, tm(u), tm(lam), prm)).cpu().numpy()
    er = oracle.rel_l2(r, oracle.rhs(coords, m.conn, u, p, oprm))
    eg = oracle.rel_l2(g, oracle.vjp(coords, m.conn, u, lam, oprm))
    log(f"{model} at L={scale:.3g}: rhs {er:.2e} vjp {eg:.2e}")
    assert er <= TOL64 and eg <= TOL64
    mesh.close()


def _vreman_exact_mu(xf, conn, uf, rho, mu, cs):
    """Per-element mu + mu_t(Vreman) to ~40 digits: exact rational geometry and
    velocity gradient, B and alpha:alpha as exact rationals, the roots in
    50-digit decimals."""
    from decimal import Decimal, getcontext
    from fractions import Fraction

    from oracle import exact

    getcontext().prec = 50
    out = []
    for tet in conn:
        xe = [[Fraction(float(v)) for v in xf[n]] for n in tet]
        vol, gn = exact.element_geometry(xe)
        ue = [[Fraction(float(v)) for v in uf[n]] for n in tet]
        G = [[sum(ue[a][i] * gn[a][j] for a in range(4)) for j in range(3)] for i in range(3)]
        P = [[sum(G[i][k] * G[j][k] for k in range(3)) for j in range(3)] for i in range(3)]
        A = P[0][0] + P[1][1] + P[2][2]
        B = (P[0][0] * P[1][1] - P[0][1] ** 2 + P[0][0] * P[2][2] - P[0][2] ** 2 + P[1][1] * P[2][2]
             - P[1][2] ** 2)
        dec = lambda q: Decimal(q.numerator) / Decimal(q.denominator)
        delta2 = (dec(vol) ** (Decimal(1) / Decimal(3))) ** 2
        # Vreman's B_beta = Delta^4 e2(P) and alpha:alpha = A, so nu_t = c Delta^2 sqrt(e2(P) / A)
        s = (dec(B) / dec(A)).sqrt() if A > 0 and B > 0 else Decimal(0)
        mut = Decimal(rho) * Decimal(2.5) * Decimal(cs) ** 2 * delta2 * s
        out.append(Fraction(Decimal(mu) + mut))
    return out


def test_anisotropic_elements_vreman():
    """Vreman's B is a sum of 2x2 minors of P = G G^T.  On elements squashed by
    1e-4 the velocity gradient is nearly rank one and B cancels to 1e-6..1e-11
    of its terms, so FP64 evaluations that differ only in rounding (FMA
    contraction, operation order) differ by far more than 1e-12.  Both the
    kernel and the oracle are therefore compared with a high-precision
    reference (exact rational assembly with the per-element viscosity to 40
    digits) on a 4^3 squashed mesh: the kernel must be as close to it as the
    FP64 oracle, within a factor of 10."""
    from fractions import Fraction

    from oracle import exact
    from paper_2403_08777_amd import api, synth

    m = synth.cube_mesh(4, jitter=True, permute=True)
    coords = m.coords * np.array([1.0, 1.0, 1e-4])
    u, p = synth.taylor_green(m)
    rho, mu, cs = 1.0, 1e-3, 0.1
    mu_elem = _vreman_exact_mu(coords, m.conn, u, rho, mu, cs)
    fq = [Fraction(float(v)) for v in synth.BODY_FORCE]
    cq = [[Fraction(float(v)) for v in row] for row in coords]
    uq = [[Fraction(float(v)) for v in row] for row in u]
    pq = [Fraction(float(v)) for v in p]
    ref = np.array([[float(v) for v in row] for row in
                    exact.assemble_rhs(cq, m.conn, uq, pq, Fraction(rho), Fraction(mu), fq, mu_elem)])
    ora = oracle.rhs(coords, m.conn, u, p, oracle.Params(rho, mu, cs, synth.BODY_FORCE, model="vreman"))
    dev = torch.device("cuda")
    mesh = api.Mesh(torch.from_numpy(coords).to(dev), torch.from_numpy(m.conn).to(dev))
    tm = lambda a: mesh.to_mesh_order(torch.from_numpy(np.ascontiguousarray(a)).to(dev))
    got = mesh.from_mesh_order(api.assemble_rhs(mesh, tm(u), tm(p), api.Params(rho, mu, cs, synth.BODY_FORCE,
                                                                              "vreman"))).cpu().numpy()
    e_gpu, e_ora = oracle.rel_l2(got, ref), oracle.rel_l2(ora, ref)
    log(f"anisotropic vreman vs high precision: kernel {e_gpu:.2e}, oracle {e_ora:.2e}")
    assert e_gpu <= max(1e-13, 10 * e_ora)
    # mixed precision: the kernel's cofactor form of B keeps FP32 meaningful here
    t32 = lambda a: mesh.to_mesh_order(torch.from_numpy(np.ascontiguousarray(a)).to(dev, torch.float32))
    got32 = mesh.from_mesh_order(api.assemble_rhs(mesh, t32(u), t32(p), api.Params(rho, mu, cs, synth.BODY_FORCE,
                                                                                  "vreman"))).double().cpu().numpy()
    e32 = oracle.rel_l2(got32, ref)
    log(f"  mixed: {e32:.2e}")
    assert e32 <= TOL_MIXED


def test_auto_halves_patches_for_a_tet_strip():
    """A strip of tetrahedra on a helix, tet k = (k, k+1, k+2, k+3): 256
    consecutive tets touch 259 nodes, 128 touch 131.  The default options
    must fall back to 128-element patches (not to atomic scatter) and keep
    FP64 parity."""
    from paper_2403_08777_amd import api, synth

    nt = 1000
    k = np.arange(nt + 3)
    ang = 2 * np.pi * k / 3.3
    coords = np.stack([0.05 * k, np.cos(ang), np.sin(ang)], axis=1)
    conn = np.stack([k[:nt], k[:nt] + 1, k[:nt] + 2, k[:nt] + 3], axis=1).astype(np.int32)
    vol, _ = oracle.geometry(coords, conn)
    assert vol.min() > 1e-3
    rng = np.random.default_rng(7)
    u = rng.standard_normal((nt + 3, 3))
    p = rng.standard_normal(nt + 3)
    dev = torch.device("cuda")
    mesh = api.Mesh(torch.from_numpy(coords).to(dev), torch.from_numpy(conn).to(dev))
    info = mesh.info
    log(f"tet strip: {info}")
    assert info["scatter"] == "patch_gather" and info["patch_elems"] == 128
    assert info["max_patch_nodes"] <= 256
    prm = api.Params(1.0, 1e-3, 0.1, synth.BODY_FORCE)
    tm = lambda a: mesh.to_mesh_order(torch.from_numpy(np.ascontiguousarray(a)).to(dev))
    got = mesh.from_mesh_order(api.assemble_rhs(mesh, tm(u), tm(p), prm)).cpu().numpy()
    ref = oracle.rhs(coords, conn, u, p, oracle.Params(1.0, 1e-3, 0.1, synth.BODY_FORCE))
    assert oracle.rel_l2(got, ref) <= TOL64
    # an explicit 256-element request cannot be served with patches
    with pytest.raises(api.NsasmError):
        api.Mesh(torch.from_numpy(coords).to(dev), torch.from_numpy(conn).to(dev), scatter="patch_gather",
                 patch_elems=256)


def _helix_strip(nt):
    """Tetrahedra on a helix, tet k = (k, k+1, k+2, k+3): nt + 3 nodes."""
    k = np.arange(nt + 3)
    ang = 2 * np.pi * k / 3.3
    coords = np.stack([0.05 * k, np.cos(ang), np.sin(ang)], axis=1)
    conn = np.stack([k[:nt], k[:nt] + 1, k[:nt] + 2, k[:nt] + 3], axis=1).astype(np.int32)
    return coords, conn


@pytest.mark.parametrize("scatter", ["patch", "patch_gather"])
def test_patch_with_the_maximum_256_nodes(scatter):
    """253 strip tetrahedra form one patch that touches exactly 256 nodes:
    every one-byte LDS position and every slot of the bank colouring is used.
    FP64 forward and VJP at parity, mixed within its bound; one tetrahedron
    more (257 nodes) makes the default fall back to 128-element patches."""
    from paper_2403_08777_amd import api, synth

    coords, conn = _helix_strip(253)
    rng = np.random.default_rng(17)
    u, p, lam = rng.standard_normal((256, 3)), rng.standard_normal(256), rng.standard_normal((256, 3))
    dev = torch.device("cuda")
    mesh = api.Mesh(torch.from_numpy(coords).to(dev), torch.from_numpy(conn).to(dev), scatter=scatter)
    info = mesh.info
    log(f"256-node patch ({scatter}): {info}")
    assert info["n_patches"] == 1 and info["max_patch_nodes"] == 256 and info["patch_elems"] == 256
    prm = api.Params(1.0, 1e-3, 0.1, synth.BODY_FORCE)
    oprm = oracle.Params(1.0, 1e-3, 0.1, synth.BODY_FORCE)
    for dtype, tol in ((torch.float64, TOL64), (torch.float32, 1e-5)):
        tm = lambda a: mesh.to_mesh_order(torch.from_numpy(np.ascontiguousarray(a)).to(dev, dtype))
        got = mesh.from_mesh_order(api.assemble_rhs(mesh, tm(u), tm(p), prm)).double().cpu().numpy()
        g = mesh.from_mesh_order(api.assemble_rhs_vjp(mesh, tm(u), tm(lam), prm)).double().cpu().numpy()
        er = oracle.rel_l2(got, oracle.rhs(coords, conn, u, p, oprm))
        eg = oracle.rel_l2(g, oracle.vjp(coords, conn, u, lam, oprm))
        log(f"  {str(dtype)[6:]}: rhs {er:.2e}, grad {eg:.2e}")
        assert er <= tol and eg <= tol
    mesh.close()
    coords, conn = _helix_strip(254)
    mesh = api.Mesh(torch.from_numpy(coords).to(dev), torch.from_numpy(conn).to(dev))
    assert mesh.info["patch_elems"] == 128 and mesh.info["max_patch_nodes"] <= 256
    mesh.close()


@pytest.mark.parametrize("scatter", ["atomic", "patch", "patch_gather"])
def test_high_valence_fan(scatter):
    """200 tetrahedra around an axis share its two end nodes: each hub's run
    holds 200 contributions in one patch (unstructured meshes have such
    nodes; the cube meshes stop at 24).  FP64 and mixed forward + VJP."""
    from paper_2403_08777_amd import api, synth

    n = 200
    ang = 2 * np.pi * np.arange(n) / n
    ring = np.stack([np.cos(ang), np.sin(ang), 0.5 + 0.1 * np.sin(3 * ang)], axis=1)
    coords = np.vstack([[0.0, 0.0, 0.0], [0.0, 0.0, 1.0], ring])
    k = np.arange(n)
    conn = np.stack([np.zeros(n, int), np.ones(n, int), 2 + k, 2 + (k + 1) % n], axis=1).astype(np.int32)
    vol, _ = oracle.geometry(coords, conn)
    assert vol.min() > 1e-4
    rng = np.random.default_rng(19)
    nn = coords.shape[0]
    u, p, lam = rng.standard_normal((nn, 3)), rng.standard_normal(nn), rng.standard_normal((nn, 3))
    dev = torch.device("cuda")
    mesh = api.Mesh(torch.from_numpy(coords).to(dev), torch.from_numpy(conn).to(dev), scatter=scatter)
    log(f"fan ({scatter}): {mesh.info}")
    prm = api.Params(1.0, 1e-2, 0.1, synth.BODY_FORCE)
    oprm = oracle.Params(1.0, 1e-2, 0.1, synth.BODY_FORCE)
    for dtype, tol in ((torch.float64, TOL64), (torch.float32, 1e-5)):
        tm = lambda a: mesh.to_mesh_order(torch.from_numpy(np.ascontiguousarray(a)).to(dev, dtype))
        got = mesh.from_mesh_order(api.assemble_rhs(mesh, tm(u), tm(p), prm)).double().cpu().numpy()
        g = mesh.from_mesh_order(api.assemble_rhs_vjp(mesh, tm(u), tm(lam), prm)).double().cpu().numpy()
        er = oracle.rel_l2(got, oracle.rhs(coords, conn, u, p, oprm))
        eg = oracle.rel_l2(g, oracle.vjp(coords, conn, u, lam, oprm))
        log(f"  {str(dtype)[6:]}: rhs {er:.2e}, grad {eg:.2e}")
        assert er <= tol and eg <= tol
    mesh.close()


def test_anisotropic_elements_vreman_vjp():
    """The Vreman VJP on the same kind of squashed elements (3^3 jittered cube,
    z scaled by 1e-4), against the 60-digit reference of tests/hp_vreman.py
    (exact frozen-viscosity VJP plus Vreman's viscosity differentiated in
    high-precision decimals): the kernel must be as close to it as the FP64
    oracle, within a factor of 10; mixed precision within its usual error."""
    from paper_2403_08777_amd import api, synth
    from tests import hp_vreman

    m = synth.cube_mesh(3, jitter=True, permute=True)
    coords = m.coords * np.array([1.0, 1.0, 1e-4])
    u, _ = synth.taylor_green(m)
    lam = synth.adjoint(m.n_nodes)
    rho, mu, cs = 1.0, 1e-3, 0.1
    log("anisotropic vreman vjp: building the 60-digit reference on the host")
    ref = hp_vreman.vjp(coords, m.conn, u, lam, rho, mu, cs, synth.BODY_FORCE)
    ora = oracle.vjp(coords, m.conn, u, lam, oracle.Params(rho, mu, cs, synth.BODY_FORCE, model="vreman"))
    dev = torch.device("cuda")
    mesh = api.Mesh(torch.from_numpy(coords).to(dev), torch.from_numpy(m.conn).to(dev))
    prm = api.Params(rho, mu, cs, synth.BODY_FORCE, "vreman")
    e_ora = oracle.rel_l2(ora, ref)
    for dtype in (torch.float64, torch.float32):
        tm = lambda a: mesh.to_mesh_order(torch.from_numpy(np.ascontiguousarray(a)).to(dev, dtype))
        got = mesh.from_mesh_order(api.assemble_rhs_vjp(mesh, tm(u), tm(lam), prm)).double().cpu().numpy()
        e_gpu = oracle.rel_l2(got, ref)
        log(f"  {dtype}: kernel {e_gpu:.2e}, oracle {e_ora:.2e}")
        if dtype == torch.float64:
            assert e_gpu <= max(1e-13, 10 * e_ora)
        else:
            assert e_gpu <= TOL_MIXED
