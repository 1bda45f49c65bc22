"""The stored exact result tests/golden/cube2_exact.txt (exact Galerkin
integrals of the momentum RHS and its derivatives on a skewed, relabelled
2^3 Kuhn cube; how it was made is in tests/golden/make_cube2_exact.py).
The exact checker must reproduce it bit for bit, and the FP64 C oracle must
match it to rounding.  CPU only."""

import numpy as np

import oracle
from tests.golden.make_cube2_exact import compute, load

G = load()


def as_np(rows):
    return np.array([[float(v) for v in r] if isinstance(r, list) else float(r) for r in rows])


def test_fixture_shape():
    assert len(G["conn"]) == G["n_elems"] == 48
    assert len(G["x"]) == 27
    # every node is used and every element is positively or negatively oriented but not flat
    assert sorted({n for tet in G["conn"] for n in tet}) == list(range(27))
    x = as_np(G["x"])
    for tet in G["conn"]:
        assert abs(np.linalg.det(x[tet[1:]] - x[tet[0]])) > 1e-3


def test_exact_checker_reproduces_fixture():
    out = compute(G["x"], G["conn"], G["u"], G["p"], G["lam"], G["du"], G["dp"])
    for name, rows in out.items():
        assert rows == G[name], name


def test_c_oracle_matches_fixture(oracle_lib):
    x, conn = as_np(G["x"]), np.array(G["conn"], dtype=np.int32)
    u, p, lam, du, dp = (as_np(G[k]) for k in ("u", "p", "lam", "du", "dp"))
    prm = oracle.Params(float(G["rho"]), float(G["mu"]), 0.0, [float(v) for v in G["f"]])
    emac = oracle.Params(float(G["rho"]), float(G["mu"]), 0.0, [float(v) for v in G["f"]], form="emac")
    got = {
        "rhs": oracle.rhs(x, conn, u, p, prm),
        "rhs_emac": oracle.rhs(x, conn, u, p, emac),
        "vjp": oracle.vjp(x, conn, u, lam, prm),
        "vjp_p": oracle.vjp_p(x, conn, lam),
        "jvp": oracle.jvp(x, conn, u, p, du, dp, prm),
    }
    for name, val in got.items():
        assert oracle.rel_l2(val, as_np(G[name])) < 1e-14, name
