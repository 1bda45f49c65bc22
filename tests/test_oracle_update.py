"""Pins of the oracle's explicit-update epilogue: the lumped volume against
the textbook consistent mass matrix and the lattice, the update against the
body-force closed form, and the Dirichlet mask.  CPU only."""

import numpy as np
import pytest

import oracle
from paper_2403_08777_amd import synth
from tests.test_oracle_pins import consistent_mass


@pytest.mark.parametrize("jitter", [False, True])
def test_lumped_volume_is_consistent_mass_row_sum(oracle_lib, jitter):
    """Row-sum lumping: sum_b M_ab = V (2 + 3)/20 = V/4 per element, so V^L is
    the row sum of the consistent mass matrix (textbook M^e_ab = V(1+d_ab)/20
    with numpy determinants), and the V^L sum to the domain volume."""
    m = synth.cube_mesh(4, jitter=jitter, permute=True)
    vl = oracle.lumped_volume(m.coords, m.conn)
    np.testing.assert_allclose(vl, consistent_mass(m.coords, m.conn).sum(1), rtol=1e-14)
    assert abs(vl.sum() - 1.0) < 1e-14


def test_lumped_volume_on_lattice(oracle_lib):
    """Unjittered Kuhn mesh: an interior node is shared by 24 tetrahedra of
    volume h^3/6, so V^L = h^3; the cube corners (0,0,0) and (1,1,1) lie in all
    6 tetrahedra of their cell (h^3/4), the other six corners in 2 (h^3/12)."""
    n = 5
    h = 1.0 / n
    m = synth.cube_mesh(n)
    vl = oracle.lumped_volume(m.coords, m.conn)
    interior = np.all((m.coords > 1e-12) & (m.coords < 1 - 1e-12), axis=1)
    np.testing.assert_allclose(vl[interior], h ** 3, rtol=1e-13)
    corner = np.all((m.coords < 1e-12) | (m.coords > 1 - 1e-12), axis=1)
    diag = corner & (np.abs(m.coords[:, 0] - m.coords[:, 1]) < 1e-12) & (np.abs(m.coords[:, 1] - m.coords[:, 2]) < 1e-12)
    np.testing.assert_allclose(vl[diag], h ** 3 / 4, rtol=1e-13)
    np.testing.assert_allclose(vl[corner & ~diag], h ** 3 / 12, rtol=1e-13)
    assert diag.sum() == 2 and (corner & ~diag).sum() == 6


def test_update_body_force_closed_form(oracle_lib):
    """u = 0, p = 0: the only non-zero term is the body force, R_n = rho f V^L_n
    (row-sum of the consistent mass times constant f), so one explicit stage
    gives u_new = dt f at every node, whatever rho, mu and the mesh."""
    m = synth.cube_mesh(4, jitter=True, permute=True)
    f = np.array([0.7, -1.1, 0.4])
    prm = oracle.Params(1.7, 3e-3, 0.1, f)
    un, R = oracle.explicit_update(m.coords, m.conn, np.zeros((m.n_nodes, 3)), np.zeros(m.n_nodes), prm, 0.25)
    np.testing.assert_allclose(un, np.tile(0.25 * f, (m.n_nodes, 1)), rtol=1e-13, atol=0)


def test_update_mask_and_linearity(oracle_lib):
    """Masked components keep u bit for bit; free components move by
    dt R / (rho V^L), so u_new - u is exactly linear in dt."""
    m = synth.cube_mesh(4, jitter=True, permute=True)
    u, p = synth.taylor_green(m)
    prm = oracle.Params(1.3, 1e-3, 0.1, synth.BODY_FORCE, model="vreman", form="skew")
    mask = np.random.default_rng(3).integers(0, 8, m.n_nodes).astype(np.uint8)
    u1, R = oracle.explicit_update(m.coords, m.conn, u, p, prm, 1e-2, mask)
    fixed = np.stack([(mask >> i) & 1 for i in range(3)], axis=1).astype(bool)
    assert np.array_equal(u1[fixed], u[fixed])
    u2, _ = oracle.explicit_update(m.coords, m.conn, u, p, prm, 2e-2, mask)
    np.testing.assert_allclose((u2 - u)[~fixed], 2 * (u1 - u)[~fixed], rtol=1e-12, atol=1e-17)
    # the free increment times the lumped mass gives R back
    vl = oracle.lumped_volume(m.coords, m.conn)
    inc = (u1 - u) * (prm.rho * vl)[:, None] / 1e-2
    np.testing.assert_allclose(inc[~fixed], R[~fixed], rtol=1e-10, atol=1e-14)


def test_update_leaves_unreferenced_nodes_unchanged(oracle_lib):
    """A node that no element references has V^L = 0 and R = 0: the stage
    leaves it unchanged (u_new = u, finite) instead of producing 0/0, and the
    referenced nodes are updated exactly as on the mesh without the extra
    nodes."""
    m = synth.cube_mesh(3, jitter=True, permute=True)
    u, p = synth.taylor_green(m)
    extra = 5
    rng = np.random.default_rng(11)
    coords = np.vstack([m.coords, rng.uniform(2.0, 3.0, (extra, 3))])
    u2 = np.vstack([u, rng.uniform(-1.0, 1.0, (extra, 3))])
    p2 = np.concatenate([p, rng.uniform(-1.0, 1.0, extra)])
    prm = oracle.Params(1.0, 1e-3, 0.1, synth.BODY_FORCE)
    un, R = oracle.explicit_update(coords, m.conn, u2, p2, prm, 1e-2)
    assert np.isfinite(un).all()
    assert np.array_equal(un[-extra:], u2[-extra:]) and np.array_equal(R[-extra:], np.zeros((extra, 3)))
    ref, _ = oracle.explicit_update(m.coords, m.conn, u, p, prm, 1e-2)
    assert np.array_equal(un[:-extra], ref)
