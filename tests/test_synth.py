"""Synthetic mesh/field generator: sizes, validity, seeds."""

import numpy as np
import pytest

from paper_2403_08777_amd import synth


@pytest.mark.parametrize("n", [1, 2, 5])
def test_counts(n):
    m = synth.cube_mesh(n)
    assert m.n_nodes == (n + 1) ** 3
    assert m.n_elems == 6 * n ** 3
    assert m.conn.dtype == np.int32 and m.coords.dtype == np.float64
    assert m.conn.min() == 0 and m.conn.max() == m.n_nodes - 1


def _signed_volumes(coords, conn):
    d1 = coords[conn[:, 1]] - coords[conn[:, 0]]
    d2 = coords[conn[:, 2]] - coords[conn[:, 0]]
    d3 = coords[conn[:, 3]] - coords[conn[:, 0]]
    return np.einsum("ij,ij->i", d1, np.cross(d2, d3)) / 6.0


@pytest.mark.parametrize("n,jitter", [(4, False), (4, True), (7, True)])
def test_volume_and_no_inversion(n, jitter):
    m = synth.cube_mesh(n, jitter=jitter)
    ref = synth.cube_mesh(n)
    v = _signed_volumes(m.coords, m.conn)
    v0 = _signed_volumes(ref.coords, ref.conn)
    assert abs(np.abs(v).sum() - 1.0) < 1e-12
    # jitter keeps each tetrahedron's orientation (no inversion)
    assert np.all(np.sign(v) == np.sign(v0))
    assert np.abs(v).min() * 6 * n ** 3 > 0.1


def test_conforming_faces():
    m = synth.cube_mesh(3)
    faces = {}
    for tet in m.conn:
        for drop in range(4):
            f = tuple(sorted(np.delete(tet, drop)))
            faces[f] = faces.get(f, 0) + 1
    counts = np.array(list(faces.values()))
    assert counts.max() == 2
    # boundary faces: 2 triangles per cell face on the 6 cube faces
    assert np.sum(counts == 1) == 6 * 2 * 3 * 3


def test_permutation_and_seeds():
    a = synth.cube_mesh(4, jitter=True, permute=True)
    b = synth.cube_mesh(4, jitter=True, permute=True)
    assert np.array_equal(a.coords, b.coords) and np.array_equal(a.conn, b.conn)
    assert np.array_equal(np.sort(a.perm), np.arange(a.n_nodes))
    nat = synth.cube_mesh(4, jitter=True)
    np.testing.assert_array_equal(a.coords[a.perm], nat.coords)
    np.testing.assert_array_equal(a.conn, a.perm[nat.conn])
    ua, pa = synth.taylor_green(a)
    un, pn = synth.taylor_green(nat)
    np.testing.assert_array_equal(ua[a.perm], un)
    np.testing.assert_array_equal(pa[a.perm], pn)


def test_fields_shape_and_noise_amplitude():
    m = synth.cube_mesh(8)
    u, p = synth.taylor_green(m)
    u0, _ = synth.taylor_green(m, noise=False)
    assert u.shape == (m.n_nodes, 3) and p.shape == (m.n_nodes,)
    assert 0.009 < np.abs(u - u0).max() <= 0.01
    lam = synth.adjoint(m.n_nodes)
    assert lam.shape == (m.n_nodes, 3)
    assert abs(lam.std() - 1.0) < 0.1


def test_workloads_sizes():
    w = synth.WORKLOADS
    assert 6 * w["cube96_jit_perm"].n ** 3 == 5_308_416
    assert 6 * w["cube160_jit_perm_smag"].n ** 3 == 24_576_000
    assert (w["cube160_jit_perm_smag"].n + 1) ** 3 == 4_173_281


def test_delaunay_mesh_and_fields():
    coords, conn = synth.delaunay_mesh(500, seed=3)
    assert coords.shape == (500, 3) and coords.dtype == np.float64
    assert conn.dtype == np.int32 and conn.ndim == 2 and conn.shape[1] == 4 and conn.shape[0] > 500
    assert conn.min() >= 0 and conn.max() < 500
    assert all(len(set(row)) == 4 for row in conn.tolist())
    d = coords[conn[:, 1:]] - coords[conn[:, :1]]
    vol = np.abs(np.einsum("ij,ij->i", d[:, 0], np.cross(d[:, 1], d[:, 2]))) / 6.0
    # a tetrahedralisation of the points' convex hull: positive volumes that
    # add up to the hull's volume
    from scipy.spatial import ConvexHull

    assert vol.min() > 0.0 and abs(vol.sum() - ConvexHull(coords).volume) < 1e-12
    c2, k2 = synth.delaunay_mesh(500, seed=3)
    assert np.array_equal(coords, c2) and np.array_equal(conn, k2)
    u, p, lam, du, dp = synth.unstructured_fields(coords, seed=5)
    assert u.shape == lam.shape == du.shape == (500, 3) and p.shape == dp.shape == (500,)
    assert np.array_equal(u, synth.unstructured_fields(coords, seed=5)[0])
    with pytest.raises(ValueError):
        synth.delaunay_mesh(4)
