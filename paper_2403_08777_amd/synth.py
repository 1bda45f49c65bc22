"""Seeded synthetic tetrahedral meshes and nodal fields.

This module only builds inputs: a structured cube lattice split into linear
tetrahedra, optional interior jitter and node relabelling, a Taylor-Green
velocity with uniform noise, a pressure field and an adjoint vector.  It holds
none of the assembly arithmetic, so that the CPU oracle and the GPU library can
both be fed from it without sharing any of the method.

The paper measures on an unstructured LES mesh of the Bolund cliff (5.6 M
nodes, 32 M linear tetrahedra; Sec. III-A), which is not available.  The cubes
below stand in for it: at 160^3 cells they hold 24.6 M tetrahedra with the same
elements-per-node ratio (about 5.9), jitter and a random node numbering stand
in for unstructured geometry and ordering, and a noisy Taylor-Green vortex
stands in for the LES velocity.

Recipe (every array is int32 / float64):

* lattice node (i, j, k), 0 <= i, j, k <= N, lattice id L = i + (N+1)(j + (N+1)k),
  position (i, j, k) / N;
* cells in the same order (i fastest); each cell is cut into the 6 tetrahedra of
  the Kuhn (Freudenthal) split along its (0,0,0)-(1,1,1) diagonal, one per
  permutation s of the axes in lexicographic order, with vertices
  (v, v + e_s0, v + e_s0 + e_s1, v + (1,1,1));
* jitter: interior nodes, in increasing L, move by U(-0.2h, 0.2h) per coordinate
  drawn from ``default_rng(1)``;
* relabelling: ``perm = default_rng(2).permutation(Nn)``; lattice node L gets user
  id perm[L]; element order is unchanged;
* velocity: (sin 2pi x cos 2pi y cos 2pi z, -cos 2pi x sin 2pi y cos 2pi z, 0) plus
  U(-1e-2, 1e-2) noise per node and component from ``default_rng(3)`` (drawn in
  lattice order); pressure: sin 2pi x cos 2pi y;
* adjoint: ``default_rng(4).standard_normal((Nn, 3))`` in user order.

An unstructured mesh (``delaunay_mesh``) complements the cubes: the Delaunay
tetrahedralisation (scipy's Qhull) of P points drawn uniformly in the unit cube
by ``default_rng(seed)``, with nodes in drawing order.  Its node valence varies
(4 to about 120, mean 27) and its worst elements are slivers, so it probes the
mesh preprocessing and the patch layout on irregular topology; fields on it
use ``unstructured_fields``.
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

# The six axis permutations in lexicographic order; one tetrahedron each.
_KUHN_PERMS = tuple(itertools.permutations(range(3)))

BODY_FORCE = (0.1, -0.2, 0.3)


@dataclass
class SynthMesh:
    """A cube mesh in user numbering.  ``coords``: (Nn, 3) float64;
    ``conn``: (Ne, 4) int32; ``perm``: user id of each lattice node (or None
    when the natural numbering is kept); ``lattice_xyz``: the (jittered)
    positions in lattice order."""

    n: int
    coords: np.ndarray
    conn: np.ndarray
    perm: np.ndarray | None
    lattice_xyz: np.ndarray
    jitter: bool
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return self.coords.shape[0]

    @property
    def n_elems(self) -> int:
        return self.conn.shape[0]

    def to_user(self, lattice_values: np.ndarray) -> np.ndarray:
        """Reorder a per-node array from lattice order into user order."""
        if self.perm is None:
            return np.ascontiguousarray(lattice_values)
        out = np.empty_like(lattice_values)
        out[self.perm] = lattice_values
        return out


def lattice_conn(n: int) -> np.ndarray:
    """Kuhn split of an n^3 cell lattice, in lattice node ids, shape (6 n^3, 4)."""
    n1 = n + 1
    ci, cj, ck = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    # cell order: i fastest, then j, then k
    base = (ci + n1 * (cj + n1 * ck)).transpose(2, 1, 0).reshape(-1).astype(np.int64)
    step = np.array([1, n1, n1 * n1], dtype=np.int64)
    tets = []
    for s in _KUHN_PERMS:
        o1 = step[s[0]]
        o2 = o1 + step[s[1]]
        o3 = step.sum()
        tets.append(np.stack([base, base + o1, base + o2, base + o3], axis=1))
    # element index = 6 * cell + permutation index
    conn = np.stack(tets, axis=1).reshape(-1, 4)
    return conn.astype(np.int32)


def lattice_coords(n: int, jitter: bool) -> np.ndarray:
    """Node positions in lattice order, shape ((n+1)^3, 3)."""
    n1 = n + 1
    k, j, i = np.meshgrid(np.arange(n1), np.arange(n1), np.arange(n1), indexing="ij")
    xyz = np.stack([i.reshape(-1), j.reshape(-1), k.reshape(-1)], axis=1).astype(np.float64)
    interior = np.all((xyz > 0) & (xyz < n), axis=1)
    xyz /= n
    if jitter:
        h = 1.0 / n
        idx = np.nonzero(interior)[0]
        rng = np.random.default_rng(1)
        xyz[idx] += rng.uniform(-0.2 * h, 0.2 * h, (idx.size, 3))
    return xyz


def cube_mesh(n: int, jitter: bool = False, permute: bool = False) -> SynthMesh:
    """The n^3-cell unit cube of the recipe above."""
    if n < 1:
        raise ValueError("n must be >= 1")
    xyz = lattice_coords(n, jitter)
    conn_l = lattice_conn(n)
    nn = xyz.shape[0]
    if permute:
        perm = np.random.default_rng(2).permutation(nn).astype(np.int32)
        coords = np.empty_like(xyz)
        coords[perm] = xyz
        conn = perm[conn_l]
    else:
        perm = None
        coords = xyz.copy()
        conn = conn_l
    return SynthMesh(n=n, coords=np.ascontiguousarray(coords), conn=np.ascontiguousarray(conn),
                     perm=perm, lattice_xyz=xyz, jitter=jitter)


def taylor_green(mesh: SynthMesh, noise: bool = True):
    """Velocity (Nn, 3) and pressure (Nn,) in user order."""
    x, y, z = (mesh.lattice_xyz[:, c] for c in range(3))
    tp = 2.0 * np.pi
    u = np.stack([np.sin(tp * x) * np.cos(tp * y) * np.cos(tp * z),
                  -np.cos(tp * x) * np.sin(tp * y) * np.cos(tp * z),
                  np.zeros_like(x)], axis=1)
    if noise:
        u += np.random.default_rng(3).uniform(-1e-2, 1e-2, u.shape)
    p = np.sin(tp * x) * np.cos(tp * y)
    return mesh.to_user(u), mesh.to_user(p)


def adjoint(n_nodes: int) -> np.ndarray:
    """Seeded standard-normal adjoint vector (Nn, 3), user order."""
    return np.random.default_rng(4).standard_normal((n_nodes, 3))


def delaunay_mesh(n_points: int, seed: int = 1):
    """Delaunay tetrahedralisation of n_points uniform points in the unit
    cube: coords (n_points, 3) float64 and conn (Ne, 4) int32."""
    if n_points < 5:
        raise ValueError("n_points must be >= 5")
    from scipy.spatial import Delaunay

    pts = np.random.default_rng(seed).random((n_points, 3))
    return pts, np.ascontiguousarray(Delaunay(pts).simplices.astype(np.int32))


def unstructured_fields(coords: np.ndarray, seed: int = 2):
    """Fields on an arbitrary node set, drawn in this order from
    ``default_rng(seed)``: velocity u (the smooth field (sin 3y, cos 2z, xy)
    plus normal noise of standard deviation 0.1), then standard-normal
    pressure p, adjoint lambda, velocity tangent du and pressure tangent dp."""
    rng = np.random.default_rng(seed)
    x, y, z = (coords[:, c] for c in range(3))
    u = np.stack([np.sin(3.0 * y), np.cos(2.0 * z), x * y], axis=1) + 0.1 * rng.standard_normal(coords.shape)
    p = rng.standard_normal(coords.shape[0])
    lam = rng.standard_normal(coords.shape)
    du = rng.standard_normal(coords.shape)
    dp = rng.standard_normal(coords.shape[0])
    return u, p, lam, du, dp


@dataclass(frozen=True)
class Workload:
    """One of the synthetic cases: mesh recipe plus physical parameters."""

    name: str
    n: int
    jitter: bool
    permute: bool
    mu: float
    cs: float
    rho: float = 1.0
    body_force: tuple = BODY_FORCE


WORKLOADS = {
    # 16^3 cube, natural numbering, FP64 forward (also the FD-gradient mesh)
    "cube16": Workload("cube16", 16, False, False, 1e-3, 0.0),
    # 96^3 cube, relabelled nodes, FP64 forward
    "cube96_perm": Workload("cube96_perm", 96, False, True, 1e-3, 0.0),
    # 160^3 cube, jitter + relabelling, Smagorinsky 0.1, FP64 forward
    "cube160_jit_perm_smag": Workload("cube160_jit_perm_smag", 160, True, True, 1e-4, 0.1),
    # 96^3 cube, jitter + relabelling, FP64 forward + velocity VJP
    "cube96_jit_perm": Workload("cube96_jit_perm", 96, True, True, 1e-3, 0.0),
}


def build(workload: Workload):
    """Mesh, u, p and adjoint for a workload (all numpy, user order)."""
    mesh = cube_mesh(workload.n, workload.jitter, workload.permute)
    u, p = taylor_green(mesh)
    lam = adjoint(mesh.n_nodes)
    return mesh, u, p, lam
