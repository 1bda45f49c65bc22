"""Writes and reads cube2_exact.txt, a stored exact result for the momentum
right-hand side assembly (Sec. II, P1 tetrahedra) and its derivatives.

The paper prints no worked example of an assembled residual, so the stored
values are the exact Galerkin integrals of oracle/exact.py (rational
arithmetic, closed-form integrals of products of barycentric coordinates, no
quadrature and no floating-point inverse) on a tiny mesh whose coordinates and
fields are dyadic rationals, i.e. exactly representable in FP64:

* the 2^3-cell unit cube split into 6 Kuhn tetrahedra per cell, node ids
  relabelled by the seeded permutation of the input generator, mapped by the
  dyadic affine map x -> A x + b below (every element skewed) and its one
  interior node moved by (3, -2, 1) h/16 before the map;
* u, p, lambda, du, dp: integers in [-64, 64] divided by 32 (seed 2403);
* rho = 5/4, mu = 3/1000, f = (1/10, -1/5, 3/10), no eddy viscosity.

Blocks: rhs (advective convective form), rhs_emac (the EMAC form, one of the
selectable forms for the energy-preserving scheme the introduction attributes
to Alya), vjp = (dR/du)^T lambda, vjp_p = (dR/dp)^T lambda,
jvp = (dR/du) du + (dR/dp) dp.

Run from the repository root:  python tests/golden/make_cube2_exact.py
Only oracle/ computes; paper_2403_08777_amd.synth supplies the lattice and
the relabelling (input generation, no assembly arithmetic).
"""

from __future__ import annotations

import os
import sys
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))
PATH = os.path.join(HERE, "cube2_exact.txt")

A = [[Fraction(1), Fraction(1, 4), Fraction(0)],
     [Fraction(0), Fraction(3, 4), Fraction(1, 8)],
     [Fraction(1, 8), Fraction(0), Fraction(5, 4)]]
B = [Fraction(1, 2), Fraction(-1, 4), Fraction(1, 8)]
RHO, MU = Fraction(5, 4), Fraction(3, 1000)
F = [Fraction(1, 10), Fraction(-1, 5), Fraction(3, 10)]
VECTOR_BLOCKS = ("x", "u", "lam", "du", "rhs", "rhs_emac", "vjp", "jvp")
SCALAR_BLOCKS = ("p", "dp", "vjp_p")


def _inputs():
    import numpy as np

    sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
    from paper_2403_08777_amd import synth

    n = 2
    m = synth.cube_mesh(n, permute=True)
    idx = np.rint(m.coords * n).astype(np.int64)
    x = []
    for row in idx:
        c = [Fraction(int(v), n) for v in row]
        if all(0 < v < n for v in row):
            c = [c[i] + Fraction(d, 16 * n) for i, d in enumerate((3, -2, 1))]
        x.append([sum(A[i][j] * c[j] for j in range(3)) + B[i] for i in range(3)])
    rng = np.random.default_rng(2403)
    nn = len(x)

    def field(ncomp):
        vals = rng.integers(-64, 65, (nn, ncomp))
        return [[Fraction(int(v), 32) for v in row] for row in vals]

    u, p, lam, du, dp = field(3), field(1), field(3), field(3), field(1)
    return x, [[int(v) for v in row] for row in m.conn], u, [r[0] for r in p], lam, du, [r[0] for r in dp]


def compute(x, conn, u, p, lam, du, dp):
    """Expected blocks from the exact checker."""
    from oracle import exact

    return {
        "rhs": exact.assemble_rhs(x, conn, u, p, RHO, MU, F),
        "rhs_emac": exact.assemble_rhs(x, conn, u, p, RHO, MU, F, form="emac"),
        "vjp": exact.assemble_vjp(x, conn, u, lam, RHO, MU, F),
        "vjp_p": exact.assemble_vjp_p(x, conn, u, lam, RHO, MU, F),
        "jvp": exact.assemble_jvp(x, conn, u, p, du, dp, RHO, MU, F),
    }


def write():
    x, conn, u, p, lam, du, dp = _inputs()
    out = compute(x, conn, u, p, lam, du, dp)
    lines = ["# exact P1 momentum RHS and derivatives on a skewed, relabelled 2^3 Kuhn cube",
             "# written by tests/golden/make_cube2_exact.py (oracle/exact.py); see its docstring",
             f"nodes {len(x)}", f"elems {len(conn)}",
             f"rho {RHO}", f"mu {MU}", "f " + " ".join(str(v) for v in F)]
    lines += [f"e {k} " + " ".join(str(v) for v in row) for k, row in enumerate(conn)]
    blocks = {"x": x, "u": u, "lam": lam, "du": du, "p": p, "dp": dp, **out}
    for name in VECTOR_BLOCKS:
        lines += [f"{name} {k} " + " ".join(str(v) for v in row) for k, row in enumerate(blocks[name])]
    for name in SCALAR_BLOCKS:
        lines += [f"{name} {k} {v}" for k, v in enumerate(blocks[name])]
    with open(PATH, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def load(path: str = PATH) -> dict:
    """Fixture as a dict: 'conn' (list of 4-lists), rho, mu, f, and every
    vector/scalar block as lists of Fractions indexed by node."""
    d = {"conn": []}
    nn = None
    with open(path) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            tok = line.split()
            key = tok[0]
            if key == "nodes":
                nn = int(tok[1])
                for name in VECTOR_BLOCKS + SCALAR_BLOCKS:
                    d[name] = [None] * nn
            elif key == "elems":
                d["n_elems"] = int(tok[1])
            elif key in ("rho", "mu"):
                d[key] = Fraction(tok[1])
            elif key == "f":
                d["f"] = [Fraction(v) for v in tok[1:]]
            elif key == "e":
                d["conn"].append([int(v) for v in tok[2:]])
            elif key in VECTOR_BLOCKS:
                d[key][int(tok[1])] = [Fraction(v) for v in tok[2:]]
            elif key in SCALAR_BLOCKS:
                d[key][int(tok[1])] = Fraction(tok[2])
            else:
                raise ValueError(f"unknown fixture line: {line!r}")
    return d


if __name__ == "__main__":
    write()
    print(f"wrote {PATH}")
