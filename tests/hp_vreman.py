"""High-precision reference of the Vreman-model assembly and its velocity VJP
(test infrastructure shared by CPU and GPU tests).

On strongly anisotropic elements Vreman's B is a small difference of products
of the velocity gradient, so two FP64 evaluations that differ only in rounding
order disagree far above 1e-12; the kernel and the FP64 oracle are then both
compared with this reference.  Geometry, the velocity gradient and the
frozen-viscosity parts are exact rationals (oracle.exact); the eddy viscosity
follows Vreman's definition (alpha_ij = du_j/dx_i, beta = Delta^2 alpha^T alpha,
B_beta the sum of the principal 2x2 minors of beta, nu_t = c sqrt(B_beta /
alpha:alpha), c = 2.5 C_s^2) in 60-digit decimals, and its derivative by
central differences in those decimals (step 1e-25 of the gradient's scale:
truncation ~1e-50, rounding ~1e-35 relative)."""

from __future__ import annotations

from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np

from oracle import exact


def _dec(q: Fraction) -> Decimal:
    return Decimal(q.numerator) / Decimal(q.denominator)


def vreman_mu_t(G, vol, rho, cs):
    """rho nu_t of Vreman's model for the velocity gradient G[i][j] = du_i/dx_j
    (Decimals) on an element of volume vol, Delta = vol^(1/3)."""
    d2 = (vol ** (Decimal(1) / Decimal(3))) ** 2
    al = [[G[j][i] for j in range(3)] for i in range(3)]
    be = [[d2 * sum(al[m][i] * al[m][j] for m in range(3)) for j in range(3)] for i in range(3)]
    b = (be[0][0] * be[1][1] - be[0][1] ** 2 + be[0][0] * be[2][2] - be[0][2] ** 2 + be[1][1] * be[2][2]
         - be[1][2] ** 2)
    aa = sum(al[i][j] ** 2 for i in range(3) for j in range(3))
    if aa <= 0 or b <= 0:
        return Decimal(0)
    return Decimal(rho) * Decimal(2.5) * Decimal(cs) ** 2 * (b / aa).sqrt()


def _elements(coords, conn, u):
    cq = [[Fraction(float(v)) for v in row] for row in coords]
    uq = [[Fraction(float(v)) for v in row] for row in u]
    for tet in conn:
        ids = [int(t) for t in tet]
        vol, gn = exact.element_geometry([cq[n] for n in ids])
        ue = [uq[n] for n in ids]
        G = [[sum(ue[a][i] * gn[a][j] for a in range(4)) for j in range(3)] for i in range(3)]
        yield ids, vol, gn, G


def element_viscosity(coords, conn, u, rho, mu, cs):
    """Per-element mu + mu_t (Fractions of 60-digit decimals)."""
    getcontext().prec = 60
    out = []
    for _, vol, _, G in _elements(coords, conn, u):
        Gd = [[_dec(G[i][j]) for j in range(3)] for i in range(3)]
        out.append(Fraction(Decimal(mu) + vreman_mu_t(Gd, _dec(vol), rho, cs)))
    return out


def vjp(coords, conn, u, lam, rho, mu, cs, f):
    """(dR/du)^T lam with Vreman's eddy viscosity, as float64 (Nn, 3):
    the frozen-viscosity VJP exactly, plus -V Phi d mu_t / d u_b per element,
    Phi = sum_a lam_a . G grad N_a (d/du of -mu_e V Phi, the viscous term's
    contribution to lam . R)."""
    getcontext().prec = 60
    nn = len(coords)
    lq = [[Fraction(float(v)) for v in row] for row in lam]
    mu_elem = []
    eddy = [[Decimal(0)] * 3 for _ in range(nn)]
    for ids, vol, gn, G in _elements(coords, conn, u):
        Gd = [[_dec(G[i][j]) for j in range(3)] for i in range(3)]
        vd = _dec(vol)
        mu_elem.append(Fraction(Decimal(mu) + vreman_mu_t(Gd, vd, rho, cs)))
        h = max(abs(v) for row in Gd for v in row) * Decimal("1e-25")
        D = [[Decimal(0)] * 3 for _ in range(3)]
        for i in range(3):
            for j in range(3):
                gp = [row[:] for row in Gd]
                gm = [row[:] for row in Gd]
                gp[i][j] += h
                gm[i][j] -= h
                D[i][j] = (vreman_mu_t(gp, vd, rho, cs) - vreman_mu_t(gm, vd, rho, cs)) / (2 * h)
        le = [lq[n] for n in ids]
        phi = _dec(sum(le[a][i] * sum(G[i][j] * gn[a][j] for j in range(3)) for a in range(4) for i in range(3)))
        for b, n in enumerate(ids):
            for k in range(3):
                eddy[n][k] -= vd * phi * sum(D[k][j] * _dec(gn[b][j]) for j in range(3))
    cq = [[Fraction(float(v)) for v in row] for row in coords]
    uq = [[Fraction(float(v)) for v in row] for row in u]
    fq = [Fraction(float(v)) for v in f]
    frozen = exact.assemble_vjp(cq, conn, uq, lq, Fraction(rho), Fraction(mu), fq, mu_elem=mu_elem)
    return np.array([[float(_dec(frozen[n][k]) + eddy[n][k]) for k in range(3)] for n in range(nn)])
