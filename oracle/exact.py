"""Exact rational checker for the RHS assembly -- TEST INFRASTRUCTURE.

Computes the Galerkin integrals of the momentum right-hand side (no eddy
viscosity) over linear tetrahedra in exact rational arithmetic, without Gauss
points and without a floating-point inverse, so it can pin the FP64 oracle.

Every integrand is a product of barycentric coordinates (the P1 shape functions
N_a are the barycentric coordinates of the tetrahedron), integrated with the
closed form

    int_e N_0^k0 N_1^k1 N_2^k2 N_3^k3 dx = 6 V k0! k1! k2! k3! / (k0+k1+k2+k3+3)!

so the element contribution is
    R^e_{a,i} = -rho sum_b (int N_a N_b) (K u_b)_i          convective, K = G
                                                            (advective form)
                - q_i int N_a + rho f_i int N_a             pressure, body
                - mu (int 1) grad N_a . G_i,:               viscous
with G = grad u and q = grad p constant on the element.  With mu_t = 0 the
assembled RHS is a quadratic polynomial in u, so the velocity vector-Jacobian
product is obtained exactly by central differences with unit step.
"""

from __future__ import annotations

from fractions import Fraction
from math import factorial


def monomial_integral(vol: Fraction, k) -> Fraction:
    """Integral over a tetrahedron of volume vol of prod_a N_a^k[a]."""
    num = 6 * vol
    for ka in k:
        num *= factorial(ka)
    return num / factorial(sum(k) + 3)


def _det3(m):
    return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
            - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
            + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))


def element_geometry(xe):
    """Exact (V, grad N) from 4 rational vertices."""
    J = [[xe[c + 1][i] - xe[0][i] for c in range(3)] for i in range(3)]
    D = _det3(J)
    if D == 0:
        raise ValueError("degenerate element")
    # Cramer: (J^-1)[r][c] = cofactor(J)[c][r] / D
    def minor(r, c):
        rows = [i for i in range(3) if i != r]
        cols = [j for j in range(3) if j != c]
        return (J[rows[0]][cols[0]] * J[rows[1]][cols[1]] - J[rows[0]][cols[1]] * J[rows[1]][cols[0]])
    inv = [[((-1) ** (r + c)) * minor(c, r) / D for c in range(3)] for r in range(3)]
    grad = [None, inv[0], inv[1], inv[2]]
    grad[0] = [-(inv[0][j] + inv[1][j] + inv[2][j]) for j in range(3)]
    return abs(D) / 6, grad


# The convective forms as c = K u with K = G + alpha tr(G) I + beta G^T:
# advective (u.grad)u; divergence div(u (x) u) = (u.grad)u + (div u)u;
# skew-symmetric, their mean; rotational (curl u) x u = (u.grad)u - grad|u|^2/2;
# EMAC 2 D(u) u + (div u) u.
FORM_COEFFICIENTS = {"advective": (0, 0), "divergence": (1, 0), "skew": (Fraction(1, 2), 0),
                     "rotational": (0, -1), "emac": (1, 1)}


def element_rhs(xe, ue, pe, rho, mu, f, form="advective"):
    """Exact element vector R^e (4 x 3) for mu_t = 0.  With G constant, the
    convective integrand K u_h is linear in u_h, so int N_a K u_h =
    sum_b (int N_a N_b) K u_b exactly."""
    vol, gN = element_geometry(xe)
    G = [[sum(ue[a][i] * gN[a][j] for a in range(4)) for j in range(3)] for i in range(3)]
    q = [sum(pe[a] * gN[a][j] for a in range(4)) for j in range(3)]
    alpha, beta = FORM_COEFFICIENTS[form]
    tr = G[0][0] + G[1][1] + G[2][2]
    K = [[G[i][j] + (alpha * tr if i == j else 0) + beta * G[j][i] for j in range(3)] for i in range(3)]
    Gu = [[sum(K[i][j] * ue[b][j] for j in range(3)) for i in range(3)] for b in range(4)]
    int1 = monomial_integral(vol, (0, 0, 0, 0))
    re = []
    for a in range(4):
        ka = [0, 0, 0, 0]
        ka[a] = 1
        int_na = monomial_integral(vol, ka)
        row = []
        for i in range(3):
            conv = Fraction(0)
            for b in range(4):
                k = [0, 0, 0, 0]
                k[a] += 1
                k[b] += 1
                conv += monomial_integral(vol, k) * Gu[b][i]
            visc = int1 * sum(gN[a][j] * G[i][j] for j in range(3))
            row.append(-rho * conv - q[i] * int_na + rho * f[i] * int_na - mu * visc)
        re.append(row)
    return re


def assemble_rhs(coords, conn, u, p, rho, mu, f, mu_elem=None, form="advective"):
    """Exact assembled RHS as a list of Nn rows of 3 Fractions.  ``mu_elem``
    optionally gives each element its own (rational) viscosity; ``form`` names
    the convective form."""
    nn = len(coords)
    out = [[Fraction(0)] * 3 for _ in range(nn)]
    for e, tet in enumerate(conn):
        ids = [int(t) for t in tet]
        mu_e = mu if mu_elem is None else mu_elem[e]
        re = element_rhs([coords[n] for n in ids], [u[n] for n in ids], [p[n] for n in ids], rho, mu_e, f, form)
        for a, n in enumerate(ids):
            for i in range(3):
                out[n][i] += re[a][i]
    return out


def assemble_vjp(coords, conn, u, lam, rho, mu, f, form="advective", mu_elem=None):
    """Exact (dR/du)^T lam for mu_t = 0, by unit-step central differences of
    the quadratic element functional lam_e . R^e(u_e) (exact for quadratics).
    ``mu_elem`` optionally gives each element its own viscosity, held fixed
    (the derivative of a velocity-dependent viscosity is not included)."""
    nn = len(coords)
    zero_p = [Fraction(0)] * 4
    out = [[Fraction(0)] * 3 for _ in range(nn)]
    for e, tet in enumerate(conn):
        ids = [int(t) for t in tet]
        xe = [coords[n] for n in ids]
        le = [lam[n] for n in ids]
        mu_e = mu if mu_elem is None else mu_elem[e]

        def functional(ue):
            re = element_rhs(xe, ue, zero_p, rho, mu_e, f, form)
            return sum(le[a][i] * re[a][i] for a in range(4) for i in range(3))

        base = [list(u[n]) for n in ids]
        for b in range(4):
            for k in range(3):
                up = [row[:] for row in base]
                um = [row[:] for row in base]
                up[b][k] += 1
                um[b][k] -= 1
                out[ids[b]][k] += (functional(up) - functional(um)) / 2
    return out


def assemble_vjp_p(coords, conn, u, lam, rho, mu, f):
    """Exact (dR/dp)^T lam: R is affine in p, so a unit step in p_b changes
    lam . R by exactly the derivative."""
    nn = len(coords)
    out = [Fraction(0)] * nn
    for tet in conn:
        ids = [int(t) for t in tet]
        xe = [coords[n] for n in ids]
        ue = [u[n] for n in ids]
        le = [lam[n] for n in ids]
        zero = [Fraction(0)] * 4
        base = element_rhs(xe, ue, zero, rho, mu, f)
        for b in range(4):
            pe = [Fraction(0)] * 4
            pe[b] = Fraction(1)
            re = element_rhs(xe, ue, pe, rho, mu, f)
            out[ids[b]] += sum(le[a][i] * (re[a][i] - base[a][i]) for a in range(4) for i in range(3))
    return out


def assemble_jvp(coords, conn, u, p, du, dp, rho, mu, f, form="advective"):
    """Exact (dR/du) du + (dR/dp) dp for mu_t = 0: R is quadratic in u and
    affine in p, so the unit-step central difference is exact."""
    nn = len(coords)
    plus = [[u[n][i] + du[n][i] for i in range(3)] for n in range(nn)]
    minus = [[u[n][i] - du[n][i] for i in range(3)] for n in range(nn)]
    pp = [p[n] + dp[n] for n in range(nn)]
    pm = [p[n] - dp[n] for n in range(nn)]
    rp = assemble_rhs(coords, conn, plus, pp, rho, mu, f, form=form)
    rm = assemble_rhs(coords, conn, minus, pm, rho, mu, f, form=form)
    return [[(rp[n][i] - rm[n][i]) / 2 for i in range(3)] for n in range(nn)]
