"""Operation counts of the literal element method -- TEST INFRASTRUCTURE.

The algorithmic flop count per element that the roofline of the assembly is
priced against: the element steps of the method evaluated literally, as the
paper's kernel and the C oracle do (Sec. V-B: the Jacobian and its inverse,
the constant gradients, the eddy viscosity once per element, four Gauss points
with the shape-function values as constants, the viscous term, then the
scatter of the 12 element values), with a scalar type that counts its
arithmetic.  Conventions: add, subtract, multiply and divide count one flop
each (a fused multiply-add is two), square and cube roots one each; negation,
comparisons and arithmetic on parameters alone (rho f, cs^2: the same for
every element) count nothing.  Forms: the advective convective term, with and
without Smagorinsky eddy viscosity (the benchmarked configurations).

The velocity VJP follows the per-Gauss-point formula of its definition:
  g_b,k = -rho sum_g (V/4) [ N_b(g) sum_i lambda^g_i G_ik + lambda^g_k (u^g . grad N_b) ]
          - mu_e V (grad N_b . Lambda_k,:) - V Phi d mu_t / d u_b,k,
  Lambda_kj = sum_a lambda_a,k d_j N_a,  Phi = Lambda : G,
  d mu_t / d u_b,k = rho (cs Delta)^2 (2 / |S|) sum_j S_kj d_j N_b.

The same functions run on plain floats, so tests pin this transcription to the
C oracle's values before its counts are used.
"""

from __future__ import annotations

import math

GAUSS_ALPHA = (5.0 + 3.0 * math.sqrt(5.0)) / 20.0
GAUSS_BETA = (5.0 - math.sqrt(5.0)) / 20.0


class Counter:
    def __init__(self):
        self.flops = 0


class Counted:
    """A float that adds one to its counter for every arithmetic operation."""

    __slots__ = ("v", "c")

    def __init__(self, v, c):
        self.v, self.c = float(v), c

    def _op(self, other, f):
        self.c.flops += 1
        o = other.v if isinstance(other, Counted) else other
        return Counted(f(self.v, o), self.c)

    def _rop(self, other, f):
        self.c.flops += 1
        return Counted(f(other, self.v), self.c)

    def __add__(self, o): return self._op(o, lambda a, b: a + b)
    def __radd__(self, o): return self._rop(o, lambda a, b: a + b)
    def __sub__(self, o): return self._op(o, lambda a, b: a - b)
    def __rsub__(self, o): return self._rop(o, lambda a, b: a - b)
    def __mul__(self, o): return self._op(o, lambda a, b: a * b)
    def __rmul__(self, o): return self._rop(o, lambda a, b: a * b)
    def __truediv__(self, o): return self._op(o, lambda a, b: a / b)
    def __rtruediv__(self, o): return self._rop(o, lambda a, b: a / b)
    def __neg__(self): return Counted(-self.v, self.c)
    def __abs__(self): return Counted(abs(self.v), self.c)
    def __float__(self): return self.v
    def __eq__(self, o): return self.v == (o.v if isinstance(o, Counted) else o)
    def __gt__(self, o): return self.v > (o.v if isinstance(o, Counted) else o)
    __hash__ = None


def _sqrt(x):
    if isinstance(x, Counted):
        x.c.flops += 1
        return Counted(math.sqrt(x.v), x.c)
    return math.sqrt(x)


def _cbrt(x):
    if isinstance(x, Counted):
        x.c.flops += 1
        return Counted(math.copysign(abs(x.v) ** (1.0 / 3.0), x.v), x.c)
    return math.copysign(abs(x) ** (1.0 / 3.0), x)


def geometry(xe):
    """Jacobian columns x_c - x_0, determinant, adjugate inverse, shape-function
    gradients (rows of the inverse; grad N_0 = -sum), volume |D| / 6."""
    J = [[xe[c + 1][i] - xe[0][i] for c in range(3)] for i in range(3)]
    D = (J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
         - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
         + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]))
    inv = [[(J[1][1] * J[2][2] - J[1][2] * J[2][1]) / D, (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / D,
            (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / D],
           [(J[1][2] * J[2][0] - J[1][0] * J[2][2]) / D, (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / D,
            (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / D],
           [(J[1][0] * J[2][1] - J[1][1] * J[2][0]) / D, (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / D,
            (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / D]]
    gN = [None, inv[0], inv[1], inv[2]]
    gN[0] = [-(gN[1][j] + gN[2][j] + gN[3][j]) for j in range(3)]
    vol = abs(D) / 6.0
    return gN, vol


def gradients(gN, ue, pe):
    G = [[ue[0][i] * gN[0][j] + ue[1][i] * gN[1][j] + ue[2][i] * gN[2][j] + ue[3][i] * gN[3][j]
          for j in range(3)] for i in range(3)]
    q = [pe[0] * gN[0][j] + pe[1] * gN[1][j] + pe[2] * gN[2][j] + pe[3] * gN[3][j] for j in range(3)]
    return G, q


def smagorinsky(G, vol, rho, cs):
    """mu_t, S and |S| (mu_t = 0 when cs = 0, and nothing is counted then)."""
    if cs <= 0.0:
        return 0.0, None, None
    S = [[0.5 * (G[i][j] + G[j][i]) for j in range(3)] for i in range(3)]
    ss = S[0][0] * S[0][0]
    for i in range(3):
        for j in range(3):
            if i or j:
                ss = ss + S[i][j] * S[i][j]
    smag = _sqrt(2.0 * ss)
    delta = _cbrt(vol)
    cd = cs * delta
    return rho * cd * cd * smag, S, smag


def _gauss_values(g):
    return [GAUSS_ALPHA if a == g else GAUSS_BETA for a in range(4)]


def element_rhs(xe, ue, pe, rho, mu, cs, f):
    """R^e[a][i]: Gauss-point convective, pressure and body terms, viscous term."""
    gN, vol = geometry(xe)
    G, q = gradients(gN, ue, pe)
    mu_t, _, _ = smagorinsky(G, vol, rho, cs)
    mu_e = mu + mu_t if cs > 0.0 else mu
    w = vol / 4.0
    rf = [rho * fi for fi in f]  # parameters only
    re = [[None] * 3 for _ in range(4)]
    for g in range(4):
        N = _gauss_values(g)
        ug = [N[0] * ue[0][j] + N[1] * ue[1][j] + N[2] * ue[2][j] + N[3] * ue[3][j] for j in range(3)]
        conv = [G[i][0] * ug[0] + G[i][1] * ug[1] + G[i][2] * ug[2] for i in range(3)]
        r = [-rho * conv[i] - q[i] + rf[i] for i in range(3)]
        for a in range(4):
            wn = w * N[a]
            for i in range(3):
                t = wn * r[i]
                re[a][i] = t if re[a][i] is None else re[a][i] + t
    mv = mu_e * vol
    for a in range(4):
        for i in range(3):
            v = gN[a][0] * G[i][0] + gN[a][1] * G[i][1] + gN[a][2] * G[i][2]
            re[a][i] = re[a][i] - mv * v
    return re


def element_vjp(xe, ue, le, rho, mu, cs):
    """g^e[b][k] by the definition's per-Gauss-point formula."""
    gN, vol = geometry(xe)
    G = [[ue[0][i] * gN[0][j] + ue[1][i] * gN[1][j] + ue[2][i] * gN[2][j] + ue[3][i] * gN[3][j]
          for j in range(3)] for i in range(3)]
    mu_t, S, smag = smagorinsky(G, vol, rho, cs)
    mu_e = mu + mu_t if cs > 0.0 else mu
    Lam = [[le[0][k] * gN[0][j] + le[1][k] * gN[1][j] + le[2][k] * gN[2][j] + le[3][k] * gN[3][j]
            for j in range(3)] for k in range(3)]
    wr = -rho * (vol / 4.0)
    ge = [[None] * 3 for _ in range(4)]
    for g in range(4):
        N = _gauss_values(g)
        ug = [N[0] * ue[0][j] + N[1] * ue[1][j] + N[2] * ue[2][j] + N[3] * ue[3][j] for j in range(3)]
        lg = [N[0] * le[0][j] + N[1] * le[1][j] + N[2] * le[2][j] + N[3] * le[3][j] for j in range(3)]
        gtl = [lg[0] * G[0][k] + lg[1] * G[1][k] + lg[2] * G[2][k] for k in range(3)]
        for b in range(4):
            udn = ug[0] * gN[b][0] + ug[1] * gN[b][1] + ug[2] * gN[b][2]
            for k in range(3):
                t = wr * (N[b] * gtl[k] + lg[k] * udn)
                ge[b][k] = t if ge[b][k] is None else ge[b][k] + t
    mv = mu_e * vol
    for b in range(4):
        for k in range(3):
            lv = gN[b][0] * Lam[k][0] + gN[b][1] * Lam[k][1] + gN[b][2] * Lam[k][2]
            ge[b][k] = ge[b][k] - mv * lv
    if cs > 0.0 and smag > 0.0:
        Phi = Lam[0][0] * G[0][0]
        for i in range(3):
            for j in range(3):
                if i or j:
                    Phi = Phi + Lam[i][j] * G[i][j]
        delta = _cbrt(vol)
        cd = cs * delta
        k2 = rho * cd * cd * 2.0 / smag
        vp = vol * Phi
        for b in range(4):
            for k in range(3):
                sn = S[k][0] * gN[b][0] + S[k][1] * gN[b][1] + S[k][2] * gN[b][2]
                ge[b][k] = ge[b][k] - vp * (k2 * sn)
    return ge


def assemble(kind, coords, conn, u, second, rho, mu, cs, f=(0.1, -0.2, 0.3)):
    """Assembled result on plain floats (kind 'rhs': second = p; 'vjp':
    second = lambda), for pinning this transcription to the C oracle."""
    nn = len(coords)
    out = [[0.0] * 3 for _ in range(nn)]
    for tet in conn:
        xe = [list(map(float, coords[n])) for n in tet]
        ue = [list(map(float, u[n])) for n in tet]
        if kind == "rhs":
            re = element_rhs(xe, ue, [float(second[n]) for n in tet], rho, mu, cs, f)
        else:
            re = element_vjp(xe, ue, [list(map(float, second[n])) for n in tet], rho, mu, cs)
        for a, n in enumerate(tet):
            for i in range(3):
                out[n][i] += float(re[a][i])
    return out


def flops_per_element(kind: str, eddy: bool) -> int:
    """Counted flops of one element (kind 'fwd' or 'vjp', Smagorinsky on or
    off), the 12 additions of the scatter included."""
    c = Counter()
    xe = [[Counted(v, c) for v in row] for row in
          ([0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 1.0, 0.1], [0.1, 0.2, 1.0])]
    ue = [[Counted(v, c) for v in row] for row in
          ([0.3, -0.2, 0.1], [0.5, 0.1, -0.4], [-0.1, 0.6, 0.2], [0.2, -0.3, 0.7])]
    cs = 0.1 if eddy else 0.0
    if kind == "fwd":
        pe = [Counted(v, c) for v in (0.1, -0.2, 0.3, 0.05)]
        element_rhs(xe, ue, pe, 1.0, 1e-3, cs, (0.1, -0.2, 0.3))
    elif kind == "vjp":
        le = [[Counted(v, c) for v in row] for row in
              ([0.4, 0.1, -0.2], [-0.3, 0.2, 0.5], [0.1, -0.6, 0.3], [0.7, 0.2, -0.1])]
        element_vjp(xe, ue, le, 1.0, 1e-3, cs)
    else:
        raise ValueError(kind)
    return c.flops + 12
