"""CPU oracle for the Navier-Stokes momentum RHS assembly -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and this
package never imports the GPU library: the two share no code.

``nsasm_oracle.c`` is a plain FP64 element loop (see its header for the weak
form and the readings taken where the paper is silent); ``exact.py`` is an
exact rational checker that pins it.  This module builds the C library with gcc
and wraps it with ctypes/numpy.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "nsasm_oracle.c"), os.path.join(_HERE, "element_body.inc")]
LIB_PATH = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no fast-math, no FMA contraction)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-shared", "-fPIC", "-Wall", "-Wextra", "-o", tmp, _SRC[0], "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int32)
    i64 = ctypes.c_int64
    d = ctypes.c_double
    lib.oracle_default_threads.restype = ctypes.c_int
    lib.oracle_geometry.argtypes = [i64, dp, i64, ip, dp, dp]
    ci = ctypes.c_int
    lib.oracle_eddy.argtypes = [i64, dp, i64, ip, dp, d, d, d, dp, ci, ci, dp]
    lib.oracle_rhs.argtypes = [i64, dp, i64, ip, dp, dp, d, d, d, dp, ci, ci, dp, ci]
    lib.oracle_rhs_complex.argtypes = [i64, dp, i64, ip, dp, dp, dp, dp, d, d, d, dp, ci, ci, dp, dp]
    lib.oracle_vjp.argtypes = [i64, dp, i64, ip, dp, dp, d, d, d, dp, ci, ci, dp, ci]
    lib.oracle_vjp_p.argtypes = [i64, dp, i64, ip, dp, dp, ci]
    for fn in ("oracle_geometry", "oracle_eddy", "oracle_rhs", "oracle_rhs_complex", "oracle_vjp", "oracle_vjp_p"):
        getattr(lib, fn).restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError(f"expected shape {shape}, got {a.shape}")
    return a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a, ctype=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


_ERRORS = {1: "node id out of range", 2: "degenerate element (det J == 0)", 3: "out of memory"}


def _check(status):
    if status != 0:
        raise ValueError(f"oracle: {_ERRORS.get(status, status)}")


EDDY_MODELS = {"smagorinsky": 0, "vreman": 1}
CONVECTIVE_FORMS = {"advective": 0, "divergence": 1, "skew": 2, "rotational": 3, "emac": 4}


class Params:
    """Physical parameters: density, molecular viscosity, model constant cs
    (0 = no eddy viscosity; Smagorinsky constant, Vreman uses c = 2.5 cs^2),
    constant body-force acceleration, the eddy-viscosity model and the form of
    the convective term."""

    def __init__(self, rho=1.0, mu=1e-3, cs=0.0, f=(0.1, -0.2, 0.3), model="smagorinsky", form="advective"):
        self.rho, self.mu, self.cs = float(rho), float(mu), float(cs)
        self.f = np.asarray(f, dtype=np.float64).reshape(3).copy()
        self.model = EDDY_MODELS[model]
        self.form = CONVECTIVE_FORMS[form]

    def args(self):
        return (self.rho, self.mu, self.cs, _ptr(self.f), self.model, self.form)


def default_threads() -> int:
    return _load().oracle_default_threads()


def geometry(coords, conn):
    """(V_e, grad N) per element: shapes (Ne,), (Ne, 4, 3)."""
    x, c = _f64(coords), _i32(conn)
    ne = c.shape[0]
    vol = np.empty(ne)
    gn = np.empty((ne, 4, 3))
    _check(_load().oracle_geometry(x.shape[0], _ptr(x), ne, _ptr(c, ctypes.c_int32), _ptr(vol), _ptr(gn)))
    return vol, gn


def eddy(coords, conn, u, prm: Params):
    """Per-element eddy viscosity mu_t, shape (Ne,)."""
    x, c, uu = _f64(coords), _i32(conn), _f64(u)
    out = np.empty(c.shape[0])
    _check(_load().oracle_eddy(x.shape[0], _ptr(x), c.shape[0], _ptr(c, ctypes.c_int32), _ptr(uu),
                               *prm.args(), _ptr(out)))
    return out


def rhs(coords, conn, u, p, prm: Params, nthreads: int = 0):
    """Assembled RHS (Nn, 3)."""
    x, c = _f64(coords), _i32(conn)
    nn = x.shape[0]
    uu, pp = _f64(u, (nn, 3)), _f64(p, (nn,))
    out = np.empty((nn, 3))
    _check(_load().oracle_rhs(nn, _ptr(x), c.shape[0], _ptr(c, ctypes.c_int32), _ptr(uu), _ptr(pp),
                              *prm.args(), _ptr(out), int(nthreads)))
    return out


def rhs_complex(coords, conn, u, p, prm: Params):
    """RHS for complex velocity and pressure fields (complex-step
    differentiation)."""
    x, c = _f64(coords), _i32(conn)
    nn = x.shape[0]
    u = np.asarray(u, dtype=np.complex128).reshape(nn, 3)
    p = np.asarray(p, dtype=np.complex128).reshape(nn)
    ur, ui = _f64(u.real), _f64(u.imag)
    pr, pi = _f64(p.real), _f64(p.imag)
    rr, ri = np.empty((nn, 3)), np.empty((nn, 3))
    _check(_load().oracle_rhs_complex(nn, _ptr(x), c.shape[0], _ptr(c, ctypes.c_int32), _ptr(ur),
                                      _ptr(ui), _ptr(pr), _ptr(pi), *prm.args(), _ptr(rr), _ptr(ri)))
    return rr + 1j * ri


def jvp(coords, conn, u, p, du, dp, prm: Params, h: float = 1e-30):
    """Directional derivative (dR/du) du + (dR/dp) dp by complex-step
    differentiation of the oracle: Im R(u + i h du, p + i h dp) / h."""
    nn = np.asarray(coords).shape[0]
    u, du = _f64(u, (nn, 3)), _f64(du, (nn, 3))
    p = _f64(p, (nn,))
    dp = np.zeros(nn) if dp is None else _f64(dp, (nn,))
    return rhs_complex(coords, conn, u + 1j * h * du, p + 1j * h * dp, prm).imag / h


def vjp_p(coords, conn, lam, nthreads: int = 0):
    """Pressure VJP (dR/dp)^T lam, shape (Nn,)."""
    x, c = _f64(coords), _i32(conn)
    nn = x.shape[0]
    ll = _f64(lam, (nn, 3))
    out = np.empty(nn)
    _check(_load().oracle_vjp_p(nn, _ptr(x), c.shape[0], _ptr(c, ctypes.c_int32), _ptr(ll), _ptr(out),
                                int(nthreads)))
    return out


def vjp(coords, conn, u, lam, prm: Params, nthreads: int = 0):
    """Velocity VJP (dR/du)^T lam, shape (Nn, 3)."""
    x, c = _f64(coords), _i32(conn)
    nn = x.shape[0]
    uu, ll = _f64(u, (nn, 3)), _f64(lam, (nn, 3))
    out = np.empty((nn, 3))
    _check(_load().oracle_vjp(nn, _ptr(x), c.shape[0], _ptr(c, ctypes.c_int32), _ptr(uu), _ptr(ll),
                              *prm.args(), _ptr(out), int(nthreads)))
    return out


def dense_jacobian_complex_step(coords, conn, u, p, prm: Params, h: float = 1e-30, wrt: str = "u"):
    """dR/du (3 Nn x 3 Nn) or dR/dp (3 Nn x Nn) as a dense matrix by
    complex-step differentiation (Squire & Trapp 1998): column k =
    Im R(v + i h e_k) / h, free of subtractive cancellation."""
    nn = np.asarray(coords).shape[0]
    u, p = _f64(u, (nn, 3)), _f64(p, (nn,))
    ncol = 3 * nn if wrt == "u" else nn
    jac = np.empty((3 * nn, ncol))
    for k in range(ncol):
        e = np.zeros(ncol)
        e[k] = h
        if wrt == "u":
            r = rhs_complex(coords, conn, u + 1j * e.reshape(nn, 3), p, prm)
        else:
            r = rhs_complex(coords, conn, u, p + 1j * e, prm)
        jac[:, k] = r.imag.reshape(-1) / h
    return jac


def rel_l2(a, b) -> float:
    """||a - b||_2 / ||b||_2 (b is the reference)."""
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def lumped_volume(coords, conn):
    """Row-sum lumped volume V^L_n = sum over elements e containing n of
    V_e / 4 (the P1 lumped mass divided by the density), shape (Nn,)."""
    vol, _ = geometry(coords, conn)
    c = _i32(conn)
    out = np.zeros(np.asarray(coords).shape[0])
    np.add.at(out, c.reshape(-1), np.repeat(vol / 4.0, 4))
    return out


def explicit_update(coords, conn, u, p, prm: Params, dt, mask=None):
    """One explicit momentum stage of the fractional-step scheme (Sec. II:
    explicit time integration of the momentum equation): with the lumped
    mass M_L,n = rho V^L_n,
        u_new[n, i] = u[n, i] + dt R[n, i] / (rho V^L_n)
    for free components, and u_new[n, i] = u[n, i] where bit i of mask[n] is
    set (Dirichlet-constrained components keep the value the caller put in
    u).  A node that no element references has no mass (V^L_n = 0) and no
    residual; the stage leaves it unchanged (u_new = u), the reading taken
    where the update would otherwise be 0/0.  Returns (u_new, R)."""
    u = _f64(u)
    R = rhs(coords, conn, u, p, prm)
    vl = lumped_volume(coords, conn)
    inv_mass = np.zeros_like(vl)
    np.divide(1.0, prm.rho * vl, out=inv_mass, where=vl > 0)
    step = u + dt * R * inv_mass[:, None]
    if mask is None:
        return step, R
    m = np.asarray(mask, dtype=np.uint8)
    fixed = np.stack([(m >> i) & 1 for i in range(3)], axis=1).astype(bool)
    return np.where(fixed, u, step), R
