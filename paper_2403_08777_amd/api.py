"""Python binding of libnsasm (ctypes).  Argument marshalling only: every step
of the assembly runs in the HIP library; PyTorch provides device memory and the
current stream.  Importing this module loads the library and raises if it has
not been built (``python -m paper_2403_08777_amd.build``)."""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnsasm.so")

FP64 = 0
MIXED = 1
_SCATTER = {"auto": 0, "atomic": 1, "patch": 2, "patch_gather": 3}
_SCATTER_NAMES = {v: k for k, v in _SCATTER.items()}
ACCUMULATE = 1

STATUS_NAMES = {
    0: "OK", 1: "INVALID_ARGUMENT", 2: "BAD_CONNECTIVITY", 3: "DEGENERATE_ELEMENT",
    4: "OUT_OF_MEMORY", 5: "DEVICE", 6: "UNSUPPORTED",
}


class NsasmError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        self.status_name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"nsasm {self.status_name}: {message}")


class _Params(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("mu", ctypes.c_double), ("smagorinsky_cs", ctypes.c_double),
                ("body_force", ctypes.c_double * 3), ("flags", ctypes.c_uint32), ("eddy_model", ctypes.c_uint32),
                ("convective_form", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class _MeshOptions(ctypes.Structure):
    _fields_ = [("renumber", ctypes.c_int32), ("scatter", ctypes.c_int32), ("patch_elems", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _MeshInfo(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_elems", ctypes.c_int64), ("scatter", ctypes.c_int32),
                ("renumbered", ctypes.c_int32), ("n_patches", ctypes.c_int32), ("patch_elems", ctypes.c_int32),
                ("max_patch_nodes", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("patch_node_refs", ctypes.c_int64)]


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_2403_08777_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, st = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
    lib.nsasm_mesh_create.argtypes = [vp, i64, vp, i64, ctypes.POINTER(_MeshOptions), vp, ctypes.POINTER(vp)]
    lib.nsasm_mesh_destroy.argtypes = [vp]
    lib.nsasm_mesh_info.argtypes = [vp, ctypes.POINTER(_MeshInfo)]
    lib.nsasm_mesh_permutation.argtypes = [vp, vp, vp]
    lib.nsasm_mesh_connectivity.argtypes = [vp, vp, vp, vp]
    lib.nsasm_to_mesh_order.argtypes = [vp, i32, st, vp, vp, vp]
    lib.nsasm_from_mesh_order.argtypes = [vp, i32, st, vp, vp, vp]
    lib.nsasm_assemble_rhs.argtypes = [vp, ctypes.POINTER(_Params), st, vp, vp, vp, vp]
    lib.nsasm_assemble_rhs_noalloc.argtypes = [vp, ctypes.POINTER(_Params), st, vp, vp, vp, vp]
    lib.nsasm_assemble_rhs_vjp.argtypes = [vp, ctypes.POINTER(_Params), st, vp, vp, vp, vp]
    lib.nsasm_assemble_rhs_vjp_p.argtypes = [vp, ctypes.POINTER(_Params), st, vp, vp, vp]
    lib.nsasm_assemble_rhs_jvp.argtypes = [vp, ctypes.POINTER(_Params), st, vp, vp, vp, vp, vp]
    lib.nsasm_mesh_lumped_volume.argtypes = [vp, vp, vp]
    lib.nsasm_explicit_update.argtypes = [vp, ctypes.POINTER(_Params), st, ctypes.c_double, vp, vp, vp, vp, vp,
                                          vp]
    lib.nsasm_stream_scale.argtypes = [vp, vp, i64, ctypes.c_double, vp]
    lib.nsasm_scatter_add.argtypes = [vp, i64, i32, st, ctypes.c_double, vp, i64, vp]
    lib.nsasm_set_kernel_events.argtypes = [vp, vp, vp, vp]
    for name in ("nsasm_mesh_create", "nsasm_mesh_destroy", "nsasm_mesh_info", "nsasm_mesh_permutation",
                 "nsasm_mesh_connectivity", "nsasm_to_mesh_order", "nsasm_from_mesh_order",
                 "nsasm_assemble_rhs", "nsasm_assemble_rhs_noalloc", "nsasm_assemble_rhs_vjp",
                 "nsasm_assemble_rhs_vjp_p", "nsasm_assemble_rhs_jvp", "nsasm_mesh_lumped_volume", "nsasm_explicit_update",
                 "nsasm_stream_scale", "nsasm_scatter_add", "nsasm_set_kernel_events"):
        getattr(lib, name).restype = st
    lib.nsasm_last_error.restype = ctypes.c_char_p
    lib.nsasm_last_error.argtypes = []
    lib.nsasm_version.restype = ctypes.c_char_p
    lib.nsasm_version.argtypes = []
    return lib


lib = _load()


def _check(status: int) -> None:
    if status != 0:
        raise NsasmError(status, lib.nsasm_last_error().decode())


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _dev(t: torch.Tensor, dtype, shape, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


EDDY_MODELS = {"smagorinsky": 0, "vreman": 1}
CONVECTIVE_FORMS = {"advective": 0, "divergence": 1, "skew": 2, "rotational": 3, "emac": 4}


@dataclass
class Params:
    """Density, molecular viscosity, eddy-viscosity model constant C_s
    (0 = no eddy viscosity), constant body-force acceleration, the model
    ("smagorinsky", or "vreman" with c = 2.5 C_s^2) and the convective form
    ("advective", "divergence", "skew", "rotational" or "emac"; see
    NSASM_CONVECTIVE_* in nsasm.h)."""

    rho: float = 1.0
    mu: float = 1e-3
    cs: float = 0.0
    body_force: tuple = (0.1, -0.2, 0.3)
    eddy_model: str = "smagorinsky"
    convective_form: str = "advective"

    def c_struct(self, accumulate: bool = False) -> _Params:
        f = tuple(float(v) for v in self.body_force)
        return _Params(float(self.rho), float(self.mu), float(self.cs), (ctypes.c_double * 3)(*f),
                       ACCUMULATE if accumulate else 0, EDDY_MODELS[self.eddy_model],
                       CONVECTIVE_FORMS[self.convective_form], 0)


class Mesh:
    """A preprocessed tetrahedral mesh on the current GPU.

    coords: (Nn, 3) float64, conn: (Ne, 4) int32, both CUDA tensors in user
    numbering.  ``renumber`` reorders elements/nodes for locality; fields
    passed to the assembly are in mesh order (see to_mesh_order)."""

    def __init__(self, coords: torch.Tensor, conn: torch.Tensor, renumber: bool = True,
                 scatter: str = "auto", patch_elems: int = 0, stream=None):
        if scatter not in _SCATTER:
            raise ValueError(f"scatter must be one of {sorted(_SCATTER)}")
        nn, ne = int(coords.shape[0]), int(conn.shape[0])
        _dev(coords, torch.float64, (nn, 3), "coords")
        _dev(conn, torch.int32, (ne, 4), "conn")
        self.device = coords.device
        opts = _MeshOptions(1 if renumber else 0, _SCATTER[scatter], int(patch_elems), 0)
        handle = ctypes.c_void_p()
        _check(lib.nsasm_mesh_create(coords.data_ptr(), nn, conn.data_ptr(), ne, ctypes.byref(opts),
                                     _stream(stream), ctypes.byref(handle)))
        self._h = handle
        info = _MeshInfo()
        _check(lib.nsasm_mesh_info(self._h, ctypes.byref(info)))
        self.n_nodes, self.n_elems = int(info.n_nodes), int(info.n_elems)
        self.info = {f: getattr(info, f) for f, _ in _MeshInfo._fields_ if f != "reserved"}
        self.info["scatter"] = _SCATTER_NAMES[self.info["scatter"]]

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise ValueError("mesh has been closed")
        return self._h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            _check(lib.nsasm_mesh_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def permutation(self, stream=None) -> torch.Tensor:
        """int32 (Nn,): mesh-order index of every user node."""
        out = torch.empty(self.n_nodes, dtype=torch.int32, device=self.device)
        _check(lib.nsasm_mesh_permutation(self.handle, out.data_ptr(), _stream(stream)))
        return out

    def connectivity(self, stream=None):
        """(conn_mesh (Ne, 4) int32 in mesh numbering/order, user element index (Ne,))."""
        conn = torch.empty((self.n_elems, 4), dtype=torch.int32, device=self.device)
        elem = torch.empty(self.n_elems, dtype=torch.int32, device=self.device)
        _check(lib.nsasm_mesh_connectivity(self.handle, conn.data_ptr(), elem.data_ptr(), _stream(stream)))
        return conn, elem

    def _reorder(self, t: torch.Tensor, to_mesh: bool, stream) -> torch.Tensor:
        prec = {torch.float64: FP64, torch.float32: MIXED}.get(t.dtype)
        if prec is None:
            raise TypeError("fields must be float64 or float32")
        ncomp = 1 if t.dim() == 1 else int(t.shape[1])
        _dev(t, t.dtype, (self.n_nodes,) if t.dim() == 1 else (self.n_nodes, ncomp), "field")
        out = torch.empty_like(t)
        fn = lib.nsasm_to_mesh_order if to_mesh else lib.nsasm_from_mesh_order
        _check(fn(self.handle, ncomp, prec, t.data_ptr(), out.data_ptr(), _stream(stream)))
        return out

    def lumped_volume(self, stream=None) -> torch.Tensor:
        """float64 (Nn,), mesh order: V^L_n = sum of V_e / 4 over the elements
        containing node n (the lumped mass divided by the density)."""
        out = torch.empty(self.n_nodes, dtype=torch.float64, device=self.device)
        _check(lib.nsasm_mesh_lumped_volume(self.handle, out.data_ptr(), _stream(stream)))
        return out

    def to_mesh_order(self, t: torch.Tensor, stream=None) -> torch.Tensor:
        return self._reorder(t, True, stream)

    def from_mesh_order(self, t: torch.Tensor, stream=None) -> torch.Tensor:
        return self._reorder(t, False, stream)


def _precision_of(u: torch.Tensor) -> int:
    if u.dtype == torch.float64:
        return FP64
    if u.dtype == torch.float32:
        return MIXED
    raise TypeError("u must be float64 (FP64) or float32 (mixed precision)")


def assemble_rhs(mesh: Mesh, u: torch.Tensor, p: torch.Tensor, params: Params, out: torch.Tensor = None,
                 accumulate: bool = False, stream=None) -> torch.Tensor:
    """Momentum RHS (Nn, 3) in mesh order.  float64 fields -> FP64 path,
    float32 fields -> mixed path (FP64 geometry)."""
    prec = _precision_of(u)
    nn = mesh.n_nodes
    _dev(u, u.dtype, (nn, 3), "u")
    _dev(p, u.dtype, (nn,), "p")
    if out is None:
        out = torch.empty((nn, 3), dtype=u.dtype, device=u.device)
    else:
        _dev(out, u.dtype, (nn, 3), "out")
    prm = params.c_struct(accumulate)
    _check(lib.nsasm_assemble_rhs(mesh.handle, ctypes.byref(prm), prec, u.data_ptr(), p.data_ptr(),
                                  out.data_ptr(), _stream(stream)))
    return out


def assemble_rhs_noalloc(mesh: Mesh, u: torch.Tensor, p: torch.Tensor, params: Params, out: torch.Tensor,
                        accumulate: bool = False, stream=None) -> torch.Tensor:
    """As assemble_rhs, through nsasm_assemble_rhs_noalloc: the library
    allocates nothing (the gather scatter's partial sums use its fixed
    per-GPU region), so `out` must be given."""
    prec = _precision_of(u)
    nn = mesh.n_nodes
    _dev(u, u.dtype, (nn, 3), "u")
    _dev(p, u.dtype, (nn,), "p")
    _dev(out, u.dtype, (nn, 3), "out")
    prm = params.c_struct(accumulate)
    _check(lib.nsasm_assemble_rhs_noalloc(mesh.handle, ctypes.byref(prm), prec, u.data_ptr(), p.data_ptr(),
                                          out.data_ptr(), _stream(stream)))
    return out


def assemble_rhs_vjp(mesh: Mesh, u: torch.Tensor, adjoint: torch.Tensor, params: Params,
                     out: torch.Tensor = None, accumulate: bool = False, stream=None) -> torch.Tensor:
    """(d rhs / d u)^T adjoint, (Nn, 3) in mesh order."""
    prec = _precision_of(u)
    nn = mesh.n_nodes
    _dev(u, u.dtype, (nn, 3), "u")
    _dev(adjoint, u.dtype, (nn, 3), "adjoint")
    if out is None:
        out = torch.empty((nn, 3), dtype=u.dtype, device=u.device)
    else:
        _dev(out, u.dtype, (nn, 3), "out")
    prm = params.c_struct(accumulate)
    _check(lib.nsasm_assemble_rhs_vjp(mesh.handle, ctypes.byref(prm), prec, u.data_ptr(), adjoint.data_ptr(),
                                      out.data_ptr(), _stream(stream)))
    return out


def assemble_rhs_vjp_p(mesh: Mesh, adjoint: torch.Tensor, params: Params, out: torch.Tensor = None,
                       accumulate: bool = False, stream=None) -> torch.Tensor:
    """(d rhs / d p)^T adjoint, (Nn,) in mesh order."""
    prec = _precision_of(adjoint)
    nn = mesh.n_nodes
    _dev(adjoint, adjoint.dtype, (nn, 3), "adjoint")
    if out is None:
        out = torch.empty(nn, dtype=adjoint.dtype, device=adjoint.device)
    else:
        _dev(out, adjoint.dtype, (nn,), "out")
    prm = params.c_struct(accumulate)
    _check(lib.nsasm_assemble_rhs_vjp_p(mesh.handle, ctypes.byref(prm), prec, adjoint.data_ptr(), out.data_ptr(),
                                        _stream(stream)))
    return out


def assemble_rhs_jvp(mesh: Mesh, u: torch.Tensor, du: torch.Tensor, dp: torch.Tensor, params: Params,
                     out: torch.Tensor = None, accumulate: bool = False, stream=None) -> torch.Tensor:
    """(d rhs / d u) du + (d rhs / d p) dp, (Nn, 3) in mesh order; dp may be None."""
    prec = _precision_of(u)
    nn = mesh.n_nodes
    _dev(u, u.dtype, (nn, 3), "u")
    _dev(du, u.dtype, (nn, 3), "du")
    if dp is not None:
        _dev(dp, u.dtype, (nn,), "dp")
    if out is None:
        out = torch.empty((nn, 3), dtype=u.dtype, device=u.device)
    else:
        _dev(out, u.dtype, (nn, 3), "out")
    prm = params.c_struct(accumulate)
    _check(lib.nsasm_assemble_rhs_jvp(mesh.handle, ctypes.byref(prm), prec, u.data_ptr(), du.data_ptr(),
                                      None if dp is None else dp.data_ptr(), out.data_ptr(), _stream(stream)))
    return out


def explicit_update(mesh: Mesh, u: torch.Tensor, p: torch.Tensor, params: Params, dt: float,
                    dirichlet_mask: torch.Tensor = None, rhs: torch.Tensor = None, out: torch.Tensor = None,
                    stream=None) -> torch.Tensor:
    """One explicit momentum stage in mesh order: u + dt rhs / (rho V^L) for
    free components, u for components whose bit (0..2) is set in the uint8
    dirichlet_mask (Nn,).  ``rhs`` (Nn, 3) optionally receives the assembled
    RHS; meshes that do not use the gather scatter need it as workspace, and
    it is allocated here when not given.  ``out`` may be ``u`` itself (in-place
    update).  Returns the updated velocity."""
    prec = _precision_of(u)
    nn = mesh.n_nodes
    _dev(u, u.dtype, (nn, 3), "u")
    _dev(p, u.dtype, (nn,), "p")
    if dirichlet_mask is not None:
        _dev(dirichlet_mask, torch.uint8, (nn,), "dirichlet_mask")
    if rhs is None and mesh.info["scatter"] != "patch_gather":
        rhs = torch.empty((nn, 3), dtype=u.dtype, device=u.device)
    if rhs is not None:
        _dev(rhs, u.dtype, (nn, 3), "rhs")
    if out is None:
        out = torch.empty((nn, 3), dtype=u.dtype, device=u.device)
    else:
        _dev(out, u.dtype, (nn, 3), "out")
    prm = params.c_struct()
    _check(lib.nsasm_explicit_update(mesh.handle, ctypes.byref(prm), prec, float(dt), u.data_ptr(), p.data_ptr(),
                                     None if dirichlet_mask is None else dirichlet_mask.data_ptr(),
                                     None if rhs is None else rhs.data_ptr(), out.data_ptr(), _stream(stream)))
    return out


def stream_scale(a: torch.Tensor, s: float, out: torch.Tensor = None, stream=None) -> torch.Tensor:
    """out = s * a for a 1-D float64 tensor (the Scale bandwidth kernel); out
    must not overlap a."""
    if not isinstance(a, torch.Tensor) or a.dim() != 1:
        raise ValueError("a must be a 1-D torch.Tensor")
    _dev(a, torch.float64, a.shape, "a")
    if out is None:
        out = torch.empty_like(a)
    else:
        _dev(out, torch.float64, a.shape, "out")
    _check(lib.nsasm_stream_scale(a.data_ptr(), out.data_ptr(), a.numel(), float(s), _stream(stream)))
    return out


def scatter_add(index: torch.Tensor, out: torch.Tensor, value: float = 1.0, stream=None) -> torch.Tensor:
    """out[index[k], :] += value with one device-scope atomic add per entry
    and column (the atomic-rate measurement kernel); index is a 1-D int32
    tensor, out a 2-D float64 (FP64) or float32 (mixed) tensor.  Entries of
    index outside [0, out.shape[0]) are skipped."""
    if index.dim() != 1 or out.dim() != 2:
        raise ValueError("index must be 1-D and out 2-D")
    _dev(index, torch.int32, index.shape, "index")
    prec = _precision_of(out)
    _dev(out, out.dtype, out.shape, "out")
    _check(lib.nsasm_scatter_add(index.data_ptr(), index.numel(), out.shape[1], prec, float(value), out.data_ptr(),
                                 out.shape[0], _stream(stream)))
    return out


def set_kernel_events(element_start=None, element_stop=None, gather_start=None, gather_stop=None) -> None:
    """Have the next assembly call on this thread record these events (each a
    ``torch.cuda.Event`` already recorded once, so that its HIP event exists,
    or None) at the start and end of its element kernel and of its gather
    kernel (nsasm_set_kernel_events); no arguments cancel."""
    handles = []
    for ev in (element_start, element_stop, gather_start, gather_stop):
        if ev is None:
            handles.append(None)
            continue
        if not ev.cuda_event:
            raise ValueError("record the event once before passing it (its HIP event is created lazily)")
        handles.append(ev.cuda_event)
    _check(lib.nsasm_set_kernel_events(*handles))


class NSAssembleRHS(torch.autograd.Function):
    """rhs = NSAssembleRHS.apply(u, p, mesh, params); differentiable in u and p,
    in reverse mode (hand-written VJP kernels) and forward mode (the JVP
    kernel).  Element quantities are recomputed, never stored.  The backward
    is differentiable once: asking for a second-order derivative through it
    (create_graph=True, then another backward) raises instead of silently
    dropping the terms the kernels do not provide."""

    @staticmethod
    def forward(ctx, u, p, mesh, params):
        ctx.mesh, ctx.params = mesh, params
        u, p = u.contiguous(), p.contiguous()
        ctx.save_for_backward(u)
        ctx.save_for_forward(u)
        return assemble_rhs(mesh, u, p, params)

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, grad_rhs):
        (u,) = ctx.saved_tensors
        lam = grad_rhs.contiguous()
        gu = assemble_rhs_vjp(ctx.mesh, u, lam, ctx.params) if ctx.needs_input_grad[0] else None
        gp = assemble_rhs_vjp_p(ctx.mesh, lam, ctx.params) if ctx.needs_input_grad[1] else None
        return gu, gp, None, None

    @staticmethod
    def jvp(ctx, du, dp, _mesh_t, _params_t):
        (u,) = ctx.saved_tensors
        if du is None:
            du = torch.zeros_like(u)
        return assemble_rhs_jvp(ctx.mesh, u, du.contiguous(), None if dp is None else dp.contiguous(), ctx.params)


def version() -> str:
    return lib.nsasm_version().decode()
