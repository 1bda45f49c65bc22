"""nsasm: MI355X-native element-by-element assembly of the incompressible
Navier-Stokes momentum right-hand side over linear tetrahedra.

The compute path is the HIP library ``libnsasm.so`` (C ABI, ``include/nsasm.h``);
this package only marshals arguments to it.  Importing the GPU-facing names
(``Mesh``, ``assemble_rhs``, ...) loads the library and fails loudly if it has not
been built.  ``synth`` (synthetic inputs) needs only numpy.
"""

__version__ = "0.2.0"

_LAZY = {
    "Mesh": "api", "Params": "api", "assemble_rhs": "api", "assemble_rhs_vjp": "api",
    "NSAssembleRHS": "api", "FP64": "api", "MIXED": "api", "stream_scale": "api",
}


def __getattr__(name):
    mod = _LAZY.get(name)
    if mod is None:
        raise AttributeError(name)
    import importlib

    return getattr(importlib.import_module(f"{__name__}.{mod}"), name)
