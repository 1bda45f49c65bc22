"""C-ABI boundary on the host: the library loads, exports every declared entry
point, its struct layouts match the Python binding, and host-side argument
checks return the documented status without touching a GPU."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nsasm.h")
LIB = os.path.join(ROOT, "paper_2403_08777_amd", "libnsasm.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libnsasm.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nsasm_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 11
    lib = ctypes.CDLL(LIB)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\b(nsasm_[a-z_]+)\b", out))
    assert set(names) <= exported


def test_struct_layout_matches_header(tmp_path):
    """Compile a C probe against the header and compare sizes/offsets with the
    ctypes structs the binding uses."""
    from paper_2403_08777_amd import api

    src = tmp_path / "probe.c"
    src.write_text(r'''
#include <stddef.h>
#include <stdio.h>
#include "nsasm.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(nsasm_params), offsetof(nsasm_params, body_force),
         offsetof(nsasm_params, flags), offsetof(nsasm_params, eddy_model),
         offsetof(nsasm_params, convective_form), offsetof(nsasm_params, reserved));
  printf("%zu %zu %zu\n", sizeof(nsasm_mesh_options), offsetof(nsasm_mesh_options, scatter),
         offsetof(nsasm_mesh_options, patch_elems));
  printf("%zu %zu %zu\n", sizeof(nsasm_mesh_info_t), offsetof(nsasm_mesh_info_t, scatter),
         offsetof(nsasm_mesh_info_t, patch_node_refs));
  return 0;
}
''')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", f"-I{os.path.dirname(HEADER)}", str(src), "-o", str(exe)], check=True)
    lines = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    p = [int(v) for v in lines[0].split()]
    assert p == [ctypes.sizeof(api._Params), api._Params.body_force.offset, api._Params.flags.offset,
                 api._Params.eddy_model.offset, api._Params.convective_form.offset, api._Params.reserved.offset]
    o = [int(v) for v in lines[1].split()]
    assert o == [ctypes.sizeof(api._MeshOptions), api._MeshOptions.scatter.offset,
                 api._MeshOptions.patch_elems.offset]
    i = [int(v) for v in lines[2].split()]
    assert i == [ctypes.sizeof(api._MeshInfo), api._MeshInfo.scatter.offset, api._MeshInfo.patch_node_refs.offset]


def test_host_side_argument_checks():
    from paper_2403_08777_amd import api

    lib = api.lib
    h = ctypes.c_void_p(1234)
    dummy = ctypes.c_void_p(0x1000)
    # out == NULL
    assert lib.nsasm_mesh_create(dummy, 8, dummy, 1, None, None, None) == 1
    assert b"out" in lib.nsasm_last_error()
    # NULL inputs: out is cleared
    assert lib.nsasm_mesh_create(None, 8, dummy, 1, None, None, ctypes.byref(h)) == 1
    assert h.value is None
    assert lib.nsasm_mesh_create(dummy, 8, None, 1, None, None, ctypes.byref(h)) == 1
    # sizes
    assert lib.nsasm_mesh_create(dummy, 0, dummy, 1, None, None, ctypes.byref(h)) == 1
    assert lib.nsasm_mesh_create(dummy, 8, dummy, 0, None, None, ctypes.byref(h)) == 1
    assert lib.nsasm_mesh_create(dummy, 8, dummy, 1 << 29, None, None, ctypes.byref(h)) == 1
    assert lib.nsasm_mesh_create(dummy, 1 << 31, dummy, 1, None, None, ctypes.byref(h)) == 1
    # options
    for opts in (api._MeshOptions(2, 0, 0, 0), api._MeshOptions(1, 4, 0, 0), api._MeshOptions(1, 0, 48, 0),
                 api._MeshOptions(1, 0, 512, 0), api._MeshOptions(1, 0, 0, 7)):
        assert lib.nsasm_mesh_create(dummy, 8, dummy, 1, ctypes.byref(opts), None, ctypes.byref(h)) == 1
    # NULL mesh everywhere
    prm = api.Params().c_struct()
    assert lib.nsasm_assemble_rhs(None, ctypes.byref(prm), 0, dummy, dummy, dummy, None) == 1
    assert lib.nsasm_assemble_rhs_vjp(None, ctypes.byref(prm), 0, dummy, dummy, dummy, None) == 1
    assert lib.nsasm_mesh_info(None, None) == 1
    assert lib.nsasm_mesh_permutation(None, dummy, None) == 1
    assert lib.nsasm_mesh_connectivity(None, None, None, None) == 1
    assert lib.nsasm_to_mesh_order(None, 3, 0, dummy, dummy, None) == 1
    assert lib.nsasm_from_mesh_order(None, 3, 0, dummy, dummy, None) == 1
    assert lib.nsasm_last_error()
    # the Scale kernel: n < 0 is an error, n == 0 does nothing, NULL arrays are errors
    assert lib.nsasm_stream_scale(None, None, -1, 2.0, None) == 1
    assert lib.nsasm_stream_scale(None, None, 0, 2.0, None) == 0
    assert lib.nsasm_stream_scale(None, None, 5, 2.0, None) == 1 and b"a is NULL" in lib.nsasm_last_error()
    assert lib.nsasm_mesh_destroy(None) == 0
    assert api.version() == "0.2.0"


def test_error_class():
    from paper_2403_08777_amd import api

    e = api.NsasmError(3, "x")
    assert e.status_name == "DEGENERATE_ELEMENT" and "DEGENERATE_ELEMENT" in str(e)


def test_binding_rejects_host_tensors_before_the_library():
    """The Python binding validates tensors itself: host tensors, wrong dtypes
    and shapes raise before any library call."""
    import torch

    from paper_2403_08777_amd import api

    coords = torch.zeros((4, 3), dtype=torch.float64)
    conn = torch.tensor([[0, 1, 2, 3]], dtype=torch.int32)
    with pytest.raises(ValueError, match="CUDA"):
        api.Mesh(coords, conn)
    with pytest.raises(ValueError, match="scatter"):
        api.Mesh(coords, conn, scatter="colour")
    with pytest.raises(KeyError):
        api.Params(eddy_model="wale").c_struct()
    with pytest.raises(KeyError):
        api.Params(convective_form="upwind").c_struct()
    prm = api.Params(convective_form="emac", eddy_model="vreman").c_struct(accumulate=True)
    assert prm.convective_form == 4 and prm.eddy_model == 1 and prm.flags == 1 and prm.reserved == 0
