"""The HIP path through the C-ABI against the stored exact result
tests/golden/cube2_exact.txt, in every scatter strategy: FP64 to 1e-12
relative L2, mixed precision to 1e-5."""

import numpy as np
import pytest
import torch

import oracle
from tests.golden.make_cube2_exact import load
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu

G = load()


def as_np(rows):
    return np.array([[float(v) for v in r] if isinstance(r, list) else float(r) for r in rows])


@pytest.mark.parametrize("scatter", ["atomic", "patch", "patch_gather"])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_gpu_matches_exact_fixture(scatter, dtype, tol):
    from paper_2403_08777_amd import api

    dev = torch.device("cuda")
    mesh = api.Mesh(torch.from_numpy(as_np(G["x"])).to(dev),
                    torch.tensor(G["conn"], dtype=torch.int32, device=dev), scatter=scatter)
    rho, mu, f = float(G["rho"]), float(G["mu"]), [float(v) for v in G["f"]]
    prm = api.Params(rho, mu, 0.0, f)
    emac = api.Params(rho, mu, 0.0, f, convective_form="emac")
    dm = lambda k: mesh.to_mesh_order(torch.from_numpy(as_np(G[k])).to(dev, dtype))
    um = lambda t: mesh.from_mesh_order(t).double().cpu().numpy()
    u, p, lam, du, dp = (dm(k) for k in ("u", "p", "lam", "du", "dp"))
    got = {
        "rhs": um(api.assemble_rhs(mesh, u, p, prm)),
        "rhs_emac": um(api.assemble_rhs(mesh, u, p, emac)),
        "vjp": um(api.assemble_rhs_vjp(mesh, u, lam, prm)),
        "vjp_p": um(api.assemble_rhs_vjp_p(mesh, lam, prm)),
        "jvp": um(api.assemble_rhs_jvp(mesh, u, du, dp, prm)),
    }
    for name, val in got.items():
        err = oracle.rel_l2(val, as_np(G[name]))
        log(f"golden cube2 {scatter} {str(dtype)[6:]} {name}: rel_l2 {err:.2e}")
        assert err <= tol, name
    mesh.close()
