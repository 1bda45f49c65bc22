"""The largest mesh the library accepts: exactly 2^29 - 1 tetrahedra (the
n_elems limit), with 64-bit byte offsets in every element array, a ragged
last patch (255 elements), randomly relabelled node ids and unreferenced
nodes (the lattice is cut inside its top cell layers).  The mesh is built on
the GPU with torch; the FP64 forward and VJP are checked at sampled nodes
against the oracle run on the sub-mesh of the elements around them (a node's
value depends only on its own elements), and unreferenced nodes must come out
exactly zero; then the same in mixed precision, within 1e-5 of the FP64
oracle."""

import numpy as np
import pytest
import torch

import oracle
from tests.gpu_helpers import log

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N = 448                    # lattice cells per side: 6 N^3 = 539,492,352 >= the limit
NE = (1 << 29) - 1         # the largest n_elems nsasm_mesh_create accepts
RHO, MU, CS, F = 1.0, 1e-4, 0.1, (0.1, -0.2, 0.3)


def _lattice_conn(dev):
    """Cell-major Kuhn tetrahedra of the (N+1)^3 lattice (6 per cell, the axis
    permutations in lexicographic order), lattice node ids, cut to NE."""
    n1 = N + 1
    e = (1, n1, n1 * n1)
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    offs = torch.tensor([[0, e[s[0]], e[s[0]] + e[s[1]], sum(e)] for s in perms], dtype=torch.int64, device=dev)
    conn = torch.empty((NE, 4), dtype=torch.int32, device=dev)
    ncell = (NE + 5) // 6
    chunk = 1 << 24
    for c0 in range(0, ncell, chunk):
        c = torch.arange(c0, min(c0 + chunk, ncell), device=dev, dtype=torch.int64)
        v = c % N + n1 * ((c // N) % N + n1 * (c // (N * N)))
        blk = (v[:, None, None] + offs[None]).reshape(-1, 4)
        e0 = 6 * c0
        e1 = min(e0 + blk.shape[0], NE)
        conn[e0:e1] = blk[: e1 - e0].to(torch.int32)
        del c, v, blk
    return conn


def _incident(conn, node):
    return torch.nonzero((conn == node).any(dim=1)).squeeze(1)


def test_maximum_element_count():
    from paper_2403_08777_amd import api

    dev = torch.device("cuda")
    g = torch.Generator(device=dev).manual_seed(29)
    n1 = N + 1
    nn = n1 ** 3
    log(f"max-size mesh: {NE} tets, {nn} nodes")
    conn_lat = _lattice_conn(dev)
    assert int(conn_lat.max()) < nn and int(conn_lat.min()) >= 0
    perm = torch.randperm(nn, device=dev, generator=g)
    conn = perm.to(torch.int32).index_select(0, conn_lat.view(-1)).view(NE, 4)
    del conn_lat
    lat = torch.arange(nn, device=dev, dtype=torch.int64)
    xl = torch.stack([lat % n1, (lat // n1) % n1, lat // (n1 * n1)], dim=1).to(torch.float64) / N
    del lat
    xl += (torch.rand(xl.shape, generator=g, device=dev, dtype=torch.float64) * 0.4 - 0.2) / N
    coords = torch.empty_like(xl)
    coords[perm] = xl
    del xl
    u = torch.randn((nn, 3), generator=g, device=dev, dtype=torch.float64)
    p = torch.randn((nn,), generator=g, device=dev, dtype=torch.float64)
    lam = torch.randn((nn, 3), generator=g, device=dev, dtype=torch.float64)
    torch.cuda.synchronize()

    mesh = api.Mesh(coords, conn)
    log(f"mesh info {mesh.info}")
    assert mesh.n_elems == NE and mesh.n_nodes == nn
    prm = api.Params(RHO, MU, CS, F)
    rhs = mesh.from_mesh_order(api.assemble_rhs(mesh, mesh.to_mesh_order(u), mesh.to_mesh_order(p), prm))
    grad = mesh.from_mesh_order(api.assemble_rhs_vjp(mesh, mesh.to_mesh_order(u), mesh.to_mesh_order(lam), prm))
    torch.cuda.synchronize()
    log("assembled; sampling")

    # sampled nodes: random lattice nodes, the nodes of the first and last
    # elements (the last sits in the ragged last patch), and top-layer nodes
    # (some of which the cut leaves without elements)
    rng = np.random.default_rng(29)
    lat_samples = list(rng.integers(0, nn, 24)) + list(n1 * n1 * N + rng.integers(0, n1 * n1, 24))
    perm_h = perm.cpu().numpy()
    samples = sorted(set(int(perm_h[s]) for s in lat_samples)
                     | set(conn[0].cpu().tolist()) | set(conn[NE - 1].cpu().tolist()))
    elems, unreferenced = [], []
    for s in samples:
        idx = _incident(conn, s)
        if idx.numel() == 0:
            unreferenced.append(s)
        else:
            elems.append(idx)
    log(f"{len(samples)} sampled nodes, {len(unreferenced)} without elements")
    assert unreferenced, "the cut top layer should leave some sampled nodes without elements"
    referenced = [s for s in samples if s not in unreferenced]
    un = torch.tensor(unreferenced, device=dev, dtype=torch.int64)
    assert torch.all(rhs[un] == 0) and torch.all(grad[un] == 0)

    e_idx = torch.unique(torch.cat(elems))
    sub = conn.index_select(0, e_idx).cpu().numpy().astype(np.int64)
    nodes, local = np.unique(sub, return_inverse=True)
    local = local.reshape(sub.shape).astype(np.int32)
    nidx = torch.from_numpy(nodes).to(dev)
    x_s, u_s, p_s, l_s = (t.index_select(0, nidx).cpu().numpy() for t in (coords, u, p, lam))
    oprm = oracle.Params(RHO, MU, CS, F)
    pos = np.searchsorted(nodes, referenced)
    ref_r = oracle.rhs(x_s, local, u_s, p_s, oprm)[pos]
    ref_g = oracle.vjp(x_s, local, u_s, l_s, oprm)[pos]
    ridx = torch.tensor(referenced, device=dev, dtype=torch.int64)
    got_r = rhs[ridx].cpu().numpy()
    got_g = grad[ridx].cpu().numpy()
    er, eg = oracle.rel_l2(got_r, ref_r), oracle.rel_l2(got_g, ref_g)
    log(f"max-size sampled {len(referenced)} nodes over {len(e_idx)} elements: rhs rel_l2 {er:.2e}, vjp {eg:.2e}")
    assert er <= 1e-12 and eg <= 1e-12

    # mixed precision on the same mesh: FP32 fields, error against the FP64 oracle
    del rhs, grad
    u32, p32, l32 = (mesh.to_mesh_order(t.float()) for t in (u, p, lam))
    r32 = mesh.from_mesh_order(api.assemble_rhs(mesh, u32, p32, prm))
    g32 = mesh.from_mesh_order(api.assemble_rhs_vjp(mesh, u32, l32, prm))
    assert torch.all(r32[un] == 0) and torch.all(g32[un] == 0)
    mr = oracle.rel_l2(r32[ridx].double().cpu().numpy(), ref_r)
    mg = oracle.rel_l2(g32[ridx].double().cpu().numpy(), ref_g)
    log(f"max-size mixed: rhs rel_l2 {mr:.2e}, vjp {mg:.2e}")
    assert mr <= 1e-5 and mg <= 1e-5
    mesh.close()
