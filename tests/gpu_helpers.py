"""Shared helpers for the GPU tests: build a synthetic case, run the HIP path
through the Python binding, and run the oracle on the same inputs."""

from __future__ import annotations

import sys
from dataclasses import dataclass

import numpy as np
import torch

import oracle
from paper_2403_08777_amd import synth


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


@dataclass
class Case:
    n: int
    jitter: bool = False
    permute: bool = False
    mu: float = 1e-3
    cs: float = 0.0
    rho: float = 1.0
    model: str = "smagorinsky"
    form: str = "advective"

    def params(self):
        from paper_2403_08777_amd import api

        return api.Params(self.rho, self.mu, self.cs, synth.BODY_FORCE, self.model, self.form)

    def oracle_params(self):
        return oracle.Params(self.rho, self.mu, self.cs, synth.BODY_FORCE, model=self.model, form=self.form)

    def label(self):
        m = "" if self.model == "smagorinsky" else f" {self.model}"
        f = "" if self.form == "advective" else f" {self.form}"
        return f"n={self.n} jit={self.jitter} perm={self.permute} mu={self.mu} cs={self.cs}{m}{f}"


class Prepared:
    """Host inputs, the GPU mesh and mesh-ordered device fields of one case."""

    def __init__(self, case: Case, renumber=True, scatter="auto", patch_elems=0):
        from paper_2403_08777_amd import api

        self.case = case
        self.m = synth.cube_mesh(case.n, case.jitter, case.permute)
        self.u, self.p = synth.taylor_green(self.m)
        self.lam = synth.adjoint(self.m.n_nodes)
        dev = torch.device("cuda")
        self.mesh = api.Mesh(torch.from_numpy(self.m.coords).to(dev), torch.from_numpy(self.m.conn).to(dev),
                             renumber=renumber, scatter=scatter, patch_elems=patch_elems)
        self.dev = dev

    def fields(self, dtype):
        t = lambda a: self.mesh.to_mesh_order(torch.from_numpy(np.ascontiguousarray(a)).to(self.dev, dtype))
        return t(self.u), t(self.p), t(self.lam)

    def rhs(self, dtype=torch.float64):
        from paper_2403_08777_amd import api

        u, p, _ = self.fields(dtype)
        r = api.assemble_rhs(self.mesh, u, p, self.case.params())
        return self.mesh.from_mesh_order(r).double().cpu().numpy()

    def vjp(self, dtype=torch.float64):
        from paper_2403_08777_amd import api

        u, _, lam = self.fields(dtype)
        g = api.assemble_rhs_vjp(self.mesh, u, lam, self.case.params())
        return self.mesh.from_mesh_order(g).double().cpu().numpy()

    def oracle_rhs(self):
        return oracle.rhs(self.m.coords, self.m.conn, self.u, self.p, self.case.oracle_params())

    def oracle_vjp(self):
        return oracle.vjp(self.m.coords, self.m.conn, self.u, self.lam, self.case.oracle_params())
