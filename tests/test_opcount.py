"""The op-counting transcription of the literal element method (oracle/opcount.py)
and the algorithmic flop counts bench.py prices its roofline against.  CPU only."""

import numpy as np
import pytest

import oracle
from oracle import opcount
from paper_2403_08777_amd import synth


def test_counter_counts_each_operation_once():
    c = opcount.Counter()
    a, b = opcount.Counted(2.0, c), opcount.Counted(3.0, c)
    x = a * b + 1.0 - b / a  # mul, add, div, sub
    assert c.flops == 4 and abs(float(x) - 5.5) < 1e-15
    c.flops = 0
    y = -a                   # negation is free
    _ = 2.0 * 3.0            # constants alone are not counted
    assert c.flops == 0 and float(y) == -2.0
    # a 3x3 matrix-vector product written as sums of products: 9 mul + 6 add
    M = [[opcount.Counted(i + j, c) for j in range(3)] for i in range(3)]
    v = [opcount.Counted(k, c) for k in range(3)]
    _ = [M[i][0] * v[0] + M[i][1] * v[1] + M[i][2] * v[2] for i in range(3)]
    assert c.flops == 15


@pytest.mark.parametrize("cs", [0.0, 0.1])
def test_transcription_matches_the_c_oracle(oracle_lib, cs):
    m = synth.cube_mesh(2, jitter=True, permute=True)
    u, p = synth.taylor_green(m)
    lam = synth.adjoint(m.n_nodes)
    prm = oracle.Params(1.3, 1e-2, cs, synth.BODY_FORCE)
    r = np.array(opcount.assemble("rhs", m.coords, m.conn, u, p, 1.3, 1e-2, cs, synth.BODY_FORCE))
    g = np.array(opcount.assemble("vjp", m.coords, m.conn, u, lam, 1.3, 1e-2, cs))
    assert oracle.rel_l2(r, oracle.rhs(m.coords, m.conn, u, p, prm)) < 1e-14
    assert oracle.rel_l2(g, oracle.vjp(m.coords, m.conn, u, lam, prm)) < 1e-14


def test_bench_prices_the_counted_flops():
    import bench

    for kind in ("fwd", "vjp"):
        for eddy in (False, True):
            assert bench.ALGORITHMIC_FLOPS[(kind, eddy)] == opcount.flops_per_element(kind, eddy)
    # the eddy model only adds work; the VJP is the heavier call
    assert bench.ALGORITHMIC_FLOPS[("fwd", True)] > bench.ALGORITHMIC_FLOPS[("fwd", False)]
    assert bench.ALGORITHMIC_FLOPS[("vjp", False)] > bench.ALGORITHMIC_FLOPS[("fwd", True)]
