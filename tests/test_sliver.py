"""A rounding-level sliver: four vertices on one plane up to the rounding of
their coordinates.  The exact determinant of the stored coordinates (exact
rational arithmetic) is non-zero but far below the rounding error of any
floating-point evaluation of det J, so the element must be refused by mesh
creation (the GPU test in test_gpu_mesh.py checks NSASM_ERR_DEGENERATE_ELEMENT);
a thin but sound element eight orders of magnitude above that bound must not be.
CPU only."""

from fractions import Fraction

import numpy as np

import oracle

EPS = np.finfo(np.float64).eps
REL_TOL = 64 * EPS  # the library's bound on |det J| / (|d1||d2||d3|)


def _exact_det_ratio(xe):
    """|det J| / (|d1||d2||d3|) with det J exact for the stored doubles."""
    q = [[Fraction(float(v)) for v in row] for row in xe]
    d = [[q[k + 1][i] - q[0][i] for i in range(3)] for k in range(3)]
    det = (d[0][0] * (d[1][1] * d[2][2] - d[1][2] * d[2][1]) - d[0][1] * (d[1][0] * d[2][2] - d[1][2] * d[2][0])
           + d[0][2] * (d[1][0] * d[2][1] - d[1][1] * d[2][0]))
    lens = np.prod([np.sqrt(float(sum(c * c for c in row))) for row in d])
    return abs(det), float(abs(det)) / lens


def sliver_coords():
    """Vertices x0..x2 of a general triangle and x3 = x0 + a (x1 - x0) + b (x2 - x0)
    evaluated in doubles, for the first (a, b) whose stored result is off the
    plane (exact det != 0)."""
    x0 = np.array([0.1, 0.2, 0.3])
    x1 = np.array([1.3, 0.4, 0.2])
    x2 = np.array([0.2, 1.1, 0.7])
    for k in range(1, 200):
        a, b = 0.3 + 0.001 * k, 0.45 - 0.0007 * k
        x3 = x0 + a * (x1 - x0) + b * (x2 - x0)
        xe = np.array([x0, x1, x2, x3])
        det, _ = _exact_det_ratio(xe)
        if det != 0:
            return xe
    raise AssertionError("no off-plane rounding found")


def thin_coords(rel=1e-6):
    """A sound element whose |det J| / (|d1||d2||d3|) is about rel."""
    xe = sliver_coords().copy()
    nrm = np.cross(xe[1] - xe[0], xe[2] - xe[0])
    xe[3] = xe[3] + rel * 2.0 * nrm / np.linalg.norm(nrm)
    return xe


def test_sliver_is_flat_to_rounding():
    det, ratio = _exact_det_ratio(sliver_coords())
    assert det != 0 and ratio < 1e-2 * REL_TOL


def test_thin_element_is_well_above_the_bound(oracle_lib):
    xe = thin_coords()
    _, ratio = _exact_det_ratio(xe)
    assert ratio > 1e6 * REL_TOL
    # the oracle's volume of it agrees with the exact determinant to rounding
    vol, _ = oracle.geometry(xe, np.array([[0, 1, 2, 3]], dtype=np.int32))
    det, _ = _exact_det_ratio(xe)
    assert abs(vol[0] - float(det) / 6) <= 1e-5 * float(det) / 6
