"""Pins of the reference Hilbert index the mesh-order GPU test compares the
library with: it must be a bijection onto consecutive integers on every
aligned block and step between face-adjacent cells, which is what defines a
Hilbert curve (a Morton or other order fails the adjacency check)."""

import numpy as np

from tests.hilbert_ref import hilbert_index


def _block(n, origin=(0, 0, 0)):
    g = np.stack(np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij"), -1).reshape(-1, 3)
    return (g + np.asarray(origin)).astype(np.uint64)


def test_first_block_is_the_curve_start():
    cells = _block(8)
    key = hilbert_index(cells)
    assert np.array_equal(np.sort(key), np.arange(512, dtype=np.uint64))
    path = cells[np.argsort(key)].astype(np.int64)
    assert np.all(np.abs(np.diff(path, axis=0)).sum(axis=1) == 1)
    assert np.array_equal(path[0], [0, 0, 0])


def test_aligned_blocks_are_contiguous_and_adjacent():
    for origin in ((32, 16, 48), (2**20, 0, 2**20 + 2**19), (2**21 - 16, 2**21 - 16, 2**21 - 16)):
        cells = _block(16, origin)
        key = np.sort(hilbert_index(cells))
        assert key[-1] - key[0] == 16**3 - 1 and len(np.unique(key)) == 16**3
        path = cells[np.argsort(hilbert_index(cells))].astype(np.int64)
        assert np.all(np.abs(np.diff(path, axis=0)).sum(axis=1) == 1)


def test_whole_curve_ends():
    corners = np.array([[0, 0, 0], [2**21 - 1, 0, 0]], dtype=np.uint64)
    key = hilbert_index(corners)
    assert key[0] == 0 and key[1] == np.uint64(2**63 - 1)
