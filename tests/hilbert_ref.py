"""Reference 3-D Hilbert index for the mesh-order tests (test code, not part of
the library): Skilling's transform of the axes into the curve's transposed
index (J. Skilling, "Programming the Hilbert curve", AIP Conf. Proc. 707,
2004), vectorised over points, and the element order the library promises:
elements sorted stably by the index of their centroid's cell on a 2^21 grid
over the bounding box's largest extent."""

import numpy as np

BITS = 21


def hilbert_index(cells: np.ndarray) -> np.ndarray:
    """(n, 3) integer cells in [0, 2^21) -> (n,) uint64 index along the curve."""
    x = [cells[:, i].astype(np.int64).copy() for i in range(3)]
    top = 1 << (BITS - 1)
    q = top
    while q > 1:
        lower = q - 1
        for i in range(3):
            set_ = (x[i] & q) != 0
            swap = (x[0] ^ x[i]) & lower
            x[0] = np.where(set_, x[0] ^ lower, x[0] ^ swap)
            if i:
                x[i] = np.where(set_, x[i], x[i] ^ swap)
        q >>= 1
    x[1] ^= x[0]
    x[2] ^= x[1]
    t = np.zeros_like(x[0])
    q = top
    while q > 1:
        t = np.where((x[2] & q) != 0, t ^ (q - 1), t)
        q >>= 1
    key = np.zeros(cells.shape[0], dtype=np.uint64)
    words = [(w ^ t).astype(np.uint64) for w in x]
    for b in range(BITS - 1, -1, -1):
        for w in words:
            key = (key << np.uint64(1)) | ((w >> np.uint64(b)) & np.uint64(1))
    return key


def element_order(coords: np.ndarray, conn: np.ndarray) -> np.ndarray:
    """User element index at each mesh position: the centroid of each element,
    in the library's rounding order, scaled onto the 2^21 grid of the bounding
    box's largest extent, then a stable sort by Hilbert index."""
    lo, hi = coords.min(axis=0), coords.max(axis=0)
    ext = max(hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2])
    scale = (2.0 ** BITS - 1.0) / ext if ext > 0 else 0.0
    x = coords[conn]
    cen = 0.25 * (((x[:, 0] + x[:, 1]) + x[:, 2]) + x[:, 3])
    q = np.minimum(np.maximum((cen - lo) * scale, 0.0), 2.0 ** BITS - 1.0).astype(np.uint64)
    return np.argsort(hilbert_index(q), kind="stable")
