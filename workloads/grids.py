"""Structured-grid helpers: node counts and stimulus masks built from integer
indices (never from floating-point coordinates), so that every consumer sees
exactly the same set of stimulated nodes.

Node ordering is lexicographic with x fastest: node (i, j, k) has flat index
``i + n0 * (j + n1 * k)``.
"""
import math

import numpy as np


def grid_num_nodes(n):
    return int(np.prod([int(v) for v in n]))


def _max_index(width, h):
    # largest integer k with k*h <= width, evaluated with a relative slack of
    # 1e-9*h so that e.g. width=1.5, h=0.1 keeps k=15
    return int(math.floor(width / h + 1e-9))


def box_mask(n, h, width):
    """uint8 mask of nodes with ||x||_inf <= width, x measured from the origin
    corner (x = index * h per axis)."""
    n = [int(v) for v in n]
    kmax = [_max_index(width, hh) for hh in h]
    axes = [np.arange(nn) <= km for nn, km in zip(n, kmax)]
    m = axes[0]
    for a in axes[1:]:
        m = np.logical_and.outer(a, m)  # later axes become slower indices
    return np.ascontiguousarray(m.reshape(-1)).astype(np.uint8)


def face_mask(n, h, axis, width):
    """uint8 mask of nodes with x_axis <= width (a slab on the x_axis=0 face)."""
    n = [int(v) for v in n]
    km = _max_index(width, h[axis])
    idx = np.indices(n[::-1])[::-1]  # idx[d] has shape (n_{D-1},...,n_0)
    m = idx[axis] <= km
    return np.ascontiguousarray(m.reshape(-1)).astype(np.uint8)
