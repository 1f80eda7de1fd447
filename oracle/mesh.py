"""Oracle: structured-box topology (TEST INFRASTRUCTURE, see ``oracle/__init__.py``).

Global nodes of an n_1 x ... x n_d box of order p are numbered
lexicographically on the (n_k p + 1) grid, first axis fastest; the vector
layout is SoA by component (x[c*N_x + g]).  Local element nodes follow the
paper's lexicographic order i = i1 + n_i i2 + n_i^2 i3 (Sec. 3.1, 0-based).
The paper fixes only the local ordering; the global numbering is this
build's convention.
"""
import itertools

import numpy as np


def box_topology(dim, ns, p):
    """(e2n int32 (E, (p+1)^dim), N_x) for the structured box.

    Element e = e_0 + n_0 (e_1 + n_1 e_2) and local node i = i_0 + n_i (i_1 + n_i i_2);
    local node i of element e is grid point g_k = e_k p + i_k on each axis k.
    """
    ni = p + 1
    M = [n * p + 1 for n in ns]
    nx = int(np.prod(M))
    strides = [int(np.prod(M[:k])) for k in range(dim)]
    # E[k, e] = e_k and I[k, i] = i_k, first axis fastest
    E = np.indices(tuple(ns[::-1])).reshape(dim, -1)[::-1]
    I = np.indices((ni,) * dim).reshape(dim, -1)[::-1]
    g = np.zeros((E.shape[1], I.shape[1]), dtype=np.int64)
    for k in range(dim):
        g += (E[k][:, None] * p + I[k][None, :]) * strides[k]
    return g.astype(np.int32), nx


def box_boundary_mask(dim, ns, p):
    """Boolean mask (dim*N_x): True for every component of every node on the box boundary."""
    M = [n * p + 1 for n in ns]
    on = np.zeros(M[::-1], dtype=bool)  # index order (g_{d-1}, ..., g_0)
    for k in range(dim):
        ax = dim - 1 - k
        sl = [slice(None)] * dim
        sl[ax] = 0
        on[tuple(sl)] = True
        sl[ax] = M[k] - 1
        on[tuple(sl)] = True
    flat = on.ravel()
    return np.tile(flat, dim)


def dof_count(dim, n, p):
    """Unique DoFs d*(n p + 1)^d of a structured n^d box of order p."""
    return dim * (n * p + 1) ** dim


def grid_index(ns, p, coords):
    """Global node index of grid coordinates (g_0, ..., g_{d-1})."""
    M = [n * p + 1 for n in ns]
    g = 0
    s = 1
    for k, c in enumerate(coords):
        g += c * s
        s *= M[k]
    return g


def all_grid_coords(ns, p):
    M = [n * p + 1 for n in ns]
    return list(itertools.product(*[range(m) for m in M[::-1]]))
