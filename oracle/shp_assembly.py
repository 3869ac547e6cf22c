"""Oracle (test infrastructure only) for the C0-assembled Helmholtz problem on a
structured grid of hexahedra: the local-to-global map, the assembled sparse
operator from the oracle's dense elemental matrices, and a sparse direct
solve.  Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg use
this module; it shares no code with the library.

The global problem of Sec. 2.1 joins the elemental systems H^e u^e = f^e with a
local-to-global map A: the global operator is A^T H A and the global right-hand
side A^T f.  On a grid whose elements all have their reference axes along the
grid directions, the modified basis in one direction has per cell two vertex
functions (shared with the neighbouring cells) and P - 1 bubbles (its own), and
a hexahedral mode is the tensor product of one such function per direction.
With homogeneous Dirichlet data the functions of the two boundary vertices of
each line are dropped.

Numbering (the documented line order): walking a line from its first cell to
its last, each cell contributes its left vertex, then its bubbles; the last
cell's right vertex closes the line.  Dirichlet drops the first and last
vertex.  A 3D index is (g0 m1 + g1) m2 + g2, m_d the count along direction d.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import shp_oracle as O


def line_numbering(ncell: int, P: int, dirichlet: bool = True):
    """{('v', vertex) | ('b', cell, bubble): global line index}, and the count."""
    ids = {}
    k = 0
    for c in range(ncell):
        for key in [("v", c)] + [("b", c, b) for b in range(P - 1)]:
            if dirichlet and key == ("v", 0):
                continue
            ids[key] = k
            k += 1
    if not dirichlet:
        ids[("v", ncell)] = k
        k += 1
    return ids, k


def _line_key(c: int, a: int):
    """The 1D function of local index a (0: A_0, 1: A_1, >= 2: bubble) of cell c."""
    if a == 0:
        return ("v", c)
    if a == 1:
        return ("v", c + 1)
    return ("b", c, a - 2)


def hex_grid_map(n0: int, n1: int, n2: int, P: int, dirichlet: bool = True):
    """l2g [n_elem][N_P] (int64, -1 for dropped DOFs) and the number of global
    DOFs.  Element e = (i0 n1 + i1) n2 + i2; local mode (p, q, r) at
    (p n + q) n + r, n = P + 1."""
    lines = [line_numbering(nc, P, dirichlet) for nc in (n0, n1, n2)]
    m = [cnt for _, cnt in lines]
    n = P + 1
    per_dir = []
    for d, nc in enumerate((n0, n1, n2)):
        ids = lines[d][0]
        tab = np.full((nc, n), -1, dtype=np.int64)
        for c in range(nc):
            for a in range(n):
                tab[c, a] = ids.get(_line_key(c, a), -1)
        per_dir.append(tab)
    i0, i1, i2 = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij")
    g0 = per_dir[0][i0.ravel()]  # [n_elem, n]
    g1 = per_dir[1][i1.ravel()]
    g2 = per_dir[2][i2.ravel()]
    G = (g0[:, :, None, None] * m[1] + g1[:, None, :, None]) * m[2] + g2[:, None, None, :]
    dropped = (g0[:, :, None, None] < 0) | (g1[:, None, :, None] < 0) | (g2[:, None, None, :] < 0)
    G = np.where(dropped, -1, G)
    return G.reshape(len(g0), n ** 3), m[0] * m[1] * m[2]


def assemble(mats: np.ndarray, l2g: np.ndarray, n_global: int) -> sp.csr_matrix:
    """A^T blockdiag(mats) A: sum over elements of mats[e] at the rows and
    columns l2g[e] (dropped DOFs left out)."""
    ne, NP, _ = mats.shape
    rows = np.repeat(l2g[:, :, None], NP, axis=2)
    cols = np.repeat(l2g[:, None, :], NP, axis=1)
    keep = (rows >= 0) & (cols >= 0)
    return sp.coo_matrix((mats[keep], (rows[keep], cols[keep])), shape=(n_global, n_global)).tocsr()


def assemble_vector(v: np.ndarray, l2g: np.ndarray, n_global: int) -> np.ndarray:
    """A^T v for local vectors v [n_elem][N_P]."""
    out = np.zeros(n_global)
    keep = l2g >= 0
    np.add.at(out, l2g[keep], v[keep])
    return out


def element_matrices(P: int, jac: np.ndarray, kind: str, lam: float = 1.0, chunk: int = 256) -> np.ndarray:
    """Dense elemental matrices of the hexahedra: 'mass', 'laplacian' or
    'helmholtz' (lam M + L)."""
    out = []
    for e0 in range(0, jac.shape[0], chunk):
        el = O.Element("hex", P, P + 2, jac[e0:e0 + chunk])
        out.append(el.mass() if kind == "mass" else el.laplacian() if kind == "laplacian" else el.helmholtz(lam))
    return np.concatenate(out, axis=0)


def solve(H: sp.csr_matrix, b: np.ndarray) -> np.ndarray:
    """Sparse direct solve of the assembled system."""
    return spla.spsolve(H.tocsc(), b)
