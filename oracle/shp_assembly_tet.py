"""Oracle (test infrastructure only) for C0 assembly on a conforming
tetrahedral mesh: the local-to-global map with its sign changes, found from the
traces of the modes on the mesh's shared vertices, edges and faces; the
assembled operator A^T H A from the oracle's dense elemental matrices; and a
sparse direct solve.  Only tests/ use this module; it shares no code with the
library.

The global problem of Sec. 2.1 joins the elemental systems through a
local-to-global map A.  With the modified basis, a mode of a tetrahedron is
either one at a vertex, or supported on one edge, one face, or the interior
(the boundary-interior split of the C0 expansion).  A global DOF is a function
on the mesh: one per vertex, P - 1 per edge, (P - 1)(P - 2)/2 per face and
(P - 1)(P - 2)(P - 3)/6 per element interior.  Its canonical form on an edge
with end vertices lo < hi (global ids) is A_k(t), k = 2..P, with t running
from -1 at lo to +1 at hi; on a face with vertices lo < mid < hi it is
A_p(a) C_{p,q}(b), p >= 2, q >= 1, p + q <= P, in the face's collapsed
coordinates (b = -1 on the edge lo-mid and b = +1 at hi; a from -1 at lo to
+1 at mid).  A local mode is matched to the canonical functions of its entity
by its values at sample points of that entity: the fit must give one
canonical function with coefficient +1 or -1, which is the sign of the local
copy.

This identification uses nothing but the oracle's own basis functions
evaluated at points: no rule of which (p, q, r) lies on which entity.

Numbering (the documented order, shared with the library's map): interior
vertices by increasing id; interior edges by (lo, hi), then k; interior faces
by (lo, mid, hi), then (p, q) lexicographically; then the element interiors,
element by element in local mode order.  Faces that belong to one element are
the Dirichlet boundary: the DOFs of their vertices, edges and the faces
themselves are dropped.

Encoding of the sign (the library's convention): l2g = g for a copy with sign
+1, -2 - g for sign -1, -1 for a dropped DOF; in the CSR lists, local index i
or -1 - i.
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import shp_oracle as O

# reference vertices of the tetrahedron
REF_V = np.array([[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0], [-1.0, -1.0, 1.0]])


def eta_of_xi(xi: np.ndarray) -> np.ndarray:
    """Inverse of the tet's collapse map; on a collapsed line or point the free
    collapsed coordinate is set to 0 (the modes are single-valued there)."""
    x1, x2, x3 = xi[:, 0], xi[:, 1], xi[:, 2]
    e3 = x3
    d2 = 1.0 - x3
    e2 = np.where(d2 > 1e-13, 2.0 * (1.0 + x2) / np.where(d2 > 1e-13, d2, 1.0) - 1.0, 0.0)
    d1 = -x2 - x3
    e1 = np.where(d1 > 1e-13, 2.0 * (1.0 + x1) / np.where(d1 > 1e-13, d1, 1.0) - 1.0, 0.0)
    return np.stack([e1, e2, e3], axis=1)


def modes_at(P: int, bary: np.ndarray, local: np.ndarray) -> np.ndarray:
    """Values [n_pts, N_P] of the element's modes at the points with
    barycentric weights bary [n_pts, k] on its local vertices local [k]."""
    xi = bary @ REF_V[local]
    return O.basis("tet", P, eta_of_xi(xi))[0]


def _edge_samples(P: int):
    t = np.cos(np.pi * (np.arange(P + 3) + 0.5) / (P + 3))   # distinct interior points
    return t


def _face_samples(P: int):
    g = np.cos(np.pi * (np.arange(P + 2) + 0.5) / (P + 2))
    a, b = np.meshgrid(g, g, indexing="ij")
    return a.ravel(), b.ravel()


def _face_modes(P: int):
    return [(p, q) for p in range(2, P + 1) for q in range(1, P + 1 - p)]


def _match(vals: np.ndarray, basis_vals: np.ndarray, what: str):
    """The signed unit vector c with basis_vals @ c = vals: (index, sign)."""
    c, *_ = np.linalg.lstsq(basis_vals, vals, rcond=None)
    j = int(np.argmax(np.abs(c)))
    s = 1 if c[j] > 0 else -1
    e = np.zeros_like(c)
    e[j] = s
    if np.abs(c - e).max() > 1e-9 or np.abs(basis_vals @ e - vals).max() > 1e-9:
        raise AssertionError(f"{what}: trace is not one canonical function ({c})")
    return j, s


@functools.lru_cache(maxsize=None)
def _classify_ranked(P: int, ranks: tuple):
    """classify() for vertex ids whose order is given by ranks (rank of each
    local vertex among the four); entities in local vertex indices."""
    gids = np.array(ranks)
    NP = O.num_modes("tet", P)
    ent = [None] * NP
    sign = np.ones(NP, dtype=np.int64)
    # vertices: each vertex mode is one at its own vertex and zero at the others
    Bv = modes_at(P, np.eye(4), np.arange(4))                      # [4, NP]
    for m in range(NP):
        nz = np.flatnonzero(np.abs(Bv[:, m]) > 1e-12)
        if len(nz):
            assert len(nz) == 1 and abs(Bv[nz[0], m] - 1.0) < 1e-12, (m, Bv[:, m])
            ent[m] = ("v", int(nz[0]))
    # edges, in the canonical parameter from the lower to the higher id
    t = _edge_samples(P)
    canon_e = np.stack([O.fA(k, t) for k in range(2, P + 1)], axis=1) if P >= 2 else None
    for a in range(4):
        for b in range(a + 1, 4):
            lo, hi = (a, b) if gids[a] < gids[b] else (b, a)
            bary = np.stack([(1 - t) / 2, (1 + t) / 2], axis=1)
            Be = modes_at(P, bary, np.array([lo, hi]))
            for m in range(NP):
                if ent[m] is not None or np.abs(Be[:, m]).max() < 1e-12:
                    continue
                j, s = _match(Be[:, m], canon_e, f"edge mode {m}")
                ent[m] = ("e", (lo, hi), j + 2)
                sign[m] = s
    # faces, in the canonical collapsed coordinates of (lo, mid, hi)
    fa, fb = _face_samples(P)
    fm = _face_modes(P)
    canon_f = np.stack([O.fA(p, fa) * O.fC(p, q, fb) for p, q in fm], axis=1) if fm else None
    for tri in ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)):
        lo, mid, hi = sorted(tri, key=lambda v: gids[v])
        lhi = (1 + fb) / 2
        lmid = (1 - lhi) * (1 + fa) / 2
        bary = np.stack([1 - lhi - lmid, lmid, lhi], axis=1)
        Bf = modes_at(P, bary, np.array([lo, mid, hi]))
        for m in range(NP):
            if ent[m] is not None or np.abs(Bf[:, m]).max() < 1e-12:
                continue
            j, s = _match(Bf[:, m], canon_f, f"face mode {m}")
            ent[m] = ("f", (lo, mid, hi), fm[j])
            sign[m] = s
    for m in range(NP):
        if ent[m] is None:
            ent[m] = ("i",)
    return tuple(ent), sign


def classify(P: int, gids: np.ndarray):
    """For one element with global vertex ids gids [4] in local order: per
    local mode, ('v', id) | ('e', (lo, hi), k) | ('f', (lo, mid, hi), (p, q)) |
    ('i',), and the sign of the local copy.  The traces depend only on the
    order of the ids, so the matching is done once per order."""
    gids = [int(g) for g in gids]
    ranks = tuple(int(r) for r in np.argsort(np.argsort(gids)))
    ent, sign = _classify_ranked(P, ranks)
    out = []
    for k in ent:
        if k[0] == "v":
            out.append(("v", gids[k[1]]))
        elif k[0] == "e":
            out.append(("e", tuple(gids[v] for v in k[1]), k[2]))
        elif k[0] == "f":
            out.append(("f", tuple(gids[v] for v in k[1]), k[2]))
        else:
            out.append(k)
    return out, sign.copy()


def tet_map(verts: np.ndarray, P: int, dirichlet: bool = True):
    """l2g [n_elem][N_P] with the sign encoding (g, -2 - g, or -1), the
    number of global DOFs, and the CSR lists (row_ptr, col) of each global
    DOF's local copies in ascending local order (col: i or -1 - i)."""
    verts = np.asarray(verts, dtype=np.int64)
    ne = len(verts)
    NP = O.num_modes("tet", P)
    owners = {}
    for e in range(ne):
        for tri in ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)):
            key = tuple(sorted(int(verts[e, v]) for v in tri))
            owners.setdefault(key, []).append(e)
    assert all(len(o) <= 2 for o in owners.values()), "a face shared by more than two elements"
    bfaces = {f for f, o in owners.items() if len(o) == 1} if dirichlet else set()
    bverts = {v for f in bfaces for v in f}
    bedges = {(f[i], f[j]) for f in bfaces for i, j in ((0, 1), (0, 2), (1, 2))}
    ents, signs = [], []
    for e in range(ne):
        en, sg = classify(P, verts[e])
        ents.append(en)
        signs.append(sg)
    # canonical numbering
    allv = sorted({k[1] for en in ents for k in en if k[0] == "v"})
    alle = sorted({k[1] for en in ents for k in en if k[0] == "e"})
    allf = sorted({k[1] for en in ents for k in en if k[0] == "f"})
    iv = [v for v in allv if v not in bverts]
    ie = [x for x in alle if x not in bedges]
    jf = [f for f in allf if f not in bfaces]
    fm = _face_modes(P)
    nfm = len(fm)
    vpos = {v: i for i, v in enumerate(iv)}
    epos = {x: len(iv) + i * (P - 1) for i, x in enumerate(ie)}
    fpos = {f: len(iv) + len(ie) * (P - 1) + i * nfm for i, f in enumerate(jf)}
    base_i = len(iv) + len(ie) * (P - 1) + len(jf) * nfm
    n_int = (P - 1) * (P - 2) * (P - 3) // 6
    l2g = np.full((ne, NP), -1, dtype=np.int64)
    for e in range(ne):
        ii = 0
        for m, k in enumerate(ents[e]):
            if k[0] == "v":
                g = vpos.get(k[1], -1)
            elif k[0] == "e":
                g = epos[k[1]] + (k[2] - 2) if k[1] in epos else -1
            elif k[0] == "f":
                g = fpos[k[1]] + fm.index(k[2]) if k[1] in fpos else -1
            else:
                g = base_i + e * n_int + ii
                ii += 1
            if g >= 0:
                l2g[e, m] = g if signs[e][m] > 0 else -2 - g
        assert ii == n_int
    n_global = base_i + ne * n_int
    flat = l2g.ravel()
    gidx = np.where(flat >= 0, flat, -2 - flat)
    keep = flat != -1
    loc = np.flatnonzero(keep)
    order = np.lexsort((loc, gidx[keep]))
    rows = gidx[keep][order]
    cols = loc[order]
    cols = np.where(flat[cols] >= 0, cols, -1 - cols)
    row_ptr = np.zeros(n_global + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return l2g, n_global, row_ptr, cols.astype(np.int64)


def signed_map(l2g: np.ndarray, n_global: int) -> sp.csr_matrix:
    """A [n_local, n_global]: the local copy i of global DOF g with its sign."""
    flat = l2g.ravel()
    keep = flat != -1
    g = np.where(flat >= 0, flat, -2 - flat)[keep]
    s = np.where(flat >= 0, 1.0, -1.0)[keep]
    return sp.csr_matrix((s, (np.flatnonzero(keep), g)), shape=(flat.size, n_global))


def element_matrices(P: int, jac: np.ndarray, kind: str, lam: float = 1.0, chunk: int = 256) -> np.ndarray:
    """Dense elemental matrices of the tetrahedra ('mass', 'laplacian' or
    'helmholtz' = lam M + L)."""
    out = []
    for e0 in range(0, jac.shape[0], chunk):
        el = O.Element("tet", P, P + 2, jac[e0:e0 + chunk])
        out.append(el.mass() if kind == "mass" else el.laplacian() if kind == "laplacian" else el.helmholtz(lam))
    return np.concatenate(out, axis=0)


def assemble(mats: np.ndarray, l2g: np.ndarray, n_global: int) -> sp.csr_matrix:
    """A^T blockdiag(mats) A."""
    A = signed_map(l2g, n_global)
    return (A.T @ sp.block_diag(list(mats), format="csr") @ A).tocsr()


def assemble_vector(v: np.ndarray, l2g: np.ndarray, n_global: int) -> np.ndarray:
    """A^T v for local vectors v [n_elem][N_P]."""
    return signed_map(l2g, n_global).T @ np.asarray(v).ravel()


def scatter(xg: np.ndarray, l2g: np.ndarray) -> np.ndarray:
    """A xg: the local coefficient vectors [n_elem][N_P] of a global vector."""
    return (signed_map(l2g, len(xg)) @ xg).reshape(l2g.shape)


def solve(H: sp.csr_matrix, b: np.ndarray) -> np.ndarray:
    return spla.spsolve(H.tocsc(), b)
