"""Seeded synthetic inputs: element meshes of the unit cube and random coefficients.

This module only generates inputs.  It holds none of the spectral/hp method's
arithmetic (no quadrature, no basis, no collapse map, no geometric factors): the
caller passes the reference-element points xi at which the mesh's Jacobian or
coordinates are wanted, and the number of modes for coefficient vectors.

Mesh model (the mixed-element benchmark mesh):

* the unit cube is cut into ``ncell**3`` cubic cells of side ``h = 1/ncell``;
* the quadrant of a cell's centre, (qx, qy) = ([x >= 1/2], [y >= 1/2]), picks its
  split: (0,0) one hexahedron, (1,0) two prisms, (0,1) six pyramids (one per face,
  apex at the cell centre), (1,1) six tetrahedra (the Kuhn split along the main
  diagonal);
* each element e has an affine map chi_e(xi) = x0_e + A_e (1 + xi)/2 from its
  reference element (xi in [-1,1]^3 restricted to the shape) to the straight-sided
  sub-cell;
* curved elements compose it with the smooth perturbation
  Phi(X) = X + amp * sin(2 pi X) sin(2 pi Y) sin(2 pi Z) * (1,1,1), amp = 0.05,
  which fixes the planes x, y, z in {0, 1/2, 1}; x(xi) = Phi(chi_e(xi)).

Reference elements (vertex coordinates):
  hex     [-1,1]^3
  prism   {xi1 + xi3 <= 0}, xi2 free
  pyramid {xi1 + xi3 <= 0, xi2 + xi3 <= 0}, apex (-1,-1,1)
  tet     {xi1 + xi2 + xi3 <= -1}, vertices (-1,-1,-1),(1,-1,-1),(-1,1,-1),(-1,-1,1)

Jacobian layout returned: ``[n_elem][9][n_pts]`` with component ``i*3 + j`` holding
d x_i / d xi_j, points contiguous.
"""
from __future__ import annotations

import numpy as np

SHAPES = ("hex", "prism", "pyr", "tet")
AMP = 0.05


class ElementMaps:
    """Affine maps chi_e(xi) = x0[e] + A[e] @ (1 + xi) / 2 of one shape's batch."""

    def __init__(self, shape: str, x0: np.ndarray, A: np.ndarray):
        self.shape = shape
        self.x0 = np.ascontiguousarray(x0, dtype=np.float64)
        self.A = np.ascontiguousarray(A, dtype=np.float64)

    def __len__(self):
        return self.x0.shape[0]

    def take(self, idx) -> "ElementMaps":
        idx = np.asarray(idx)
        return ElementMaps(self.shape, self.x0[idx], self.A[idx])


def _cell_splits(shape: str, x0: np.ndarray, h: float):
    """Sub-element affine maps of cells with lower corners x0 [n,3] for one split."""
    n = x0.shape[0]
    I = np.eye(3)
    if shape == "hex":
        return x0.copy(), np.broadcast_to(h * I, (n, 3, 3)).copy()
    if shape == "prism":
        # the cell split by the plane t1 + t3 = 1 (t = (x - x0)/h); the second
        # prism is the point reflection of the first in (t1, t3).
        A1 = np.broadcast_to(h * I, (n, 3, 3))
        x02 = x0 + h * np.array([1.0, 0.0, 1.0])
        A2 = np.broadcast_to(h * np.diag([-1.0, 1.0, -1.0]), (n, 3, 3))
        X0 = np.stack([x0, x02], axis=1).reshape(-1, 3)
        A = np.stack([A1, A2], axis=1).reshape(-1, 3, 3)
        return X0, A
    if shape == "pyr":
        c = x0 + 0.5 * h
        X0s, As = [], []
        for d in range(3):
            for s in (0, 1):
                a, b = (d + 1) % 3, (d + 2) % 3
                if s == 1:
                    a, b = b, a
                V0 = x0 + s * h * I[d]
                A = np.empty((n, 3, 3))
                A[:, :, 0] = h * I[a]
                A[:, :, 1] = h * I[b]
                A[:, :, 2] = c - V0
                X0s.append(V0)
                As.append(A)
        X0 = np.stack(X0s, axis=1).reshape(-1, 3)
        A = np.stack(As, axis=1).reshape(-1, 3, 3)
        return X0, A
    if shape == "tet":
        perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
        X0s, As = [], []
        for pi in perms:
            sign = np.linalg.det(np.stack([I[pi[0]], I[pi[1]], I[pi[2]]]))
            e1 = h * I[pi[0]]
            e2 = h * (I[pi[0]] + I[pi[1]])
            e3 = h * np.ones(3)
            cols = [e1, e2, e3] if sign > 0 else [e2, e1, e3]
            A = np.empty((n, 3, 3))
            for j in range(3):
                A[:, :, j] = cols[j]
            X0s.append(x0)
            As.append(A)
        X0 = np.stack(X0s, axis=1).reshape(-1, 3)
        A = np.stack(As, axis=1).reshape(-1, 3, 3)
        return X0, A
    raise ValueError(f"unknown shape {shape!r}")


def _cells(ncell: int, qx=None, qy=None):
    h = 1.0 / ncell
    idx = np.arange(ncell)
    I, J, K = np.meshgrid(idx, idx, idx, indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    x0 = np.stack([I, J, K], axis=1) * h
    if qx is not None:
        cx = (I + 0.5) * h
        cy = (J + 0.5) * h
        keep = ((cx >= 0.5) == bool(qx)) & ((cy >= 0.5) == bool(qy))
        x0 = x0[keep]
    return x0, h


QUADRANT = {"hex": (0, 0), "prism": (1, 0), "pyr": (0, 1), "tet": (1, 1)}


def quadrant_mesh(ncell: int = 32) -> dict:
    """The mixed mesh: {shape: ElementMaps}.  ncell = 32 gives 8192 hexes,
    16384 prisms, 49152 pyramids and 49152 tetrahedra."""
    if ncell % 2:
        raise ValueError("ncell must be even")
    out = {}
    for shape in SHAPES:
        x0, h = _cells(ncell, *QUADRANT[shape])
        X0, A = _cell_splits(shape, x0, h)
        out[shape] = ElementMaps(shape, X0, A)
    return out


def shape_batch(shape: str, n_elem: int) -> ElementMaps:
    """n_elem elements of one shape: cells of the smallest grid that holds them,
    all split by that shape's rule, the first n_elem kept."""
    per = {"hex": 1, "prism": 2, "pyr": 6, "tet": 6}[shape]
    ncell = 1
    while per * ncell ** 3 < n_elem:
        ncell += 1
    x0, h = _cells(ncell)
    X0, A = _cell_splits(shape, x0, h)
    return ElementMaps(shape, X0[:n_elem], A[:n_elem])


def affine_hex_grid(n: int = 4) -> ElementMaps:
    """n^3 axis-aligned hexahedra of side 1/n tiling the unit cube."""
    x0, h = _cells(n)
    X0, A = _cell_splits("hex", x0, h)
    return ElementMaps("hex", X0, A)



def conforming_tet_mesh(n: int):
    """The unit cube in n^3 cubes, each split into the 6 tetrahedra of the
    Freudenthal (Kuhn) triangulation: the paths (0,0,0) -> e_a -> e_a + e_b ->
    (1,1,1) over the 6 orders (a, b, c) of the axes.  Neighbouring cubes split
    their shared faces along the same diagonal, so the mesh is conforming.

    Grid vertex (i, j, k) has id (i (n+1) + j)(n+1) + k.  Along a path the ids
    increase, so its last vertex has the largest id of the four and its third
    the second largest: these are each tet's local vertices 3 and 2.  Local
    vertices 0 and 1 are the path's first two, swapped where needed so that
    det(V1 - V0, V2 - V0, V3 - V0) > 0 (reference vertices (-1,-1,-1),
    (1,-1,-1), (-1,1,-1), (-1,-1,1)); about half the tets swap them.

    Returns (ElementMaps of shape 'tet' with x0 = V0 and A = [V1 - V0, V2 - V0,
    V3 - V0], verts [n_elem][4] int64 in local order)."""
    h = 1.0 / n
    I = np.eye(3, dtype=np.int64)
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    ii, jj, kk = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    c0 = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1).astype(np.int64)      # [ncube, 3]
    gid = lambda g: (g[..., 0] * (n + 1) + g[..., 1]) * (n + 1) + g[..., 2]
    X0, A, V = [], [], []
    for a, b, c in perms:
        path = [c0, c0 + I[a], c0 + I[a] + I[b], c0 + 1]
        sign = int(round(np.linalg.det(np.stack([I[a], I[b], I[c]]).astype(float))))
        loc = path if sign > 0 else [path[1], path[0], path[2], path[3]]
        pos = [x.astype(np.float64) * h for x in loc]
        X0.append(pos[0])
        A.append(np.stack([pos[1] - pos[0], pos[2] - pos[0], pos[3] - pos[0]], axis=2))
        V.append(np.stack([gid(x) for x in loc], axis=1))
    ne = len(c0) * 6
    X0 = np.stack(X0, axis=1).reshape(ne, 3)
    A = np.stack(A, axis=1).reshape(ne, 3, 3)
    V = np.stack(V, axis=1).reshape(ne, 4)
    return ElementMaps("tet", X0, A), np.ascontiguousarray(V, dtype=np.int64)

# ---------------------------------------------------------------------------
# point evaluation
# ---------------------------------------------------------------------------

def _chi(maps: ElementMaps, xi: np.ndarray) -> np.ndarray:
    """Straight-sided physical coordinates [n_elem, n_pts, 3]."""
    t = 0.5 * (1.0 + np.asarray(xi, dtype=np.float64))  # [n_pts,3]
    return maps.x0[:, None, :] + np.einsum("eij,pj->epi", maps.A, t)


def coords(maps: ElementMaps, xi: np.ndarray, curved: bool, amp: float = AMP) -> np.ndarray:
    """Physical coordinates x(xi) as [n_elem][3][n_pts]."""
    X = _chi(maps, xi)
    if curved:
        s = np.prod(np.sin(2 * np.pi * X), axis=-1)
        X = X + amp * s[..., None]
    return np.ascontiguousarray(np.transpose(X, (0, 2, 1)))


def jacobian(maps: ElementMaps, xi: np.ndarray, curved: bool, amp: float = AMP,
             chunk: int = 8192) -> np.ndarray:
    """d x_i / d xi_j at the points, layout [n_elem][9][n_pts] (component i*3+j)."""
    xi = np.asarray(xi, dtype=np.float64)
    ne, npts = len(maps), xi.shape[0]
    out = np.empty((ne, 9, npts))
    for e0 in range(0, ne, chunk):
        e1 = min(ne, e0 + chunk)
        Ah = 0.5 * maps.A[e0:e1]                          # d chi / d xi
        if not curved:
            out[e0:e1] = np.repeat(Ah.reshape(e1 - e0, 9, 1), npts, axis=2)
            continue
        X = _chi(maps.take(np.arange(e0, e1)), xi)         # [ne,npts,3]
        sn = np.sin(2 * np.pi * X)
        cs = np.cos(2 * np.pi * X)
        ds = np.empty_like(X)                              # grad of s
        ds[..., 0] = 2 * np.pi * cs[..., 0] * sn[..., 1] * sn[..., 2]
        ds[..., 1] = 2 * np.pi * sn[..., 0] * cs[..., 1] * sn[..., 2]
        ds[..., 2] = 2 * np.pi * sn[..., 0] * sn[..., 1] * cs[..., 2]
        # dPhi_i/dX_k = delta_ik + amp * ds_k  (same for every i)
        # J_ij = sum_k dPhi_i/dX_k * Ah_kj = Ah_ij + amp * (ds . Ah[:, j])
        g = np.einsum("epk,ekj->epj", ds, Ah)              # [ne,npts,3]
        J = Ah[:, None, :, :] + amp * g[:, :, None, :]     # [ne,npts,3,3]
        out[e0:e1] = np.transpose(J.reshape(e1 - e0, npts, 9), (0, 2, 1))
    return out


def jacobian_torch(maps: ElementMaps, xi: np.ndarray, curved: bool, device, amp: float = AMP, chunk: int = 65536):
    """jacobian() evaluated with torch on a device (same formula), for large
    batches: returns a float64 tensor [n_elem][9][n_pts]."""
    import torch
    xi_t = torch.as_tensor(np.asarray(xi, dtype=np.float64), device=device)
    ne, npts = len(maps), xi_t.shape[0]
    out = torch.empty((ne, 9, npts), dtype=torch.float64, device=device)
    t = 0.5 * (1.0 + xi_t)                                              # [npts,3]
    for e0 in range(0, ne, chunk):
        e1 = min(ne, e0 + chunk)
        A = torch.as_tensor(maps.A[e0:e1], device=device)
        x0 = torch.as_tensor(maps.x0[e0:e1], device=device)
        Ah = 0.5 * A
        if not curved:
            out[e0:e1] = Ah.reshape(e1 - e0, 9, 1).expand(e1 - e0, 9, npts)
            continue
        X = x0[:, None, :] + torch.einsum("eij,pj->epi", A, t)          # [ne,npts,3]
        sn = torch.sin(2 * np.pi * X)
        cs = torch.cos(2 * np.pi * X)
        ds = torch.stack([2 * np.pi * cs[..., 0] * sn[..., 1] * sn[..., 2],
                          2 * np.pi * sn[..., 0] * cs[..., 1] * sn[..., 2],
                          2 * np.pi * sn[..., 0] * sn[..., 1] * cs[..., 2]], dim=-1)
        g = torch.einsum("epk,ekj->epj", ds, Ah)
        J = Ah[:, None, :, :] + amp * g[:, :, None, :]
        out[e0:e1] = J.reshape(e1 - e0, npts, 9).permute(0, 2, 1)
    return out


def manufactured_u_torch(maps: ElementMaps, xi: np.ndarray, device, amp: float = AMP, chunk: int = 65536):
    """manufactured_u at the curved coordinates x(xi), evaluated with torch on a
    device: float64 tensor [n_elem][n_pts]."""
    import torch
    xi_t = torch.as_tensor(np.asarray(xi, dtype=np.float64), device=device)
    ne, npts = len(maps), xi_t.shape[0]
    out = torch.empty((ne, npts), dtype=torch.float64, device=device)
    t = 0.5 * (1.0 + xi_t)
    for e0 in range(0, ne, chunk):
        e1 = min(ne, e0 + chunk)
        A = torch.as_tensor(maps.A[e0:e1], device=device)
        x0 = torch.as_tensor(maps.x0[e0:e1], device=device)
        X = x0[:, None, :] + torch.einsum("eij,pj->epi", A, t)
        X = X + amp * torch.prod(torch.sin(2 * np.pi * X), dim=-1, keepdim=True)
        out[e0:e1] = torch.prod(torch.sin(np.pi * X), dim=-1)
    return out


def iso_coords(maps: ElementMaps, vertex_idx, vertex_xi: np.ndarray, n_modes: int, seed: int,
               curved: bool = True, amp: float = 0.02) -> np.ndarray:
    """Coordinate coefficients [n_elem][3][n_modes] of iso-parametric elements:
    the mesh map's vertex positions x(xi_v) on the vertex coefficients
    vertex_idx (the caller gives the index of each vertex's coefficient and
    its reference coordinates xi_v), and every other coefficient uniform in
    [-amp h, amp h] per coordinate, h the element's size (the largest column
    norm of its affine map), from the seed: curved elements near the mesh's."""
    rng = np.random.default_rng(seed)
    ne = len(maps)
    h = np.linalg.norm(maps.A, axis=1).max(axis=1)                      # [ne]
    X = rng.uniform(-1.0, 1.0, size=(ne, 3, n_modes)) * (amp * h)[:, None, None]
    X[:, :, list(vertex_idx)] = coords(maps, np.asarray(vertex_xi, dtype=np.float64), curved)
    return X


def affine_jacobian(maps: ElementMaps) -> np.ndarray:
    """Constant d x_i / d xi_j of straight-sided elements, layout [n_elem][9]."""
    return np.ascontiguousarray((0.5 * maps.A).reshape(len(maps), 9))


# ---------------------------------------------------------------------------
# two-dimensional meshes
# ---------------------------------------------------------------------------

SHAPES2 = ("quad", "tri")


def quad_tri_mesh(ncell: int = 256) -> dict:
    """The unit square in ncell^2 cells: cells with centre x < 1/2 are
    quadrilaterals, the others two triangles each (lower-left: vertices x0,
    x0 + h e1, x0 + h e2; upper-right: its point reflection through the cell
    centre).  Reference square [-1,1]^2, reference triangle {xi1 + xi2 <= 0}
    with vertices (-1,-1), (1,-1), (-1,1).  {shape: ElementMaps} with 2D x0, A."""
    if ncell % 2:
        raise ValueError("ncell must be even")
    h = 1.0 / ncell
    ii, jj = np.meshgrid(np.arange(ncell), np.arange(ncell), indexing="ij")
    x0 = np.stack([ii.ravel() * h, jj.ravel() * h], axis=1)
    left = x0[:, 0] + 0.5 * h < 0.5
    q0 = x0[left]
    t0 = x0[~left]
    I = np.eye(2)
    quads = ElementMaps("quad", q0, np.broadcast_to(h * I, (len(q0), 2, 2)).copy())
    tx0 = np.concatenate([t0, t0 + h], axis=0)
    tA = np.concatenate([np.broadcast_to(h * I, (len(t0), 2, 2)), np.broadcast_to(-h * I, (len(t0), 2, 2))], axis=0)
    order = np.argsort(np.concatenate([np.arange(len(t0)) * 2, np.arange(len(t0)) * 2 + 1]), kind="stable")
    tris = ElementMaps("tri", tx0[order], tA[order])
    return {"quad": quads, "tri": tris}


def jacobian2d(maps: ElementMaps, xi: np.ndarray, curved: bool, amp: float = AMP) -> np.ndarray:
    """d x_i / d xi_j of 2D elements, [n_elem][4][n_pts] (component i*2 + j):
    the affine map composed with Phi(X) = X + amp sin(2 pi X) sin(2 pi Y) (1,1)
    when curved."""
    xi = np.asarray(xi, dtype=np.float64)
    ne, npts = len(maps), xi.shape[0]
    Ah = 0.5 * maps.A                                       # [ne,2,2]
    if not curved:
        return np.ascontiguousarray(np.repeat(Ah.reshape(ne, 4, 1), npts, axis=2))
    X = _chi(maps, xi)                                      # [ne,npts,2]
    sn, cs = np.sin(2 * np.pi * X), np.cos(2 * np.pi * X)
    ds = np.stack([2 * np.pi * cs[..., 0] * sn[..., 1], 2 * np.pi * sn[..., 0] * cs[..., 1]], axis=-1)
    g = np.einsum("epk,ekj->epj", ds, Ah)
    J = Ah[:, None, :, :] + amp * g[:, :, None, :]
    return np.ascontiguousarray(np.transpose(J.reshape(ne, npts, 4), (0, 2, 1)))


def affine_jacobian2d(maps: ElementMaps) -> np.ndarray:
    """Constant d x_i / d xi_j of straight-sided 2D elements, [n_elem][4]."""
    return np.ascontiguousarray((0.5 * maps.A).reshape(len(maps), 4))


def coeffs(n_elem: int, n_modes: int, seed: int) -> np.ndarray:
    """Elemental coefficients uniform in [-1, 1], [n_elem][n_modes], FP64."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(n_elem, n_modes))


def point_values(n_elem: int, n_pts: int, seed: int, ncomp: int = 0) -> np.ndarray:
    """Point data uniform in [-1, 1]: [n_elem][n_pts] or [ncomp][n_elem][n_pts]."""
    rng = np.random.default_rng(seed)
    shape = (n_elem, n_pts) if ncomp == 0 else (ncomp, n_elem, n_pts)
    return rng.uniform(-1.0, 1.0, size=shape)


def manufactured_u(x: np.ndarray) -> np.ndarray:
    """u = sin(pi x) sin(pi y) sin(pi z) at coordinates laid out [..][3][n_pts]."""
    return np.sin(np.pi * x[..., 0, :]) * np.sin(np.pi * x[..., 1, :]) * np.sin(np.pi * x[..., 2, :])


# seeds of the synthetic workloads
SEED_CFG1 = 0
SEED_MIXED = {"hex": 1, "prism": 2, "pyr": 3, "tet": 4}


def seed_sweep(P: int) -> int:
    return 1000 + P
