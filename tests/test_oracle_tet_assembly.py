"""Pins of the C0 assembly oracle on a conforming tetrahedral mesh, and the
library's host-side map (shp_c0_tet_sizes / shp_c0_tet_map) against it.

- Counts: the global DOFs are one per interior vertex, P - 1 per interior
  edge, (P - 1)(P - 2)/2 per interior face and (P - 1)(P - 2)(P - 3)/6 per
  element, with the entities counted from the mesh's own vertex lists.
- Continuity: any global vector gives local fields that agree, from both
  elements, at points of every shared face; one copy's sign flipped breaks it.
- Without Dirichlet data the vertex coefficients set to 1 represent u = 1:
  the local fields are 1 everywhere, x^T M x is the volume of the unit cube and
  L x = 0.
- With Dirichlet data the assembled Helmholtz operator is symmetric positive
  definite and the discrete solution of -lap u + lambda u = f with
  u = sin(pi x) sin(pi y) sin(pi z) converges spectrally to u.
- The library's map equals the oracle's index for index, signs included.
"""
import numpy as np
import pytest

from oracle import shp_assembly_tet as T
from oracle import shp_oracle as O
from paper_2604_04644_amd import workloads as W

FACES = ((0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3))


def _entities(V):
    edges, faces = set(), {}
    for v in V:
        for a in range(4):
            for b in range(a + 1, 4):
                edges.add(tuple(sorted((int(v[a]), int(v[b])))))
        for f in FACES:
            k = tuple(sorted(int(v[i]) for i in f))
            faces[k] = faces.get(k, 0) + 1
    return edges, faces


@pytest.mark.parametrize("n", [1, 2, 3])
@pytest.mark.parametrize("dirichlet", [True, False])
def test_counts(n, dirichlet):
    _, V = W.conforming_tet_mesh(n)
    edges, faces = _entities(V)
    assert max(faces.values()) == 2
    bf = {f for f, c in faces.items() if c == 1}
    bv = {x for f in bf for x in f}
    be = {(f[i], f[j]) for f in bf for i, j in ((0, 1), (0, 2), (1, 2))}
    verts = {int(x) for x in V.ravel()}
    for P in (1, 2, 3, 5):
        _, ng, rp, col = T.tet_map(V, P, dirichlet=dirichlet)
        nv = len(verts - bv) if dirichlet else len(verts)
        ne = len(edges - be) if dirichlet else len(edges)
        nf = len(set(faces) - bf) if dirichlet else len(faces)
        assert ng == nv + ne * (P - 1) + nf * (P - 1) * (P - 2) // 2 + len(V) * (P - 1) * (P - 2) * (P - 3) // 6
        assert rp[-1] == len(col)


def _face_points(P):
    g = np.cos(np.pi * (np.arange(4) + 0.5) / 4)
    a, b = np.meshgrid(g, g, indexing="ij")
    lhi = (1 + b.ravel()) / 2
    lmid = (1 - lhi) * (1 + a.ravel()) / 2
    return np.stack([1 - lhi - lmid, lmid, lhi], axis=1)


def _max_jump(V, xl, P):
    """Largest difference of the two elements' fields over points of every
    shared face (points given by barycentric weights on the sorted ids)."""
    owners = {}
    for e, v in enumerate(V):
        for f in FACES:
            owners.setdefault(tuple(sorted(int(v[i]) for i in f)), []).append(e)
    bary = _face_points(P)
    worst = 0.0
    for key, es in owners.items():
        if len(es) != 2:
            continue
        vals = []
        for e in es:
            local = np.array([list(V[e]).index(g) for g in key])
            vals.append(T.modes_at(P, bary, local) @ xl[e])
        worst = max(worst, float(np.abs(vals[0] - vals[1]).max()))
    return worst


@pytest.mark.parametrize("P", [3, 4, 6])
def test_continuity_across_faces(P):
    _, V = W.conforming_tet_mesh(2)
    l2g, ng, _, _ = T.tet_map(V, P, dirichlet=False)
    assert (l2g <= -2).any()                       # the mesh needs sign changes
    x = np.random.default_rng(P).uniform(-1, 1, ng)
    xl = T.scatter(x, l2g)
    assert _max_jump(V, xl, P) < 1e-12
    # a planted mistake: one negated copy read without its sign
    bad = l2g.copy()
    i = np.flatnonzero(bad.ravel() <= -2)[0]
    bad.ravel()[i] = -2 - bad.ravel()[i]
    assert _max_jump(V, T.scatter(x, bad), P) > 1e-3


@pytest.mark.parametrize("curved", [False, True])
def test_constants_and_volume(curved):
    P = 3
    maps, V = W.conforming_tet_mesh(2)
    l2g, ng, _, _ = T.tet_map(V, P, dirichlet=False)
    ones = np.zeros(ng)
    nvert = len({int(x) for x in V.ravel()})
    ones[:nvert] = 1.0                              # vertex DOFs come first, one per vertex
    xl = T.scatter(ones, l2g)
    pts = np.random.default_rng(0).dirichlet(np.ones(4), 20)
    for e in range(len(V)):
        assert np.abs(T.modes_at(P, pts, np.arange(4)) @ xl[e] - 1.0).max() < 1e-13
    xi = O.reference_points("tet", P + 2)
    jac = W.jacobian(maps, xi, curved=curved)
    M = T.assemble(T.element_matrices(P, jac, "mass"), l2g, ng)
    L = T.assemble(T.element_matrices(P, jac, "laplacian"), l2g, ng)
    assert abs(ones @ (M @ ones) - 1.0) <= (1e-13 if not curved else 1e-5)
    assert np.abs(L @ ones).max() <= 1e-12 * abs(L).max()


@pytest.mark.parametrize("curved", [False, True])
def test_spd_and_spectral_convergence(curved):
    """Straight-sided tets: the error at the points falls by more than 10x per
    two orders.  Curved by the sine map at this coarse size (h = 1/2, about a
    half period of the perturbation per element) the approximation itself
    converges more slowly (the per-element L2 projection of u has errors 0.13,
    0.064, 0.027 at P = 2, 4, 6), so the bar there is a steady fall."""
    maps, V = W.conforming_tet_mesh(2)
    lam = 1.0
    errs = []
    for P in (2, 4, 6):
        l2g, ng, _, _ = T.tet_map(V, P)
        xi = O.reference_points("tet", P + 2)
        jac = W.jacobian(maps, xi, curved=curved)
        H = T.assemble(T.element_matrices(P, jac, "helmholtz", lam), l2g, ng)
        Hd = H.toarray()
        assert np.abs(Hd - Hd.T).max() <= 1e-13 * np.abs(Hd).max()
        assert np.linalg.eigvalsh(Hd).min() > 0
        u = W.manufactured_u(W.coords(maps, xi, curved=curved))
        b = T.assemble_vector(O.apply_op("iprod", "tet", P, P + 2, jac, (lam + 3 * np.pi ** 2) * u), l2g, ng)
        x = T.solve(H, b)
        uh = O.apply_op("bwd", "tet", P, P + 2, jac, T.scatter(x, l2g))
        errs.append(float(np.abs(uh - u).max()))
    if curved:
        assert errs[0] > 2.5 * errs[1] > 6.25 * errs[2], errs
    else:
        assert errs[0] > 10 * errs[1] > 100 * errs[2], errs


@pytest.mark.parametrize("n", [1, 2, 3])
def test_library_map_equals_oracle(n):
    from paper_2604_04644_amd import shp
    _, V = W.conforming_tet_mesh(n)
    for P in range(1, 11):
        l2g, rp, col, ng = shp.c0_tet_map(V, P)
        ol2g, ong, orp, ocol = T.tet_map(V, P)
        assert ng == ong, P
        assert np.array_equal(l2g, ol2g.ravel()), P
        assert np.array_equal(rp, orp), P
        assert np.array_equal(col[:rp[-1]], ocol), P


def test_library_map_errors():
    import ctypes
    from paper_2604_04644_amd import shp
    L = shp.lib()
    _, V = W.conforming_tet_mesh(1)
    ng, nl, ne = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()

    def sizes(v, P=3):
        v = np.ascontiguousarray(v, dtype=np.int64)
        return L.shp_c0_tet_sizes(len(v), v.ctypes.data, P, ctypes.byref(ng), ctypes.byref(nl), ctypes.byref(ne))

    assert sizes(V) == 0
    bad = V.copy()
    bad[0, [2, 3]] = bad[0, [3, 2]]                 # vertex 3 not the largest id
    assert sizes(bad) == -1 and "largest" in L.shp_last_error().decode()
    bad = V.copy()
    bad[0, 0] = -5
    assert sizes(bad) == -1
    bad = V.copy()
    bad[0, 1] = bad[0, 0]
    assert sizes(bad) == -1
    assert sizes(np.concatenate([V, V[:1]])) == -1  # a face in three elements
    assert "more than two" in L.shp_last_error().decode()
    assert sizes(V, P=0) == -1 and sizes(V, P=11) == -1
    assert L.shp_c0_tet_sizes(len(V), None, 3, ctypes.byref(ng), ctypes.byref(nl), ctypes.byref(ne)) == -1
