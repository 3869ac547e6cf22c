"""Pins of the C0 assembly oracle (structured hexahedral grid) and the
library's host-side map against it.

- Sharing: a global DOF has 2 local copies per direction in which it is a
  vertex function and 1 in which it is a bubble (8 at a grid vertex, 4 on an
  edge, 2 on a face, 1 inside a cell).
- Without Dirichlet data, the vertex coefficients set to 1 represent u = 1:
  x^T M x is the volume of the unit cube and L x = 0.
- With Dirichlet data the assembled Helmholtz operator is symmetric positive
  definite, and the discrete solution of -lap u + lambda u = f with
  u = sin(pi x) sin(pi y) sin(pi z) converges spectrally to u.
- The library's map (shp_c0_hex_sizes / shp_c0_hex_map, host code) equals the
  oracle's, index for index, and its CSR lists each global DOF's local copies
  in ascending order.
"""
import ctypes

import numpy as np
import pytest

from oracle import shp_assembly as A
from oracle import shp_oracle as O
from paper_2604_04644_amd import workloads as W


def test_sharing_counts():
    P = 3
    l2g, ng = A.hex_grid_map(3, 2, 4, P, dirichlet=False)
    copies = np.bincount(l2g[l2g >= 0], minlength=ng)
    lines = [A.line_numbering(nc, P, dirichlet=False) for nc in (3, 2, 4)]
    mult = [None] * 3
    # vertex keys of interior vertices are shared by 2 cells, boundary ones by 1
    for d, (ids, cnt) in enumerate(lines):
        nc = (3, 2, 4)[d]
        m = np.ones(cnt, dtype=int)
        for key, g in ids.items():
            if key[0] == "v" and 0 < key[1] < nc:
                m[g] = 2
        mult[d] = m
    expect = (mult[0][:, None, None] * mult[1][None, :, None] * mult[2][None, None, :]).ravel()
    assert np.array_equal(copies, expect)


@pytest.mark.parametrize("curved", [False, True])
def test_volume_and_constants(curved):
    P, n = 3, 2
    maps = W.affine_hex_grid(n)
    xi = O.reference_points("hex", P + 2)
    jac = W.jacobian(maps, xi, curved=True) if curved else W.jacobian(maps, xi, curved=False)
    l2g, ng = A.hex_grid_map(n, n, n, P, dirichlet=False)
    M = A.assemble(A.element_matrices(P, jac, "mass"), l2g, ng)
    L = A.assemble(A.element_matrices(P, jac, "laplacian"), l2g, ng)
    lines = [A.line_numbering(n, P, dirichlet=False)] * 3
    is_v = np.zeros(lines[0][1], dtype=bool)
    for key, g in lines[0][0].items():
        is_v[g] = key[0] == "v"
    ones = (is_v[:, None, None] & is_v[None, :, None] & is_v[None, None, :]).ravel().astype(float)
    vol = ones @ (M @ ones)
    assert abs(vol - 1.0) <= (1e-13 if not curved else 1e-6)
    assert np.abs(L @ ones).max() <= 1e-12 * np.abs(L).max()


def _manufactured(n, P, curved):
    maps = W.affine_hex_grid(n)
    xi = O.reference_points("hex", P + 2)
    jac = W.jacobian(maps, xi, curved=curved)
    l2g, ng = A.hex_grid_map(n, n, n, P)
    lam = 1.0
    H = A.assemble(A.element_matrices(P, jac, "helmholtz", lam), l2g, ng)
    f = (lam + 3 * np.pi ** 2) * W.manufactured_u(W.coords(maps, xi, curved=curved))
    b = A.assemble_vector(O.apply_op("iprod", "hex", P, P + 2, jac, f), l2g, ng)
    x = A.solve(H, b)
    xl = np.where(l2g >= 0, x[np.maximum(l2g, 0)], 0.0)
    u = O.apply_op("bwd", "hex", P, P + 2, jac, xl)
    err = np.abs(u - W.manufactured_u(W.coords(maps, xi, curved=curved))).max()
    return H, err


def test_spd_and_spectral_convergence():
    H, _ = _manufactured(2, 3, True)
    Hd = H.toarray()
    assert np.abs(Hd - Hd.T).max() <= 1e-13 * np.abs(Hd).max()
    assert np.linalg.eigvalsh(Hd)[0] > 0
    errs = [_manufactured(2, P, False)[1] for P in (2, 4, 6)]
    assert errs[0] > 1e2 * errs[1] > 1e4 * errs[2], errs
    assert errs[2] < 1e-4


def test_library_map_matches_oracle():
    from paper_2604_04644_amd import shp
    L = shp.lib()
    for (n0, n1, n2, P) in [(1, 1, 1, 1), (2, 3, 2, 3), (3, 1, 2, 4), (2, 2, 2, 6)]:
        ng, nl, ne = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        assert L.shp_c0_hex_sizes(n0, n1, n2, P, ctypes.byref(ng), ctypes.byref(nl), ctypes.byref(ne)) == 0
        l2g = np.empty(nl.value, dtype=np.int64)
        rp = np.empty(ng.value + 1, dtype=np.int64)
        col = np.empty(max(ne.value, 1), dtype=np.int64)
        assert L.shp_c0_hex_map(n0, n1, n2, P, l2g.ctypes.data, rp.ctypes.data, col.ctypes.data) == 0
        ref, ngo = A.hex_grid_map(n0, n1, n2, P)
        assert ng.value == ngo and nl.value == ref.size and ne.value == int((ref >= 0).sum())
        assert np.array_equal(l2g, ref.ravel())
        order = np.argsort(ref.ravel()[ref.ravel() >= 0], kind="stable")
        local = np.flatnonzero(ref.ravel() >= 0)[order]
        assert np.array_equal(col[:ne.value], local)
        assert np.array_equal(np.diff(rp), np.bincount(ref.ravel()[ref.ravel() >= 0], minlength=ngo))
    assert L.shp_c0_hex_sizes(0, 1, 1, 2, ctypes.byref(ng), ctypes.byref(nl), ctypes.byref(ne)) == -1
    assert L.shp_c0_hex_map(1, 1, 1, 11, None, None, None) == -1
