"""Pins of the 2D oracle (quadrilaterals and triangles) against closed forms,
textbook element matrices and invariants -- none of them re-derived from the
oracle's own formulas."""
import math

import numpy as np
import pytest
import sympy as sp

from oracle import shp_oracle2d as O2
from paper_2604_04644_amd import workloads as W


@pytest.mark.parametrize("pts", ["gj", "radau"])
@pytest.mark.parametrize("shape", O2.SHAPES2)
def test_monomials_exact(shape, pts):
    """Tensor quadrature in eta integrates every monomial of degree <= 2Q - 3
    exactly: with t = (1 + xi)/2, the square gives prod (1 + (-1)^a)/(a + 1)
    in xi and the triangle 4 a! b! / (a + b + 2)!."""
    for Q in (3, 5, 7):
        for a in range(2 * Q - 2):
            for b in range(2 * Q - 2 - a):
                if shape == "quad":
                    f = lambda xi: xi[:, 0] ** a * xi[:, 1] ** b
                    exact = (1 + (-1) ** a) / (a + 1) * (1 + (-1) ** b) / (b + 1)
                else:
                    f = lambda xi: ((1 + xi[:, 0]) / 2) ** a * ((1 + xi[:, 1]) / 2) ** b
                    exact = 4.0 * math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
                got = O2.integrate_reference(shape, Q, f, pts)
                assert abs(got - exact) < 1e-13 * max(1.0, abs(exact)), (Q, a, b, got, exact)


def test_linear_triangle_matrices():
    """P = 1 triangle: the vertex modes are the barycentric coordinates, so M =
    area/12 (1 + delta_ij) and L = area grad(lambda_i) . grad(lambda_j) (the
    textbook linear triangle), on a skewed affine triangle."""
    V = np.array([[0.1, 0.2], [0.9, 0.35], [0.3, 1.1]])          # vertices of (-1,-1), (1,-1), (-1,1)
    A = np.stack([V[1] - V[0], V[2] - V[0]], axis=1)              # x = V0 + A (1 + xi)/2
    jac = (0.5 * A).reshape(1, 4)
    el = O2.Element2D("tri", 1, 3, jac)
    idx, _ = O2.vertex_modes("tri", 1)
    M = el.mass()[0][np.ix_(idx, idx)]
    L = el.laplacian()[0][np.ix_(idx, idx)]
    area = 0.5 * abs(np.linalg.det(A))
    assert np.allclose(M, area / 12 * (np.ones((3, 3)) + np.eye(3)), atol=1e-15)
    # gradients of the barycentric coordinates
    T = np.array([[1, *V[0]], [1, *V[1]], [1, *V[2]]])
    grads = np.linalg.inv(T)[1:].T                                # [3 vertices][2]
    assert np.allclose(L, area * grads @ grads.T, atol=1e-14)


def _exact_1d(P):
    z = sp.Symbol("z")

    def A(p):
        if p == 0:
            return (1 - z) / 2
        if p == 1:
            return (1 + z) / 2
        return (1 - z) / 2 * (1 + z) / 2 * sp.jacobi(p - 2, 1, 1, z)

    fs = [A(p) for p in range(P + 1)]
    M = np.array([[float(sp.integrate(fi * fj, (z, -1, 1))) for fj in fs] for fi in fs])
    K = np.array([[float(sp.integrate(sp.diff(fi, z) * sp.diff(fj, z), (z, -1, 1))) for fj in fs] for fi in fs])
    return M, K


@pytest.mark.parametrize("P", [1, 2, 4])
def test_affine_square_kronecker(P):
    """Square of side h: H = lam (h/2)^2 M1 x M1 + K1 x M1 + M1 x K1 with the
    exact (symbolic) 1D modified-basis mass and stiffness."""
    M1, K1 = _exact_1d(P)
    h, lam = 0.25, 1.7
    jac = np.array([[h / 2, 0.0, 0.0, h / 2]])
    H = O2.Element2D("quad", P, P + 2, jac).helmholtz(lam)[0]
    Href = lam * (h / 2) ** 2 * np.kron(M1, M1) + np.kron(K1, M1) + np.kron(M1, K1)
    assert np.abs(H - Href).max() < 1e-13 * np.abs(Href).max()


@pytest.mark.parametrize("shape", O2.SHAPES2)
def test_basis_spans_polynomials(shape):
    """The triangle's modes span exactly the polynomials of total degree <= P in
    xi, the square's the tensor polynomials of degree <= P per direction: every
    such monomial is reproduced by least squares through the points, and the
    basis values have full rank."""
    P, Q = 4, 6
    eta, _, _ = O2.quadrature(shape, Q)
    xi = O2.collapse(shape, eta)
    B, _ = O2.basis(shape, P, eta)
    assert np.linalg.matrix_rank(B) == O2.num_modes(shape, P)
    for a in range(P + 1):
        for b in range(P + 1 if shape == "quad" else P + 1 - a):
            f = xi[:, 0] ** a * xi[:, 1] ** b
            c, *_ = np.linalg.lstsq(B, f, rcond=None)
            assert np.abs(B @ c - f).max() < 1e-12, (a, b)


def test_vertex_modes_nodal():
    """Each vertex mode is one at its vertex and zero at the other vertices
    (evaluated at eta points mapping to the vertices; the triangle's top vertex
    is eta2 = 1 for any eta1)."""
    for shape in O2.SHAPES2:
        idx, vxi = O2.vertex_modes(shape, 3)
        eta = vxi.copy()
        if shape == "tri":
            eta[:, 0] = np.where(vxi[:, 1] > 0, 0.3, vxi[:, 0])   # the collapsed vertex
        B, _ = O2.basis(shape, 3, eta)
        assert np.allclose(B[:, idx], np.eye(len(idx)), atol=1e-15)


def test_curved_mesh_invariants():
    """Curved quad/triangle mesh of the unit square: the areas sum to 1 (the
    map fixes the boundary), M symmetric positive definite, L symmetric
    semidefinite with L 1 = 0 (the vertex modes sum to one)."""
    mesh = W.quad_tri_mesh(4)
    P, Q = 3, 5
    total = 0.0
    for shape in O2.SHAPES2:
        jac = W.jacobian2d(mesh[shape], O2.reference_points(shape, Q), curved=True)
        el = O2.Element2D(shape, P, Q, jac)
        M, L = el.mass(), el.laplacian()
        one = np.zeros(O2.num_modes(shape, P))
        one[O2.vertex_modes(shape, P)[0]] = 1.0
        total += float(np.einsum("m,emn,n->", one, M, one))
        assert np.abs(M - np.transpose(M, (0, 2, 1))).max() < 1e-15
        assert np.abs(L - np.transpose(L, (0, 2, 1))).max() < 1e-13
        assert np.abs(L @ one).max() < 1e-13
        assert np.linalg.eigvalsh(M).min() > 0
        assert np.linalg.eigvalsh(L).min() > -1e-12
    assert abs(total - 1.0) < 1e-6


def test_cross_operator_identities():
    """On curved elements: Mass = IProduct o BwdTrans; PhysDeriv o BwdTrans is
    the expansion's gradient, so IProductDeriv o PhysDeriv o BwdTrans = L; and
    the physical derivative of a linear field on an affine triangle is its
    constant gradient."""
    mesh = W.quad_tri_mesh(4)
    P, Q = 3, 5
    rng = np.random.default_rng(3)
    for shape in O2.SHAPES2:
        maps = mesh[shape].take(np.arange(5))
        jac = W.jacobian2d(maps, O2.reference_points(shape, Q), curved=True)
        x = rng.uniform(-1, 1, (5, O2.num_modes(shape, P)))
        u = O2.apply_op("bwd", shape, P, Q, jac, x)
        assert np.allclose(O2.apply_op("iprod", shape, P, Q, jac, u), O2.apply_op("mass", shape, P, Q, jac, x),
                           atol=1e-14)
        du = O2.apply_op("physderiv", shape, P, Q, jac, u)
        assert np.allclose(O2.apply_op("iprod_deriv", shape, P, Q, jac, du),
                           O2.apply_op("laplacian", shape, P, Q, jac, x), atol=1e-12)
    maps = mesh["tri"].take([0])
    jac = W.affine_jacobian2d(maps)
    xq = W._chi(maps, O2.reference_points("tri", Q))[0]           # physical points
    f = 0.3 + 1.7 * xq[:, 0] - 0.6 * xq[:, 1]
    d = O2.apply_op("physderiv", "tri", P, Q, jac, f[None, :])
    assert np.allclose(d[0, 0], 1.7, atol=1e-12) and np.allclose(d[1, 0], -0.6, atol=1e-12)
