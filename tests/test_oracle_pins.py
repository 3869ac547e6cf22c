"""Pins of the FP64 oracle against things other than itself.

Each test checks the oracle against a value fixed by mathematics: 50-digit
quadrature, closed-form integrals of monomials over the reference shapes, exact
rational element matrices from symbolic integration, the textbook P1
tetrahedron, Kronecker products of exact 1D matrices, nodal and conformity
properties of the modal basis, and invariants of the operators (Sec. 2.1-2.3).
"""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import shp_oracle as O
from paper_2604_04644_amd import workloads as W

mp = pytest.importorskip("mpmath")
sp = pytest.importorskip("sympy")


# ---------------------------------------------------------------------------
# 1D quadrature against 50-digit roots and moment equations
# ---------------------------------------------------------------------------

def _mp_jacobi(n, a, b, x):
    """P_n^(a,b)(x) from its explicit binomial sum (not the recurrence)."""
    s = mp.mpf(0)
    for k in range(n + 1):
        s += mp.binomial(n + a, n - k) * mp.binomial(n + b, k) * ((x - 1) / 2) ** k * ((x + 1) / 2) ** (n - k)
    return s


def _mp_moments(n, a, b):
    """int_{-1}^{1} x^k (1-x)^a (1+x)^b dx for k < n, exactly via Beta functions
    after expanding x = 2t - 1."""
    out = []
    for k in range(n):
        s = mp.mpf(0)
        for j in range(k + 1):
            # x^k = sum_j C(k,j) (2t)^j (-1)^(k-j); (1-x)^a (1+x)^b = 2^(a+b) (1-t)^a t^b
            s += mp.binomial(k, j) * (-1) ** (k - j) * 2 ** j * mp.beta(j + b + 1, a + 1)
        out.append(s * 2 ** (a + b + 1))
    return out


@pytest.mark.parametrize("Q", [3, 4, 6, 8, 12])
@pytest.mark.parametrize("ab", [(1, 0), (2, 0), (1, 1), (0, 0)])
def test_gauss_jacobi_vs_50_digits(Q, ab):
    mp.mp.dps = 50
    a, b = ab
    x, w = O.gauss_jacobi(Q, float(a), float(b))
    # nodes: zeros of P_Q^(a,b), polished at 50 digits
    for xi in x:
        r = mp.findroot(lambda t: _mp_jacobi(Q, a, b, t), mp.mpf(float(xi)))
        assert abs(float(r) - xi) < 2e-15
    # weights: the unique solution of the moment equations on these nodes
    X = [mp.findroot(lambda t: _mp_jacobi(Q, a, b, t), mp.mpf(float(xi))) for xi in x]
    V = mp.matrix([[X[i] ** k for i in range(Q)] for k in range(Q)])
    wex = mp.lu_solve(V, mp.matrix(_mp_moments(Q, a, b)))
    for i in range(Q):
        assert abs(float(wex[i]) - w[i]) < 1e-14 * max(1.0, abs(float(wex[i])))


@pytest.mark.parametrize("Q", [3, 4, 6, 8, 12])
@pytest.mark.parametrize("ab", [(1, 0), (2, 0), (0, 0)])
def test_gauss_radau_jacobi_vs_50_digits(Q, ab):
    """Radau rule with the node -1: the other Q-1 nodes are the zeros of
    P_{Q-1}^(a,b+1) (the polynomial that (1+x) times it must be orthogonal
    to everything of degree Q-2 under the weight), the weights solve the moment
    equations on the nodes, and the rule is exact up to degree 2Q-2 but not 2Q-1."""
    mp.mp.dps = 50
    a, b = ab
    x, w = O.gauss_radau_jacobi(Q, float(a), float(b))
    assert abs(x[0] + 1.0) < 1e-15
    X = [mp.mpf(-1)] + [mp.findroot(lambda t: _mp_jacobi(Q - 1, a, b + 1, t), mp.mpf(float(xi))) for xi in x[1:]]
    for i in range(Q):
        assert abs(float(X[i]) - x[i]) < 2e-15
    V = mp.matrix([[X[i] ** k for i in range(Q)] for k in range(Q)])
    wex = mp.lu_solve(V, mp.matrix(_mp_moments(Q, a, b)))
    for i in range(Q):
        assert abs(float(wex[i]) - w[i]) < 1e-14 * max(1.0, abs(float(wex[i])))
    mom = _mp_moments(2 * Q, a, b)
    got = [float(np.sum(w * x ** k)) for k in range(2 * Q)]
    for k in range(2 * Q - 1):
        assert abs(got[k] - float(mom[k])) < 1e-13 * max(1.0, abs(float(mom[k])))
    assert abs(got[2 * Q - 1] - float(mom[2 * Q - 1])) > 1e-8


def test_gauss_radau_jacobi_two_points_by_hand():
    """Q = 2 solved by hand from the moment equations: weight 1 - x, nodes -1
    and 0 (the zero of P_1^(1,1)), weights 2/3 and 4/3; weight (1-x)^2, nodes -1
    and -1/5 (the zero of P_1^(2,1) = 1/2 + 5x/2), weights 1 and 5/3; weight 1,
    nodes -1 and 1/3, weights 1/2 and 3/2."""
    for a, xs, ws in ((1, (-1.0, 0.0), (2 / 3, 4 / 3)), (2, (-1.0, -0.2), (1.0, 5 / 3)),
                      (0, (-1.0, 1 / 3), (0.5, 1.5))):
        x, w = O.gauss_radau_jacobi(2, float(a), 0.0)
        assert np.allclose(x, xs, rtol=0, atol=1e-15) and np.allclose(w, ws, rtol=0, atol=1e-15)


@pytest.mark.parametrize("Q", [3, 4, 5, 6, 8, 12])
def test_gll_vs_50_digits(Q):
    mp.mp.dps = 50
    x, w = O.gauss_lobatto_legendre(Q)
    assert x[0] == -1.0 and x[-1] == 1.0
    # interior nodes: zeros of P'_{Q-1}
    dP = lambda t: mp.diff(lambda s: mp.legendre(Q - 1, s), t)
    X = [mp.mpf(-1)] + [mp.findroot(dP, mp.mpf(float(xi))) for xi in x[1:-1]] + [mp.mpf(1)]
    for i in range(Q):
        assert abs(float(X[i]) - x[i]) < 2e-15
    V = mp.matrix([[X[i] ** k for i in range(Q)] for k in range(Q)])
    wex = mp.lu_solve(V, mp.matrix(_mp_moments(Q, 0, 0)))
    for i in range(Q):
        assert abs(float(wex[i]) - w[i]) < 1e-14


# ---------------------------------------------------------------------------
# Reference-shape quadrature: exact on monomials up to total degree 2Q-3
# ---------------------------------------------------------------------------

def _exact_monomial(shape, a, b, c):
    """int over the reference shape of t1^a t2^b t3^c, t = (1+xi)/2 (closed form)."""
    f = math.factorial
    if shape == "hex":
        return 8.0 / ((a + 1) * (b + 1) * (c + 1))
    if shape == "tet":
        return 8.0 * f(a) * f(b) * f(c) / f(a + b + c + 3)
    if shape == "prism":
        return 8.0 * f(a) * f(c) / f(a + c + 2) / (b + 1)
    if shape == "pyr":
        return 8.0 * f(c) * f(a + b + 2) / f(a + b + c + 3) / ((a + 1) * (b + 1))
    raise ValueError(shape)


@pytest.mark.parametrize("pts", O.POINTS)
@pytest.mark.parametrize("shape", O.SHAPES)
@pytest.mark.parametrize("Q", [3, 4, 6, 8])
def test_reference_quadrature_monomials(shape, Q, pts):
    deg = 2 * Q - 3
    for a, b, c in itertools.product(range(deg + 1), repeat=3):
        if a + b + c > deg:
            continue
        got = O.integrate_reference(
            shape, Q, lambda xi: ((1 + xi[:, 0]) / 2) ** a * ((1 + xi[:, 1]) / 2) ** b * ((1 + xi[:, 2]) / 2) ** c,
            pts)
        ex = _exact_monomial(shape, a, b, c)
        assert abs(got - ex) <= 1e-13 * max(1.0, ex), (a, b, c, got, ex)


# ---------------------------------------------------------------------------
# Basis: counts, derivatives, nodality at vertices, conformity at collapses
# ---------------------------------------------------------------------------

def _count(shape, P):
    n = P + 1
    return {"hex": n ** 3, "prism": n * n * (P + 2) // 2,
            "pyr": (P + 1) * (P + 2) * (2 * P + 3) // 6,
            "tet": (P + 1) * (P + 2) * (P + 3) // 6}[shape]


@pytest.mark.parametrize("shape", O.SHAPES)
def test_mode_counts(shape):
    for P in range(1, 11):
        assert O.num_modes(shape, P) == _count(shape, P)


@pytest.mark.parametrize("shape", O.SHAPES)
@pytest.mark.parametrize("P", [1, 2, 3, 5, 8])
def test_basis_derivative_vs_finite_difference(shape, P):
    rng = np.random.default_rng(7)
    eta = rng.uniform(-0.9, 0.9, size=(20, 3))
    _, dphi = O.basis(shape, P, eta)
    h = 1e-6
    for d in range(3):
        ep, em = eta.copy(), eta.copy()
        ep[:, d] += h
        em[:, d] -= h
        fd = (O.basis(shape, P, ep)[0] - O.basis(shape, P, em)[0]) / (2 * h)
        assert np.abs(fd - dphi[d]).max() < 1e-6 * max(1.0, np.abs(dphi[d]).max())


def _ref_vertices(shape):
    if shape == "hex":
        return [(a, b, c) for a in (-1, 1) for b in (-1, 1) for c in (-1, 1)]
    if shape == "prism":
        return [(-1, -1, -1), (1, -1, -1), (-1, 1, -1), (1, 1, -1), (-1, -1, 1), (-1, 1, 1)]
    if shape == "pyr":
        return [(-1, -1, -1), (1, -1, -1), (-1, 1, -1), (1, 1, -1), (-1, -1, 1)]
    return [(-1, -1, -1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)]


def _eta_of_xi(shape, xi):
    """Inverse collapse, with the collapsed coordinate set to 0 where undefined."""
    x1, x2, x3 = xi
    if shape == "hex":
        return (x1, x2, x3)
    if shape == "prism":
        return (2 * (1 + x1) / (1 - x3) - 1 if x3 < 1 else 0.0, x2, x3)
    if shape == "pyr":
        e1 = 2 * (1 + x1) / (1 - x3) - 1 if x3 < 1 else 0.0
        e2 = 2 * (1 + x2) / (1 - x3) - 1 if x3 < 1 else 0.0
        return (e1, e2, x3)
    e2 = 2 * (1 + x2) / (1 - x3) - 1 if x3 < 1 else 0.0
    e1 = 2 * (1 + x1) / (-x2 - x3) - 1 if (-x2 - x3) > 0 else 0.0
    return (e1, e2, x3)


@pytest.mark.parametrize("shape", O.SHAPES)
@pytest.mark.parametrize("P", [1, 2, 4, 7])
def test_vertex_modes_are_nodal(shape, P):
    """Each vertex mode is 1 at its own vertex and 0 at the others; every other
    mode vanishes at all vertices."""
    verts = _ref_vertices(shape)
    eta = np.array([_eta_of_xi(shape, v) for v in verts], dtype=float)
    phi, _ = O.basis(shape, P, eta)
    vm = set(O.VERTEX_MODES[shape])
    ml = O.modes(shape, P)
    vcols = [m for m, idx in enumerate(ml) if idx in vm]
    ocols = [m for m, idx in enumerate(ml) if idx not in vm]
    assert len(vcols) == len(verts)
    sub = phi[:, vcols]
    # a permutation matrix
    assert np.allclose(np.sort(sub, axis=1)[:, -1], 1.0, atol=1e-14)
    assert np.allclose(np.sort(sub, axis=0)[-1, :], 1.0, atol=1e-14)
    assert np.abs(sub).sum() == pytest.approx(len(verts), abs=1e-13)
    if ocols:
        assert np.abs(phi[:, ocols]).max() < 1e-14


@pytest.mark.parametrize("shape", ["prism", "pyr", "tet"])
@pytest.mark.parametrize("P", [1, 2, 3, 6])
def test_modes_single_valued_at_collapses(shape, P):
    """Where the Duffy map collapses a direction, every mode must take one value
    along the collapsed coordinate (it is a function of xi)."""
    rng = np.random.default_rng(3)
    t = rng.uniform(-1, 1, size=(12, 3))
    cases = []
    if shape in ("prism", "pyr", "tet"):
        # eta3 = 1: prism independent of eta1; pyramid and tet of eta1, eta2
        e = t.copy(); e[:, 2] = 1.0
        free = [0] if shape == "prism" else [0, 1]
        cases.append((e, free))
    if shape == "tet":
        e = t.copy(); e[:, 1] = 1.0
        cases.append((e, [0]))
    for e, free in cases:
        ref = e.copy()
        for d in free:
            ref[:, d] = 0.123
        a = O.basis(shape, P, e)[0]
        b = O.basis(shape, P, ref)[0]
        assert np.abs(a - b).max() < 1e-14


def _monomials_total(P):
    return [(a, b, c) for a in range(P + 1) for b in range(P + 1) for c in range(P + 1) if a + b + c <= P]


@pytest.mark.parametrize("P", [1, 2, 3, 4, 6])
def test_tet_basis_spans_total_degree_polynomials(P):
    """The tet modes are polynomials of total degree <= P in xi and span that
    space (same dimension, full rank fit)."""
    rng = np.random.default_rng(11)
    # random points inside the reference tet
    pts = []
    while len(pts) < 300:
        x = rng.uniform(-1, 1, 3)
        if x.sum() <= -1 + 1e-3 and x.sum() < -1.0 - 1e-9 + 2:
            if x.sum() <= -1:
                pts.append(x)
    xi = np.array(pts)
    eta = np.array([_eta_of_xi("tet", x) for x in xi])
    phi, _ = O.basis("tet", P, eta)
    mons = _monomials_total(P)
    V = np.stack([xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c for a, b, c in mons], axis=1)
    coef, *_ = np.linalg.lstsq(V, phi, rcond=None)
    assert np.abs(V @ coef - phi).max() < 1e-10
    assert len(mons) == O.num_modes("tet", P)
    assert np.linalg.matrix_rank(coef, tol=1e-10) == len(mons)


@pytest.mark.parametrize("P", [1, 2, 3, 5])
def test_prism_basis_spans_prism_space(P):
    """Prism modes: polynomials of total degree <= P in (xi1, xi3) times degree
    <= P in xi2, spanning that space."""
    rng = np.random.default_rng(12)
    pts = []
    while len(pts) < 400:
        x = rng.uniform(-1, 1, 3)
        if x[0] + x[2] <= 0:
            pts.append(x)
    xi = np.array(pts)
    eta = np.array([_eta_of_xi("prism", x) for x in xi])
    phi, _ = O.basis("prism", P, eta)
    mons = [(a, b, c) for a in range(P + 1) for b in range(P + 1) for c in range(P + 1) if a + c <= P]
    V = np.stack([xi[:, 0] ** a * xi[:, 1] ** b * xi[:, 2] ** c for a, b, c in mons], axis=1)
    coef, *_ = np.linalg.lstsq(V, phi, rcond=None)
    assert np.abs(V @ coef - phi).max() < 1e-10
    assert len(mons) == O.num_modes("prism", P)
    assert np.linalg.matrix_rank(coef, tol=1e-10) == len(mons)


# ---------------------------------------------------------------------------
# Element matrices
# ---------------------------------------------------------------------------

_AFF = [[1.5, 0.2, 0.0], [-0.25, 1.0, 1.0 / 3.0], [1.0 / 7.0, 0.0, 0.8]]
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.mark.parametrize("pts", O.POINTS)
@pytest.mark.parametrize("shape", O.SHAPES)
@pytest.mark.parametrize("P", [1, 2])
def test_element_matrices_exact_rational(shape, P, pts):
    """Oracle M, L of an affine element against exact symbolic integrals
    (tests/golden/make_exact_matrices.py).  The integrands are polynomials that
    both point sets integrate exactly at Q = P + 2, so the Radau rule must give
    the same matrices."""
    Mx = np.loadtxt(os.path.join(GOLDEN, f"exact_M_{shape}_P{P}.txt"))
    Lx = np.loadtxt(os.path.join(GOLDEN, f"exact_L_{shape}_P{P}.txt"))
    Q = P + 2
    jac = np.array([[v for row in _AFF for v in row]])
    el = O.Element(shape, P, Q, jac, pts)
    M, L = el.mass()[0], el.laplacian()[0]
    assert np.abs(M - Mx).max() < 1e-14 * np.abs(Mx).max() * 10
    assert np.abs(L - Lx).max() < 1e-13 * np.abs(Lx).max()


def test_p1_tet_textbook():
    """P=1 tet: vertex modes are the barycentric coordinates; M = V/20 (1 + delta)
    and L_ij = V grad(lambda_i).grad(lambda_j) with gradients from the vertices."""
    maps = W.shape_batch("tet", 5)
    Q = 3
    jac = W.affine_jacobian(maps)
    el = O.Element("tet", 1, Q, jac)
    M, L = el.mass(), el.laplacian()
    # mode order (0,0,0),(0,0,1),(0,1,0),(1,0,0) -> lambda_0, lambda_3, lambda_2, lambda_1
    ref = np.array([[-1, -1, -1], [-1, -1, 1], [-1, 1, -1], [1, -1, -1]], dtype=float)
    for e in range(5):
        X = (maps.x0[e][None, :] + (maps.A[e] @ ((1 + ref.T) / 2)).T)   # vertices in mode order
        T = np.hstack([np.ones((4, 1)), X])
        V = abs(np.linalg.det(T)) / 6
        grads = np.linalg.inv(T)[1:, :].T                                  # [4 vertices, 3]
        Mref = V / 20 * (np.ones((4, 4)) + np.eye(4))
        Lref = V * grads @ grads.T
        assert np.abs(M[e] - Mref).max() < 1e-15 + 1e-13 * Mref.max()
        assert np.abs(L[e] - Lref).max() < 1e-13 * np.abs(Lref).max()


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


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_affine_hex_kronecker(P):
    """Cube of side h: H = lam (h/2)^3 M1 x M1 x M1 + (h/2)(K1 x M1 x M1 + ...)."""
    M1, K1 = _exact_1d(P)
    maps = W.affine_hex_grid(4)
    h = 0.25
    lam = 1.0
    el = O.Element("hex", P, P + 2, W.affine_jacobian(maps.take([0, 5])))
    H = el.helmholtz(lam)
    kron = lambda a, b, c: np.kron(np.kron(a, b), c)
    Href = lam * (h / 2) ** 3 * kron(M1, M1, M1) + (h / 2) * (kron(K1, M1, M1) + kron(M1, K1, M1) + kron(M1, M1, K1))
    for e in range(2):
        assert np.abs(H[e] - Href).max() < 1e-13 * np.abs(Href).max()


@pytest.mark.parametrize("shape,P,pts", [(s, P, "gj") for s in O.SHAPES for P in (1, 3, 4)] +
                         [(s, 3, "radau") for s in O.SHAPES])
def test_curved_invariants(shape, P, pts):
    """M, L symmetric; M positive definite; L positive semidefinite with the
    constants as its one-dimensional kernel; L 1 = 0."""
    Q = P + 2
    maps = W.shape_batch(shape, 24)
    jac = W.jacobian(maps, O.reference_points(shape, Q, pts), curved=True)
    el = O.Element(shape, P, Q, jac, pts)
    M, L = el.mass(), el.laplacian()
    c1 = O.vertex_indicator(shape, P)
    assert np.abs(M - np.transpose(M, (0, 2, 1))).max() < 1e-17 + 1e-14 * np.abs(M).max()
    assert np.abs(L - np.transpose(L, (0, 2, 1))).max() < 1e-14 * np.abs(L).max()
    assert np.abs(L @ c1).max() < 1e-13 * np.abs(L).max()
    evM = np.linalg.eigvalsh(M)
    assert evM.min() > 0
    evL = np.linalg.eigvalsh(L)
    scale = evL[:, -1]
    assert np.all(np.abs(evL[:, 0]) < 1e-12 * scale)
    assert np.all(evL[:, 1] > 1e-9 * scale)


@pytest.mark.parametrize("P", [2, 4])
def test_mixed_mesh_volume(P):
    """sum_e 1^T M_e 1 = 1 for the unit cube and 1/4 per quadrant (the perturbation
    fixes the planes x, y in {0, 1/2, 1}); exact for the affine mesh."""
    mesh = W.quadrant_mesh(4)
    Q = P + 2
    for curved, tol in ((False, 1e-13), (True, 2e-4 if P == 2 else 2e-6)):
        total = 0.0
        for shape, maps in mesh.items():
            jac = W.jacobian(maps, O.reference_points(shape, Q), curved=curved)
            el = O.Element(shape, P, Q, jac)
            c1 = O.vertex_indicator(shape, P)
            vol = float(np.einsum("m,emn,n->", c1, el.mass(), c1))
            assert abs(vol - 0.25) < tol, (shape, curved, vol)
            total += vol
        assert abs(total - 1.0) < 4 * tol


@pytest.mark.parametrize("pts", O.POINTS)
@pytest.mark.parametrize("shape", O.SHAPES)
def test_collocation_derivative_exact_on_polynomials(shape, pts):
    """The Vandermonde collocation derivative differentiates polynomials of
    degree <= Q-1 per direction exactly."""
    Q = 5
    eta, _, _ = O.quadrature(shape, Q, pts)
    D = O.deriv_matrices(shape, Q, pts)
    u = eta[:, 0] ** 4 * eta[:, 1] ** 3 - 2 * eta[:, 2] ** 4 * eta[:, 0] + eta[:, 1] * eta[:, 2] ** 2
    du = [4 * eta[:, 0] ** 3 * eta[:, 1] ** 3 - 2 * eta[:, 2] ** 4,
          3 * eta[:, 0] ** 4 * eta[:, 1] ** 2 + eta[:, 2] ** 2,
          -8 * eta[:, 2] ** 3 * eta[:, 0] + 2 * eta[:, 1] * eta[:, 2]]
    for d in range(3):
        assert np.abs(D[d] @ u - du[d]).max() < 1e-12


@pytest.mark.parametrize("pts", O.POINTS)
@pytest.mark.parametrize("shape", O.SHAPES)
@pytest.mark.parametrize("P", [1, 3])
def test_cross_operator_identities(shape, P, pts):
    """PhysDeriv(BwdTrans x) = sum x_m grad phi_m (analytic); the weak Laplacian
    equals IProductDeriv(PhysDeriv(BwdTrans x)); mass = IProduct(BwdTrans x)."""
    Q = P + 2
    maps = W.shape_batch(shape, 9)
    jac = W.jacobian(maps, O.reference_points(shape, Q, pts), curved=True)
    el = O.Element(shape, P, Q, jac, pts)
    x = W.coeffs(9, O.num_modes(shape, P), 5)
    u = el.bwd_trans(x)
    g = el.phys_deriv(u)
    ga = np.einsum("eiqm,em->ieq", el.dBx, x)
    assert np.abs(g - ga).max() < 1e-11 * np.abs(ga).max()
    Lx = el.laplacian_action(x)
    assert np.abs(el.iproduct_deriv(g) - Lx).max() < 1e-11 * np.abs(Lx).max()
    Mx = el.mass_action(x)
    assert np.abs(el.iproduct(u) - Mx).max() < 1e-13 * np.abs(Mx).max()


@pytest.mark.parametrize("shape", O.SHAPES)
def test_physderiv_linear_field_affine(shape):
    """On straight-sided elements the gradient of a linear field is its constant."""
    P, Q = 2, 4
    maps = W.shape_batch(shape, 6)
    xi = O.reference_points(shape, Q)
    X = W.coords(maps, xi, curved=False)
    a = np.array([0.3, -1.2, 2.5])
    u = np.einsum("i,eiq->eq", a, X) + 0.7
    g = O.apply_op("physderiv", shape, P, Q, W.jacobian(maps, xi, curved=False), u)
    for i in range(3):
        assert np.abs(g[i] - a[i]).max() < 1e-11


@pytest.mark.parametrize("shape", O.SHAPES)
def test_helmholtz_solve_round_trip(shape):
    P, Q = 3, 5
    maps = W.shape_batch(shape, 5)
    jac = W.jacobian(maps, O.reference_points(shape, Q), curved=True)
    x = W.coeffs(5, O.num_modes(shape, P), 2)
    b = O.apply_op("helmholtz", shape, P, Q, jac, x, lam=1.0)
    xs = O.helmholtz_solve(shape, P, Q, jac, b, lam=1.0)
    assert np.abs(xs - x).max() < 1e-8


@pytest.mark.parametrize("shape", O.SHAPES)
@pytest.mark.parametrize("P", [1, 3])
def test_advection_of_linear_fields(shape, P):
    """Advection term of the advection-diffusion-reaction operator on affine
    elements with a constant velocity b: b . grad f of a linear field f = a.x + c
    is the constant b.a, so C x_f = (b.a) M 1 (M 1 the mass matrix applied to the
    constant's coefficients); constants are not advected (C 1 = 0).  The
    transposed operator fails this, and so does a wrong sign or component."""
    Q = P + 2
    maps = W.shape_batch(shape, 4)
    xi = O.reference_points(shape, Q)
    X = W.coords(maps, xi, curved=False)                     # [ne, 3, nq]
    el = O.Element(shape, P, Q, W.affine_jacobian(maps))
    b = np.array([0.7, -1.3, 0.4])
    a = np.array([0.3, -1.2, 2.5])
    vel = np.broadcast_to(b[:, None, None], (3, len(maps), Q ** 3))
    C, M = el.advection(vel), el.mass()
    c1 = O.vertex_indicator(shape, P)
    for e in range(len(maps)):
        f = a @ X[e] + 0.4
        xf = np.linalg.lstsq(el.B, f, rcond=None)[0]           # exact: f lies in the span
        assert np.abs(el.B @ xf - f).max() < 1e-12
        lhs, rhs = C[e] @ xf, (b @ a) * (M[e] @ c1)
        assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()
        assert np.abs(C[e] @ c1).max() < 1e-13 * np.abs(C[e]).max()
        assert np.abs(C[e].T @ xf - rhs).max() > 1e-3 * np.abs(rhs).max()


# ---------------------------------------------------------------------------
# iso-parametric geometry (J from coordinate coefficients)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("shape", O.SHAPES)
def test_isoparametric_jacobian_affine_vertices(shape):
    """Vertex positions of straight-sided elements on the vertex coefficients
    (all others zero) reproduce the affine map: J equals the element's constant
    d x/d xi at every point, for several orders."""
    maps = W.shape_batch(shape, 7)
    for P in (1, 2, 4):
        idx, vxi = O.vertex_modes(shape, P)
        X = np.zeros((7, 3, O.num_modes(shape, P)))
        X[:, :, idx] = W.coords(maps, vxi, curved=False)
        J = O.isoparametric_jacobian(shape, P, P + 2, X)
        assert np.abs(J - W.affine_jacobian(maps)[:, :, None]).max() < 1e-14


def _quadratic_map(xi, c):
    x = xi.copy()
    x[..., 0] += c * xi[..., 0] ** 2
    x[..., 1] += c * xi[..., 1] * xi[..., 2]
    x[..., 2] += c * xi[..., 0] * xi[..., 2]
    return x


def _quadratic_jac(xi, c):
    J = np.broadcast_to(np.eye(3), xi.shape[:-1] + (3, 3)).copy()
    J[..., 0, 0] += 2 * c * xi[..., 0]
    J[..., 1, 1] += c * xi[..., 2]
    J[..., 1, 2] += c * xi[..., 1]
    J[..., 2, 0] += c * xi[..., 2]
    J[..., 2, 2] += c * xi[..., 0]
    return J


@pytest.mark.parametrize("pts", ["gj", "radau"])
@pytest.mark.parametrize("shape", O.SHAPES)
def test_isoparametric_jacobian_quadratic_map(shape, pts):
    """A quadratic map x = xi + c (xi1^2, xi2 xi3, xi1 xi3) lies in every
    shape's space at P >= 2; its coefficients (least squares through the
    quadrature points, exact for a map in the space) give J equal to the
    analytic gradient at the points."""
    P, Q, c = 3, 5, 0.15
    eta, _, _ = O.quadrature(shape, Q, pts)
    xi = O.collapse(shape, eta)
    B, _ = O.basis(shape, P, eta)
    coef, *_ = np.linalg.lstsq(B, _quadratic_map(xi, c), rcond=None)     # [N_P, 3]
    assert np.abs(B @ coef - _quadratic_map(xi, c)).max() < 1e-13     # the map is in the space
    J = O.isoparametric_jacobian(shape, P, Q, coef.T[None, :, :], pts)[0]
    Ja = np.transpose(_quadratic_jac(xi, c).reshape(-1, 9), (1, 0))
    assert np.abs(J - Ja).max() < 1e-12
