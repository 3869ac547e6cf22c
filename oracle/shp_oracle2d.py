"""FP64 CPU oracle for the two-dimensional elemental operators (quadrilaterals
and triangles).

TEST INFRASTRUCTURE ONLY, like oracle.shp_oracle (whose 1D Jacobi polynomials,
Golub-Welsch rules, modified-basis functions and Vandermonde collocation
derivative it uses): only the tests and the benchmark's CPU baseline may import
it, and it shares no code with the HIP library.  Every operator is a dense
elemental matrix formed by explicit quadrature and applied as a matrix-vector
product.

What it computes, with the paper's passages:

* the two-dimensional discrete Helmholtz operator H = lambda M + L, by tensor
  quadrature of lambda phi_m phi_n |J| and (J^-T grad phi_m).(J^-T grad phi_n)
  |J| over the Q x Q points (Sec. 2.2, eq. helm);
* M = B^T W B with B the basis at the points and W the weights times |J|
  (Sec. 2.2, eq. mass); the Laplacian through the chain rule d/dx = (d eta/d x)
  d/d eta (Sec. 2.2, eq. Lap);
* the triangle as the collapsed square: xi_1 = (1 + eta_1)(1 - eta_2)/2 - 1,
  xi_2 = eta_2 (Sec. 2.3, the Duffy map), tensor quadrature in eta;
* the physical derivative of the Lagrange interpolant through the points
  (Sec. 2.2, eq. dphitodh), chained with d eta/d x.

Readings (the paper points to its textbook): the modified basis of the 3D
oracle restricted to two directions,
    quad  A_p(eta1) A_q(eta2)                 0 <= p, q <= P
    tri   A_p(eta1) C_{p,q}(eta2)             p + q <= P;  (0,1) -> v1(eta2)
modes (p, q) lexicographic with q fastest; Q points per direction,
Gauss-Lobatto-Legendre in eta1 (and in eta2 of the quadrilateral), Gauss-Jacobi
(1,0) or Gauss-Radau-Jacobi (1,0) in the triangle's collapsed eta2, the Jacobi
weight (1 - eta2) divided back out; point index i*Q + j with j (eta2) fastest.
"""
from __future__ import annotations

import numpy as np

from oracle.shp_oracle import dA, dC, fA, fC, lagrange_deriv_1d, rule_1d

SHAPES2 = ("quad", "tri")
ALPHA2 = {"quad": (0, 0), "tri": (0, 1)}
AREA = {"quad": 4.0, "tri": 2.0}
# vertex modes and the reference vertices where each is one
VERTEX_MODES2 = {"quad": [(0, 0), (0, 1), (1, 0), (1, 1)], "tri": [(0, 0), (1, 0), (0, 1)]}
VERTEX_XI2 = {"quad": [(-1, -1), (-1, 1), (1, -1), (1, 1)], "tri": [(-1, -1), (1, -1), (-1, 1)]}


def modes(shape: str, P: int):
    if shape == "quad":
        return [(p, q) for p in range(P + 1) for q in range(P + 1)]
    if shape == "tri":
        return [(p, q) for p in range(P + 1) for q in range(P + 1 - p)]
    raise ValueError(shape)


def num_modes(shape: str, P: int) -> int:
    return len(modes(shape, P))


def collapse(shape: str, eta: np.ndarray) -> np.ndarray:
    """eta -> xi (identity for the quadrilateral, the Duffy map for the triangle)."""
    e1, e2 = eta[..., 0], eta[..., 1]
    if shape == "quad":
        return np.stack([e1, e2], axis=-1)
    return np.stack([0.5 * (1 + e1) * (1 - e2) - 1, e2], axis=-1)


def dxi_deta(shape: str, eta: np.ndarray) -> np.ndarray:
    """d xi_a / d eta_b [..., 2, 2]."""
    e1, e2 = eta[..., 0], eta[..., 1]
    M = np.zeros(eta.shape[:-1] + (2, 2))
    M[..., 0, 0] = M[..., 1, 1] = 1.0
    if shape == "tri":
        M[..., 0, 0] = 0.5 * (1 - e2)
        M[..., 0, 1] = -0.5 * (1 + e1)
    return M


def quadrature(shape: str, Q: int, pts: str = "gj"):
    """Points eta [Q^2, 2] (j fastest), products of the 1D weights [Q^2] and the
    divisor (1 - eta2)^alpha of the collapsed direction's Jacobi weight."""
    (z1, w1), (z2, w2) = (rule_1d(Q, a, pts) for a in ALPHA2[shape])
    E1, E2 = np.meshgrid(z1, z2, indexing="ij")
    eta = np.stack([E1.ravel(), E2.ravel()], axis=1)
    w = np.outer(w1, w2).ravel()
    div = (1 - eta[:, 1]) ** ALPHA2[shape][1]
    return eta, w, div


def reference_points(shape: str, Q: int, pts: str = "gj") -> np.ndarray:
    eta, _, _ = quadrature(shape, Q, pts)
    return collapse(shape, eta)


def integrate_reference(shape: str, Q: int, f, pts: str = "gj") -> float:
    eta, w, div = quadrature(shape, Q, pts)
    det = np.linalg.det(dxi_deta(shape, eta))
    return float(np.sum(w * det / div * f(collapse(shape, eta))))


def _factors(shape: str, p: int, q: int):
    """(eta1 factor, eta2 factor); None is the constant 1."""
    if shape == "quad":
        return (fA, dA, p), (fA, dA, q)
    if p == 0 and q == 1:
        return None, "v1"
    return (fA, dA, p), (fC, dC, p, q)


def _eval(fac, z, deriv):
    z = np.asarray(z, dtype=np.float64)
    if fac is None:
        return np.zeros_like(z) if deriv else np.ones_like(z)
    if fac == "v1":
        return np.full_like(z, 0.5) if deriv else 0.5 * (1 + z)
    f, df, *args = fac
    return df(*args, z) if deriv else f(*args, z)


def basis(shape: str, P: int, eta: np.ndarray):
    """phi [n_pts, N_P] and d phi/d eta_d [2, n_pts, N_P]."""
    ml = modes(shape, P)
    phi = np.empty((eta.shape[0], len(ml)))
    dphi = np.empty((2, eta.shape[0], len(ml)))
    for m, (p, q) in enumerate(ml):
        a, b = _factors(shape, p, q)
        va, vb = _eval(a, eta[:, 0], False), _eval(b, eta[:, 1], False)
        phi[:, m] = va * vb
        dphi[0, :, m] = _eval(a, eta[:, 0], True) * vb
        dphi[1, :, m] = va * _eval(b, eta[:, 1], True)
    return phi, dphi


def vertex_modes(shape: str, P: int):
    ml = modes(shape, P)
    return [ml.index(m) for m in VERTEX_MODES2[shape]], np.array(VERTEX_XI2[shape], dtype=np.float64)


def geometry(shape: str, Q: int, jac, pts: str = "gj"):
    """jw = w |det d x/d eta| / (1 - eta2)^alpha and d eta_d/d x_i (numerical
    2x2 inverse of (d x/d xi)(d xi/d eta)).  jac: d x_i/d xi_j at component
    i*2 + j, [n_elem][4][n_pts] or constant [n_elem][4]."""
    eta, w, div = quadrature(shape, Q, pts)
    npts = eta.shape[0]
    jac = np.asarray(jac, dtype=np.float64)
    if jac.ndim == 2:
        Jxi = np.broadcast_to(jac.reshape(-1, 1, 2, 2), (jac.shape[0], npts, 2, 2))
    else:
        Jxi = np.transpose(jac, (0, 2, 1)).reshape(jac.shape[0], npts, 2, 2)
    Jeta = np.einsum("epia,pab->epib", Jxi, dxi_deta(shape, eta))
    det = np.linalg.det(Jeta)
    if np.any(~np.isfinite(det)) or np.any(det <= 0):
        raise ValueError("non-positive or non-finite Jacobian")
    return w[None, :] * det / div[None, :], np.linalg.inv(Jeta)


def deriv_matrices(shape: str, Q: int, pts: str = "gj"):
    """Collocation derivatives in eta1 and eta2 on the tensor points [Q^2, Q^2]."""
    (z1, _), (z2, _) = (rule_1d(Q, a, pts) for a in ALPHA2[shape])
    I = np.eye(Q)
    return [np.kron(lagrange_deriv_1d(z1), I), np.kron(I, lagrange_deriv_1d(z2))]


class Element2D:
    """Dense operators of a batch of 2D elements of one shape."""

    def __init__(self, shape: str, P: int, Q: int, jac, pts: str = "gj"):
        self.shape, self.P, self.Q, self.pts = shape, P, Q, pts
        eta, _, _ = quadrature(shape, Q, pts)
        self.B, self.dB = basis(shape, P, eta)
        self.jw, self.G = geometry(shape, Q, jac, pts)          # [ne, nq], [ne, nq, d, i]
        self.dBx = np.einsum("eqdi,dqm->eiqm", self.G, self.dB)  # d phi/d x_i at the points

    def mass(self):
        return np.matmul(self.B.T[None], self.jw[:, :, None] * self.B[None])

    def laplacian(self):
        L = np.zeros((self.jw.shape[0], self.B.shape[1], self.B.shape[1]))
        for i in range(2):
            Bi = self.dBx[:, i]
            L += np.matmul(np.transpose(Bi, (0, 2, 1)), self.jw[:, :, None] * Bi)
        return L

    def helmholtz(self, lam: float):
        return lam * self.mass() + self.laplacian()


def apply_op(op: str, shape: str, P: int, Q: int, jac, x, lam: float = 1.0, pts: str = "gj"):
    """op in {bwd, iprod, physderiv, iprod_deriv, mass, laplacian, helmholtz};
    x: [n_elem][N_P] or [n_elem][Q^2] or [2][n_elem][Q^2] (iprod_deriv)."""
    x = np.asarray(x, dtype=np.float64)
    el = Element2D(shape, P, Q, jac, pts)
    if op == "bwd":
        return np.einsum("qm,em->eq", el.B, x)
    if op == "iprod":
        return np.einsum("qm,eq->em", el.B, el.jw * x)
    if op == "physderiv":
        D = deriv_matrices(shape, Q, pts)
        du = np.stack([x @ Dd.T for Dd in D], axis=0)
        return np.einsum("eqdi,deq->ieq", el.G, du)
    if op == "iprod_deriv":
        return np.einsum("eiqm,eq,ieq->em", el.dBx, el.jw, x)
    if op == "mass":
        A = el.mass()
    elif op == "laplacian":
        A = el.laplacian()
    elif op == "helmholtz":
        A = el.helmholtz(lam)
    else:
        raise ValueError(op)
    return np.einsum("emn,en->em", A, x)
