"""FP64 CPU oracle for the elemental spectral/hp operators.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; the product path never does.  It shares
no code with the HIP library: its quadrature is Golub-Welsch (eigenvalues of the
Jacobi matrix), its collocation derivative is built from a Legendre Vandermonde
matrix, its inverse metric is a numerical 3x3 inverse of d x / d eta, and every
operator is a dense elemental matrix formed by explicit quadrature and applied
as a matrix-vector product.

What it computes, with the paper's passages:

* the discrete elemental Helmholtz operator H = lambda M + L, formed by explicit
  tensor-product quadrature of lambda phi_n phi_m + (J^-T grad phi_n).(J^-T grad
  phi_m) weighted by |J| (Sec. 2.1, eq. of H^e_delta and the split H = lambda M + L);
* the mass matrix M = B^T W B, with B the basis evaluated at the quadrature points
  and W the diagonal of weights times |J| (Sec. 2.2, eq. mass);
* the Laplacian written with the chain rule d/dx = (d eta/d x) d/d eta
  (Sec. 2.2, the expansion of L and eq. Lap);
* the collapsed (Duffy) coordinates of the non-hexahedral shapes and tensor
  quadrature on [-1,1]^3 in eta (Sec. 2.3);
* the physical derivative: the derivative of the tensor Lagrange interpolant
  through the quadrature points, chained with d eta/d x (Sec. 2.2, collocation
  differentiation, eq. dphitodh);
* the advection-diffusion-reaction operator lambda M + L + C with
  C[m,n] = integral phi_m b . grad phi_n for a velocity b given at the points,
  the operator the collocated reading of the Helmholtz action extends to
  (Sec. 2.2.1).

Readings of what the paper leaves to its textbook reference (each also listed in
the design notes):

* modified C0 modal basis: A_0 = (1-z)/2, A_1 = (1+z)/2,
  A_p = (1-z)/2 (1+z)/2 P^(1,1)_{p-2}(z); C_{0,r} = A_r; for k >= 1
  C_{k,0} = ((1-z)/2)^k and C_{k,r} = ((1-z)/2)^k (1+z)/2 P^(2k-1,1)_{r-1}(z);
* modes (p,q,r), lexicographic with r fastest:
    hex   A_p A_q A_r                         0 <= p,q,r <= P
    prism A_p A_q C_{p,r}                     r <= P-p;  (0,q,1) -> A_q(eta2) v1(eta3)
    pyr   A_p A_q C_{max(p,q),r}              r <= P-max(p,q);  (0,0,1) -> v1(eta3)
    tet   A_p C_{p,q} C_{p+q,r}               p+q+r <= P;  (0,0,1) -> v1(eta3),
                                              (0,1,r) -> v1(eta2) C_{1,r}(eta3)
* quadrature, Q points per direction: Gauss-Lobatto-Legendre in the directions
  that are not collapsed, Gauss-Jacobi (alpha,0) in a direction collapsed alpha
  times (prism eta3: 1; pyramid eta3: 2; tet eta2: 1, eta3: 2), or on request
  Gauss-Radau-Jacobi (alpha,0) there, which includes eta = -1; the Jacobi weight
  (1-eta)^alpha is divided back out of the integrand;
* point index (i*Q + j)*Q + k with k (eta3) fastest.

Parity pins: every function here is pinned in tests/test_oracle_pins.py against
closed forms, exact rational integrals, textbook P1 element matrices, 50-digit
quadrature and invariants of the operators.
"""
from __future__ import annotations

import math

import numpy as np

SHAPES = ("hex", "prism", "pyr", "tet")


# ---------------------------------------------------------------------------
# 1D: Jacobi polynomials
# ---------------------------------------------------------------------------

def jacobi(n: int, a: float, b: float, x):
    """Classical Jacobi polynomial P_n^(a,b)(x) by its three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if n == 0:
        return p0
    p1 = 0.5 * (a - b + (a + b + 2.0) * x)
    for k in range(2, n + 1):
        c = 2.0 * k + a + b
        a1 = 2.0 * k * (k + a + b) * (c - 2.0)
        a2 = (c - 1.0) * (a * a - b * b)
        a3 = (c - 2.0) * (c - 1.0) * c
        a4 = 2.0 * (k + a - 1.0) * (k + b - 1.0) * c
        p0, p1 = p1, ((a2 + a3 * x) * p1 - a4 * p0) / a1
    return p1


def jacobi_deriv(n: int, a: float, b: float, x):
    """d/dx P_n^(a,b) = (n + a + b + 1)/2 P_{n-1}^(a+1,b+1)."""
    x = np.asarray(x, dtype=np.float64)
    if n == 0:
        return np.zeros_like(x)
    return 0.5 * (n + a + b + 1.0) * jacobi(n - 1, a + 1.0, b + 1.0, x)


# ---------------------------------------------------------------------------
# 1D quadrature (Golub-Welsch)
# ---------------------------------------------------------------------------

def gauss_jacobi(Q: int, a: float, b: float):
    """Q-point Gauss rule for the weight (1-x)^a (1+x)^b on [-1,1]: nodes are the
    eigenvalues of the symmetric Jacobi matrix of the monic recurrence, weights
    mu0 times the squared first eigenvector components."""
    k = np.arange(Q, dtype=np.float64)
    alpha = np.empty(Q)
    alpha[0] = (b - a) / (a + b + 2.0)
    kk = k[1:]
    c = 2.0 * kk + a + b
    alpha[1:] = (b * b - a * a) / (c * (c + 2.0))
    kb = np.arange(1, Q, dtype=np.float64)
    c = 2.0 * kb + a + b
    beta = 4.0 * kb * (kb + a) * (kb + b) * (kb + a + b) / (c * c * (c + 1.0) * (c - 1.0))
    T = np.diag(alpha) + np.diag(np.sqrt(beta), 1) + np.diag(np.sqrt(beta), -1)
    x, V = np.linalg.eigh(T)
    mu0 = 2.0 ** (a + b + 1.0) * math.gamma(a + 1.0) * math.gamma(b + 1.0) / math.gamma(a + b + 2.0)
    w = mu0 * V[0, :] ** 2
    return x, w


def gauss_radau_jacobi(Q: int, a: float, b: float):
    """Q-point Gauss-Radau rule for the weight (1-x)^a (1+x)^b with the node
    x = -1 fixed (Golub's modification of Golub-Welsch): the last diagonal entry
    of the Jacobi matrix is replaced so that the monic degree-Q polynomial of
    the modified recurrence vanishes at -1, i.e.
    alpha'_{Q-1} = -1 - beta_{Q-1} p_{Q-2}(-1) / p_{Q-1}(-1) with p_k the monic
    orthogonal polynomials; nodes and weights then follow as in gauss_jacobi."""
    if Q == 1:
        mu0 = 2.0 ** (a + b + 1.0) * math.gamma(a + 1.0) * math.gamma(b + 1.0) / math.gamma(a + b + 2.0)
        return np.array([-1.0]), np.array([mu0])
    k = np.arange(Q, dtype=np.float64)
    alpha = np.empty(Q)
    alpha[0] = (b - a) / (a + b + 2.0)
    c = 2.0 * k[1:] + a + b
    alpha[1:] = (b * b - a * a) / (c * (c + 2.0))
    kb = np.arange(1, Q, dtype=np.float64)
    c = 2.0 * kb + a + b
    beta = 4.0 * kb * (kb + a) * (kb + b) * (kb + a + b) / (c * c * (c + 1.0) * (c - 1.0))
    # monic p_0 .. p_{Q-1} at x = -1 by the three-term recurrence
    pm, pk = 0.0, 1.0
    for j in range(Q - 1):
        pm, pk = pk, (-1.0 - alpha[j]) * pk - (beta[j - 1] * pm if j > 0 else 0.0)
    alpha_mod = alpha.copy()
    alpha_mod[Q - 1] = -1.0 - beta[Q - 2] * pm / pk
    T = np.diag(alpha_mod) + np.diag(np.sqrt(beta), 1) + np.diag(np.sqrt(beta), -1)
    x, V = np.linalg.eigh(T)
    mu0 = 2.0 ** (a + b + 1.0) * math.gamma(a + 1.0) * math.gamma(b + 1.0) / math.gamma(a + b + 2.0)
    w = mu0 * V[0, :] ** 2
    return x, w


def gauss_lobatto_legendre(Q: int):
    """Q-point Gauss-Lobatto-Legendre rule: the end points and the zeros of
    P'_{Q-1} (the Gauss-Jacobi(1,1) nodes), weights 2 / (Q (Q-1) P_{Q-1}(x)^2)."""
    if Q < 2:
        raise ValueError("GLL needs Q >= 2")
    inner = gauss_jacobi(Q - 2, 1.0, 1.0)[0] if Q > 2 else np.zeros(0)
    x = np.concatenate([[-1.0], inner, [1.0]])
    PL = jacobi(Q - 1, 0.0, 0.0, x)
    w = 2.0 / (Q * (Q - 1) * PL ** 2)
    return x, w


# ---------------------------------------------------------------------------
# Reference shapes: collapse maps and per-direction rules
# ---------------------------------------------------------------------------

# Jacobi exponent alpha of the rule in each eta direction (0 means GLL)
ALPHA = {"hex": (0, 0, 0), "prism": (0, 0, 1), "pyr": (0, 0, 2), "tet": (0, 1, 2)}
VOLUME = {"hex": 8.0, "prism": 4.0, "pyr": 8.0 / 3.0, "tet": 4.0 / 3.0}


POINTS = ("gj", "radau")


def rule_1d(Q: int, alpha: int, pts: str = "gj"):
    """GLL in a direction that is not collapsed; in a direction collapsed alpha
    times, Gauss-Jacobi(alpha,0) ("gj") or Gauss-Radau-Jacobi(alpha,0) with the
    node -1 ("radau")."""
    if pts not in POINTS:
        raise ValueError(pts)
    if alpha == 0:
        return gauss_lobatto_legendre(Q)
    if pts == "radau":
        return gauss_radau_jacobi(Q, float(alpha), 0.0)
    return gauss_jacobi(Q, float(alpha), 0.0)


def collapse(shape: str, eta: np.ndarray) -> np.ndarray:
    """Collapsed coordinates eta -> reference coordinates xi (Duffy maps)."""
    e1, e2, e3 = eta[..., 0], eta[..., 1], eta[..., 2]
    if shape == "hex":
        x1, x2, x3 = e1, e2, e3
    elif shape == "prism":
        x1, x2, x3 = 0.5 * (1 + e1) * (1 - e3) - 1, e2, e3
    elif shape == "pyr":
        x1 = 0.5 * (1 + e1) * (1 - e3) - 1
        x2 = 0.5 * (1 + e2) * (1 - e3) - 1
        x3 = e3
    elif shape == "tet":
        x1 = 0.25 * (1 + e1) * (1 - e2) * (1 - e3) - 1
        x2 = 0.5 * (1 + e2) * (1 - e3) - 1
        x3 = e3
    else:
        raise ValueError(shape)
    return np.stack([x1, x2, x3], axis=-1)


def dxi_deta(shape: str, eta: np.ndarray) -> np.ndarray:
    """d xi_a / d eta_b of the collapse map, [..., 3, 3] (row a, column b)."""
    e1, e2, e3 = eta[..., 0], eta[..., 1], eta[..., 2]
    M = np.zeros(eta.shape[:-1] + (3, 3))
    M[..., 0, 0] = M[..., 1, 1] = M[..., 2, 2] = 1.0
    if shape == "prism":
        M[..., 0, 0] = 0.5 * (1 - e3)
        M[..., 0, 2] = -0.5 * (1 + e1)
    elif shape == "pyr":
        M[..., 0, 0] = 0.5 * (1 - e3)
        M[..., 0, 2] = -0.5 * (1 + e1)
        M[..., 1, 1] = 0.5 * (1 - e3)
        M[..., 1, 2] = -0.5 * (1 + e2)
    elif shape == "tet":
        M[..., 0, 0] = 0.25 * (1 - e2) * (1 - e3)
        M[..., 0, 1] = -0.25 * (1 + e1) * (1 - e3)
        M[..., 0, 2] = -0.25 * (1 + e1) * (1 - e2)
        M[..., 1, 1] = 0.5 * (1 - e3)
        M[..., 1, 2] = -0.5 * (1 + e2)
    return M


def points_1d(shape: str, Q: int, pts: str = "gj"):
    """The three 1D rules (nodes, weights) of a shape."""
    return [rule_1d(Q, a, pts) for a in ALPHA[shape]]


def quadrature(shape: str, Q: int, pts: str = "gj"):
    """Tensor points in eta [Q^3, 3] (k fastest), the products of the 1D weights
    [Q^3], and the divisor prod (1 - eta_d)^alpha_d [Q^3] that removes the Jacobi
    weight functions from the rule."""
    r = points_1d(shape, Q, pts)
    z1, z2, z3 = (r[d][0] for d in range(3))
    w1, w2, w3 = (r[d][1] for d in range(3))
    E1, E2, E3 = np.meshgrid(z1, z2, z3, indexing="ij")
    eta = np.stack([E1.ravel(), E2.ravel(), E3.ravel()], axis=1)
    w = np.einsum("i,j,k->ijk", w1, w2, w3).ravel()
    al = ALPHA[shape]
    div = (1 - eta[:, 0]) ** al[0] * (1 - eta[:, 1]) ** al[1] * (1 - eta[:, 2]) ** al[2]
    return eta, w, div


def reference_points(shape: str, Q: int, pts: str = "gj") -> np.ndarray:
    """Quadrature points in reference coordinates xi, [Q^3, 3]."""
    eta, _, _ = quadrature(shape, Q, pts)
    return collapse(shape, eta)


def integrate_reference(shape: str, Q: int, f, pts: str = "gj") -> float:
    """Quadrature of f(xi) over the reference element."""
    eta, w, div = quadrature(shape, Q, pts)
    xi = collapse(shape, eta)
    det = np.linalg.det(dxi_deta(shape, eta))
    return float(np.sum(w * det / div * f(xi)))


# ---------------------------------------------------------------------------
# Modal basis
# ---------------------------------------------------------------------------

def fA(p: int, z):
    z = np.asarray(z, dtype=np.float64)
    if p == 0:
        return 0.5 * (1 - z)
    if p == 1:
        return 0.5 * (1 + z)
    return 0.25 * (1 - z) * (1 + z) * jacobi(p - 2, 1.0, 1.0, z)


def dA(p: int, z):
    z = np.asarray(z, dtype=np.float64)
    if p == 0:
        return np.full_like(z, -0.5)
    if p == 1:
        return np.full_like(z, 0.5)
    J = jacobi(p - 2, 1.0, 1.0, z)
    dJ = jacobi_deriv(p - 2, 1.0, 1.0, z)
    return -0.5 * z * J + 0.25 * (1 - z) * (1 + z) * dJ


def fC(k: int, r: int, z):
    z = np.asarray(z, dtype=np.float64)
    if k == 0:
        return fA(r, z)
    v0 = 0.5 * (1 - z)
    if r == 0:
        return v0 ** k
    return v0 ** k * 0.5 * (1 + z) * jacobi(r - 1, 2.0 * k - 1.0, 1.0, z)


def dC(k: int, r: int, z):
    z = np.asarray(z, dtype=np.float64)
    if k == 0:
        return dA(r, z)
    v0 = 0.5 * (1 - z)
    if r == 0:
        return -0.5 * k * v0 ** (k - 1)
    v1 = 0.5 * (1 + z)
    J = jacobi(r - 1, 2.0 * k - 1.0, 1.0, z)
    dJ = jacobi_deriv(r - 1, 2.0 * k - 1.0, 1.0, z)
    return (-0.5 * k * v0 ** (k - 1) * v1 * J + v0 ** k * 0.5 * J + v0 ** k * v1 * dJ)


def _v1(z):
    return 0.5 * (1 + np.asarray(z, dtype=np.float64))


def modes(shape: str, P: int):
    """Mode index list (p, q, r), lexicographic, r fastest."""
    out = []
    for p in range(P + 1):
        if shape == "tet":
            for q in range(P + 1 - p):
                for r in range(P + 1 - p - q):
                    out.append((p, q, r))
        else:
            for q in range(P + 1):
                if shape == "hex":
                    R = P
                elif shape == "prism":
                    R = P - p
                else:
                    R = P - max(p, q)
                for r in range(R + 1):
                    out.append((p, q, r))
    return out


def num_modes(shape: str, P: int) -> int:
    return len(modes(shape, P))


def _mode_factors(shape: str, p: int, q: int, r: int):
    """The mode as a product of three 1D functions [(f, df) in eta1, eta2, eta3];
    None stands for the constant 1."""
    one = None
    if shape == "hex":
        return [(fA, p), (fA, q), (fA, r)]
    if shape == "prism":
        if p == 0 and r == 1:
            return [one, (fA, q), ("v1",)]
        return [(fA, p), (fA, q), (fC, p, r)]
    if shape == "pyr":
        if (p, q, r) == (0, 0, 1):
            return [one, one, ("v1",)]
        return [(fA, p), (fA, q), (fC, max(p, q), r)]
    if shape == "tet":
        if (p, q, r) == (0, 0, 1):
            return [one, one, ("v1",)]
        if p == 0 and q == 1:
            return [one, ("v1",), (fC, 1, r)]
        return [(fA, p), (fC, p, q), (fC, p + q, r)]
    raise ValueError(shape)


def _eval_factor(fac, z, deriv: bool):
    z = np.asarray(z, dtype=np.float64)
    if fac is None:
        return np.zeros_like(z) if deriv else np.ones_like(z)
    if fac[0] == "v1":
        return np.full_like(z, 0.5) if deriv else _v1(z)
    if fac[0] is fA:
        return dA(fac[1], z) if deriv else fA(fac[1], z)
    return dC(fac[1], fac[2], z) if deriv else fC(fac[1], fac[2], z)


def basis(shape: str, P: int, eta: np.ndarray):
    """phi [n_pts, N_P] and d phi / d eta_d [3, n_pts, N_P] at points eta."""
    eta = np.asarray(eta, dtype=np.float64)
    ml = modes(shape, P)
    npts = eta.shape[0]
    phi = np.empty((npts, len(ml)))
    dphi = np.empty((3, npts, len(ml)))
    for m, (p, q, r) in enumerate(ml):
        facs = _mode_factors(shape, p, q, r)
        vals = [_eval_factor(facs[d], eta[:, d], False) for d in range(3)]
        ders = [_eval_factor(facs[d], eta[:, d], True) for d in range(3)]
        phi[:, m] = vals[0] * vals[1] * vals[2]
        dphi[0, :, m] = ders[0] * vals[1] * vals[2]
        dphi[1, :, m] = vals[0] * ders[1] * vals[2]
        dphi[2, :, m] = vals[0] * vals[1] * ders[2]
    return phi, dphi


VERTEX_MODES = {
    "hex": [(p, q, r) for p in (0, 1) for q in (0, 1) for r in (0, 1)],
    "prism": [(p, q, 0) for p in (0, 1) for q in (0, 1)] + [(0, 0, 1), (0, 1, 1)],
    "pyr": [(p, q, 0) for p in (0, 1) for q in (0, 1)] + [(0, 0, 1)],
    "tet": [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)],
}


# the reference vertex at which each mode of VERTEX_MODES is one (and the other
# vertex modes vanish): A_0 is one at z = -1, A_1 and v1 at z = +1, and a
# collapsed coordinate's vertex sits at xi = -1 in the collapsed directions
VERTEX_XI = {
    "hex": [(2 * p - 1, 2 * q - 1, 2 * r - 1) for p in (0, 1) for q in (0, 1) for r in (0, 1)],
    "prism": [(2 * p - 1, 2 * q - 1, -1) for p in (0, 1) for q in (0, 1)] + [(-1, -1, 1), (-1, 1, 1)],
    "pyr": [(2 * p - 1, 2 * q - 1, -1) for p in (0, 1) for q in (0, 1)] + [(-1, -1, 1)],
    "tet": [(-1, -1, -1), (1, -1, -1), (-1, 1, -1), (-1, -1, 1)],
}


def vertex_modes(shape: str, P: int):
    """Mode indices of the vertex modes and the reference coordinates xi
    [n_vertices, 3] of the vertex where each is one."""
    ml = modes(shape, P)
    return [ml.index(m) for m in VERTEX_MODES[shape]], np.array(VERTEX_XI[shape], dtype=np.float64)


def isoparametric_jacobian(shape: str, P: int, Q: int, X, pts: str = "gj") -> np.ndarray:
    """d x_i/d xi_j at the quadrature points of iso-parametric elements, whose
    map is a polynomial of the solution's degree in the element's own basis
    (Sec. 2.1: J is then polynomial; Sec. 4: curvilinear elements with
    iso-parametric mappings): x_c = sum_m X[e, c, m] phi_m.  The basis
    derivatives give d x/d eta = sum_m X_m (d phi_m/d eta) at the points, and
    d x/d xi = (d x/d eta)(d eta/d xi) with the collapse's d eta/d xi the
    numerical inverse of d xi/d eta.  X: [n_elem, 3, N_P].  Returns
    [n_elem][9][n_pts] with component i*3 + j, the layout Element takes."""
    X = np.asarray(X, dtype=np.float64)
    eta, _, _ = quadrature(shape, Q, pts)
    _, dB = basis(shape, P, eta)                              # [3(d), nq, N_P]
    Jeta = np.einsum("ecm,dqm->eqcd", X, dB)                  # d x_c / d eta_d
    deta_dxi = np.linalg.inv(dxi_deta(shape, eta))            # [nq, 3(d), 3(j)]
    Jxi = np.einsum("eqcd,qdj->eqcj", Jeta, deta_dxi)
    return np.ascontiguousarray(np.transpose(Jxi.reshape(X.shape[0], eta.shape[0], 9), (0, 2, 1)))


def vertex_indicator(shape: str, P: int) -> np.ndarray:
    """Coefficients of the constant function 1: the vertex modes sum to one.
    For the collapsed shapes (1, q, 1) is an edge mode, not a vertex mode."""
    ml = modes(shape, P)
    vm = set(VERTEX_MODES[shape])
    return np.array([1.0 if m in vm else 0.0 for m in ml])


# ---------------------------------------------------------------------------
# Geometry at the quadrature points
# ---------------------------------------------------------------------------

def _jac_xi(jac: np.ndarray, npts: int) -> np.ndarray:
    """[n_elem][9][n_pts] (curved) or [n_elem][9] (affine) -> [n_elem, n_pts, 3, 3]."""
    jac = np.asarray(jac, dtype=np.float64)
    if jac.ndim == 2:
        J = jac.reshape(-1, 3, 3)[:, None, :, :]
        return np.broadcast_to(J, (jac.shape[0], npts, 3, 3))
    return np.transpose(jac, (0, 2, 1)).reshape(jac.shape[0], npts, 3, 3)


def geometry(shape: str, Q: int, jac: np.ndarray, pts: str = "gj"):
    """Per-point weights jw = w |det d x/d eta| / prod (1-eta)^alpha and the
    inverse Jacobian d eta_d / d x_i, computed by numerically inverting
    d x/d eta = (d x/d xi)(d xi/d eta).  Returns jw [n_elem, n_pts] and
    deta_dx [n_elem, n_pts, 3(d), 3(i)]."""
    eta, w, div = quadrature(shape, Q, pts)
    npts = eta.shape[0]
    Jxi = _jac_xi(jac, npts)
    Jeta = np.einsum("epia,pab->epib", Jxi, dxi_deta(shape, eta))
    det = np.linalg.det(Jeta)
    if np.any(~np.isfinite(det)) or np.any(det <= 0):
        raise ValueError("non-positive or non-finite Jacobian")
    jw = w[None, :] * det / div[None, :]
    deta_dx = np.linalg.inv(Jeta)
    return jw, deta_dx


def geometric_factors(shape: str, Q: int, jac: np.ndarray, pts: str = "gj"):
    """jw, the symmetric metric g_de = jw sum_i (d eta_d/d x_i)(d eta_e/d x_i)
    [n_elem, n_pts, 3, 3] and d eta/d x."""
    jw, G = geometry(shape, Q, jac, pts)
    g = jw[..., None, None] * np.einsum("epdi,epei->epde", G, G)
    return jw, g, G


# ---------------------------------------------------------------------------
# Collocation differentiation (Legendre Vandermonde)
# ---------------------------------------------------------------------------

def lagrange_deriv_1d(z: np.ndarray) -> np.ndarray:
    """D[i][l] = h_l'(z_i) for the Lagrange basis through z, as V' V^{-1} with
    V[k][j] = P_j(z_k) (Legendre)."""
    z = np.asarray(z, dtype=np.float64)
    n = z.size
    V = np.stack([jacobi(j, 0.0, 0.0, z) for j in range(n)], axis=1)
    Vd = np.stack([jacobi_deriv(j, 0.0, 0.0, z) for j in range(n)], axis=1)
    return np.linalg.solve(V.T, Vd.T).T


def deriv_matrices(shape: str, Q: int, pts: str = "gj"):
    """Collocation derivatives in eta_1, eta_2, eta_3 on the tensor points,
    three [Q^3, Q^3] matrices."""
    r = points_1d(shape, Q, pts)
    I = np.eye(Q)
    D = [lagrange_deriv_1d(r[d][0]) for d in range(3)]
    return [np.kron(np.kron(D[0], I), I), np.kron(np.kron(I, D[1]), I), np.kron(np.kron(I, I), D[2])]


# ---------------------------------------------------------------------------
# Elemental matrices by explicit quadrature
# ---------------------------------------------------------------------------

class Element:
    """Dense operators of a batch of elements of one shape.

    jac: d x_i/d xi_j at the oracle's quadrature points of point set pts,
    [n_elem][9][Q^3], or constant per element [n_elem][9]."""

    def __init__(self, shape: str, P: int, Q: int, jac: np.ndarray, pts: str = "gj"):
        self.shape, self.P, self.Q, self.pts = shape, P, Q, pts
        eta, _, _ = quadrature(shape, Q, pts)
        self.B, self.dB = basis(shape, P, eta)                # [nq,np], [3,nq,np]
        self.jw, self.G = geometry(shape, Q, jac, pts)        # [ne,nq], [ne,nq,d,i]
        # d phi / d x_i at the points: sum_d (d eta_d/d x_i) d phi/d eta_d
        self.dBx = np.einsum("eqdi,dqm->eiqm", self.G, self.dB)

    @property
    def n_elem(self):
        return self.jw.shape[0]

    def mass(self) -> np.ndarray:
        """M = B^T W B, [n_elem, N_P, N_P]."""
        return np.matmul(self.B.T[None, :, :], self.jw[:, :, None] * self.B[None, :, :])

    def laplacian(self) -> np.ndarray:
        """L[m,n] = sum_q jw sum_i (d phi_m/d x_i)(d phi_n/d x_i)."""
        L = np.zeros((self.n_elem, self.B.shape[1], self.B.shape[1]))
        for i in range(3):
            Bi = self.dBx[:, i]                                  # [ne, nq, np]
            L += np.matmul(np.transpose(Bi, (0, 2, 1)), self.jw[:, :, None] * Bi)
        return L

    def helmholtz(self, lam: float) -> np.ndarray:
        return lam * self.mass() + self.laplacian()

    def advection(self, vel) -> np.ndarray:
        """C[m,n] = sum_q jw_q phi_m(eta_q) sum_i b_i(q) (d phi_n/d x_i)(eta_q):
        the advection term b . grad u tested with the basis, by explicit
        quadrature (the collocated reading of Sec. 2.2.1 extends the Helmholtz
        operator to advection-diffusion-reaction).  vel: [3, n_elem, N_Q]."""
        vel = np.asarray(vel, dtype=np.float64)
        bgrad = np.einsum("ieq,eiqn->eqn", vel, self.dBx)          # b . grad phi_n at the points
        return np.matmul(self.B.T[None, :, :], self.jw[:, :, None] * bgrad)

    def adr(self, lam: float, vel) -> np.ndarray:
        """lambda M + L + C (advection-diffusion-reaction)."""
        return self.helmholtz(lam) + self.advection(vel)

    # --- actions as dense matrix-vector products --------------------------
    def bwd_trans(self, x):
        """u_q = sum_m phi_m(eta_q) x_m, [n_elem, N_Q]."""
        return np.einsum("qm,em->eq", self.B, x)

    def iproduct(self, f):
        """y_m = sum_q jw_q phi_m(eta_q) f_q."""
        return np.einsum("qm,eq->em", self.B, self.jw * f)

    def iproduct_deriv(self, f3):
        """y_m = sum_i sum_q jw_q (d phi_m/d x_i)(eta_q) f_i,q ; f3 [3, n_elem, N_Q]."""
        return np.einsum("eiqm,eq,ieq->em", self.dBx, self.jw, f3)

    def phys_deriv(self, u):
        """d u/d x_i at the points of the Lagrange interpolant of u, [3, n_elem, N_Q]."""
        D = deriv_matrices(self.shape, self.Q, self.pts)
        du = np.stack([u @ Dd.T for Dd in D], axis=0)       # [3(d), ne, nq]
        return np.einsum("eqdi,deq->ieq", self.G, du)

    def mass_action(self, x):
        return np.einsum("emn,en->em", self.mass(), x)

    def laplacian_action(self, x):
        return np.einsum("emn,en->em", self.laplacian(), x)

    def helmholtz_action(self, x, lam: float):
        return np.einsum("emn,en->em", self.helmholtz(lam), x)


def apply_op(op: str, shape: str, P: int, Q: int, jac, x, lam: float = 1.0, chunk: int = 512, pts: str = "gj",
             vel=None):
    """One operator over a batch, processed in chunks of elements.
    op in {bwd, iprod, physderiv, iprod_deriv, mass, laplacian, helmholtz, adr};
    adr takes the velocity vel [3, n_elem, N_Q] at the points."""
    x = np.asarray(x, dtype=np.float64)
    jac = np.asarray(jac, dtype=np.float64)
    ne = jac.shape[0]
    outs = []
    for e0 in range(0, ne, chunk):
        e1 = min(ne, e0 + chunk)
        el = Element(shape, P, Q, jac[e0:e1], pts)
        if op == "bwd":
            outs.append(el.bwd_trans(x[e0:e1]))
        elif op == "iprod":
            outs.append(el.iproduct(x[e0:e1]))
        elif op == "physderiv":
            outs.append(el.phys_deriv(x[e0:e1]))
        elif op == "iprod_deriv":
            outs.append(el.iproduct_deriv(x[:, e0:e1]))
        elif op == "mass":
            outs.append(el.mass_action(x[e0:e1]))
        elif op == "laplacian":
            outs.append(el.laplacian_action(x[e0:e1]))
        elif op == "helmholtz":
            outs.append(el.helmholtz_action(x[e0:e1], lam))
        elif op == "adr":
            outs.append(np.einsum("emn,en->em", el.adr(lam, np.asarray(vel)[:, e0:e1]), x[e0:e1]))
        else:
            raise ValueError(op)
    axis = 1 if op == "physderiv" else 0
    return np.concatenate(outs, axis=axis)


def helmholtz_solve(shape: str, P: int, Q: int, jac, b, lam: float = 1.0, chunk: int = 512, pts: str = "gj"):
    """x with H_e x_e = b_e for every element, by dense Cholesky (H_e is SPD for
    lambda > 0)."""
    b = np.asarray(b, dtype=np.float64)
    jac = np.asarray(jac, dtype=np.float64)
    out = []
    for e0 in range(0, jac.shape[0], chunk):
        e1 = min(jac.shape[0], e0 + chunk)
        H = Element(shape, P, Q, jac[e0:e1], pts).helmholtz(lam)
        Lc = np.linalg.cholesky(H)
        y = np.linalg.solve(Lc, b[e0:e1][..., None])
        out.append(np.linalg.solve(np.transpose(Lc, (0, 2, 1)), y)[..., 0])
    return np.concatenate(out, axis=0)
