"""Writes the exact element matrices used as pins of the oracle.

For each reference shape and P in {1, 2} it forms, by exact symbolic
integration over [-1,1]^3 in the collapsed coordinates, the mass and Laplacian
matrices of the affine element x = A xi with the fixed rational matrix A below
(Sec. 2.1, H^e with the chain rule; Sec. 2.3, Duffy collapse).  The basis is the
modified C0 modal basis written out symbolically; derivatives, the collapse
Jacobian and its inverse are taken by sympy, and integrals are exact, so the
result is independent of any quadrature rule.  Uses sympy only.

Run:  python tests/golden/make_exact_matrices.py
"""
import os

import numpy as np
import sympy as sp

HERE = os.path.dirname(os.path.abspath(__file__))


def modes(shape, P):
    out = []
    for p in range(P + 1):
        if shape == "tet":
            for q in range(P + 1 - p):
                for r in range(P + 1 - p - q):
                    out.append((p, q, r))
        else:
            for q in range(P + 1):
                R = P if shape == "hex" else (P - p if shape == "prism" else P - max(p, q))
                for r in range(R + 1):
                    out.append((p, q, r))
    return out


def _sym_basis(shape, P, e1, e2, e3):
    """The modal basis as sympy expressions of eta (same definitions, symbolic)."""
    z = sp.Symbol("z")

    def A(p, x):
        if p == 0:
            return (1 - x) / 2
        if p == 1:
            return (1 + x) / 2
        return (1 - x) / 2 * (1 + x) / 2 * sp.jacobi(p - 2, 1, 1, x)

    def C(k, r, x):
        if k == 0:
            return A(r, x)
        if r == 0:
            return ((1 - x) / 2) ** k
        return ((1 - x) / 2) ** k * (1 + x) / 2 * sp.jacobi(r - 1, 2 * k - 1, 1, x)

    v1 = lambda x: (1 + x) / 2
    out = []
    for (p, q, r) in modes(shape, P):
        if shape == "hex":
            f = A(p, e1) * A(q, e2) * A(r, e3)
        elif shape == "prism":
            f = A(q, e2) * v1(e3) if (p == 0 and r == 1) else A(p, e1) * A(q, e2) * C(p, r, e3)
        elif shape == "pyr":
            f = v1(e3) if (p, q, r) == (0, 0, 1) else A(p, e1) * A(q, e2) * C(max(p, q), r, e3)
        else:
            if (p, q, r) == (0, 0, 1):
                f = v1(e3)
            elif p == 0 and q == 1:
                f = v1(e2) * C(1, r, e3)
            else:
                f = A(p, e1) * C(p, q, e2) * C(p + q, r, e3)
        out.append(sp.expand(f))
    return out


def _sym_collapse(shape, e1, e2, e3):
    if shape == "hex":
        return [e1, e2, e3]
    if shape == "prism":
        return [(1 + e1) * (1 - e3) / 2 - 1, e2, e3]
    if shape == "pyr":
        return [(1 + e1) * (1 - e3) / 2 - 1, (1 + e2) * (1 - e3) / 2 - 1, e3]
    return [(1 + e1) * (1 - e2) * (1 - e3) / 4 - 1, (1 + e2) * (1 - e3) / 2 - 1, e3]


def _exact_M_L(shape, P, Amat):
    """Exact M and L of the affine element x = Amat xi (symbolic integration over
    [-1,1]^3 in eta with the symbolic Jacobian of the collapse)."""
    e1, e2, e3 = sp.symbols("e1 e2 e3")
    phi = _sym_basis(shape, P, e1, e2, e3)
    xi = _sym_collapse(shape, e1, e2, e3)
    Jc = sp.Matrix(3, 3, lambda a, b: sp.diff(xi[a], [e1, e2, e3][b]))
    A = sp.Matrix(Amat)
    det = sp.factor(Jc.det()) * A.det()
    G = sp.simplify(Jc.inv()) * A.inv()            # d eta / d x
    grads = [G.T * sp.Matrix([sp.diff(f, v) for v in (e1, e2, e3)]) for f in phi]
    n = len(phi)
    M = np.zeros((n, n))
    L = np.zeros((n, n))

    def integ(expr):
        expr = sp.cancel(sp.together(expr))
        num, den = sp.fraction(expr)
        assert den.free_symbols == set(), den
        poly = sp.Poly(sp.expand(num), e1, e2, e3)
        tot = sp.Rational(0)
        for (a, b, c), co in poly.terms():
            m = 1
            for k in (a, b, c):
                m *= sp.Rational(2, k + 1) if k % 2 == 0 else 0
            tot += co * m
        return tot / den

    for i in range(n):
        for j in range(i, n):
            M[i, j] = M[j, i] = float(integ(phi[i] * phi[j] * det))
            L[i, j] = L[j, i] = float(integ((grads[i].T * grads[j])[0, 0] * det))
    return M, L


_AFF = [[sp.Rational(3, 2), sp.Rational(1, 5), 0],
        [sp.Rational(-1, 4), 1, sp.Rational(1, 3)],
        [sp.Rational(1, 7), 0, sp.Rational(4, 5)]]


def main():
    for shape in ("hex", "prism", "pyr", "tet"):
        for P in (1, 2):
            M, L = _exact_M_L(shape, P, _AFF)
            np.savetxt(os.path.join(HERE, f"exact_M_{shape}_P{P}.txt"), M, fmt="%.17e",
                       header=f"exact mass matrix, {shape}, P={P}, x = A xi, A = {_AFF}")
            np.savetxt(os.path.join(HERE, f"exact_L_{shape}_P{P}.txt"), L, fmt="%.17e",
                       header=f"exact Laplacian matrix, {shape}, P={P}, x = A xi, A = {_AFF}")
            print(shape, P, M.shape, flush=True)


if __name__ == "__main__":
    main()
