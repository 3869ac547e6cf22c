"""CPU study behind the precision choice of the mixed-precision solve: can a
reduced-precision elemental Helmholtz operator serve as the inner operator of
iterative refinement on the P = 6 curved mesh?

Iterative refinement with an inner operator H~ in place of H, even with exact
inner solves, updates the error by e <- (I - H~^-1 H) e, so it converges only
if the spectral radius rho(I - H~^-1 H) < 1.  H~ is H with every entry rounded
to the contraction precision: FP32 (what the library builds) or BF16 (8-bit
significand).  This is a lower bound on the error of a real reduced-precision
contraction, which also rounds its inputs and intermediate stages.  The
operators are the oracle's dense H = lambda M + L of elements sampled from the
32^3-cell quadrant mesh at P = 6.
"""
import numpy as np
import pytest

from oracle import shp_oracle as O
from paper_2604_04644_amd import workloads as W


def _bf16(a):
    """Round float32 values to the nearest bfloat16, ties to even."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)


def test_bf16_rounding_helper():
    """bfloat16 keeps 7 fraction bits: spacing 2^-7 on [1, 2) and 2^-6 on [2, 4)."""
    x = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(3.0 + 2.0 ** -7), -(3.0 + 2.0 ** -7 + 2.0 ** -9)],
                 dtype=np.float32)
    # 1 + 2^-8, 1 + 3 2^-8 and 3 + 2^-7 are ties and go to the even neighbour
    # (1, 1 + 2^-6, 3); 3 + 2^-7 + 2^-9 is past its tie and rounds up
    assert _bf16(x).tolist() == [1.0, 1.0, 1.0 + 2.0 ** -6, -3.0, -(3.0 + 2.0 ** -6)]


@pytest.mark.parametrize("shape", O.SHAPES)
def test_refinement_contraction_fp32_vs_bf16(shape):
    P, Q = 6, 8
    mesh = W.quadrant_mesh(32)
    idx = np.random.default_rng(0).choice(len(mesh[shape]), 4, replace=False)
    maps = mesh[shape].take(idx)
    H = O.Element(shape, P, Q, W.jacobian(maps, O.reference_points(shape, Q), curved=True)).helmholtz(1.0)
    rho = {"fp32": [], "bf16": []}
    for He in H:
        for prec in rho:
            Ht = (He.astype(np.float32) if prec == "fp32" else _bf16(He)).astype(np.float64)
            G = np.eye(len(He)) - np.linalg.solve(Ht, He)
            rho[prec].append(float(np.max(np.abs(np.linalg.eigvals(G)))))
    print(f"{shape}: rho fp32 max {max(rho['fp32']):.2e}, bf16 min {min(rho['bf16']):.2e} "
          f"max {max(rho['bf16']):.2e}")
    assert max(rho["fp32"]) < 1e-2          # FP32 contracts the error by >= 100x per step
    assert max(rho["bf16"]) > 1.0           # BF16 diverges on some element of every shape


def _split_bf16(a, parts):
    """a as a sum of `parts` bfloat16 values: each part the bfloat16 rounding
    of what the previous parts leave (the split behind bf16x2 / bf16x3)."""
    rest = np.asarray(a, dtype=np.float64)
    out = np.zeros_like(rest)
    for _ in range(parts):
        p = _bf16(rest.astype(np.float32)).astype(np.float64)
        out += p
        rest = rest - p
    return out


def test_bf16_split_helper():
    """Each extra part adds about 8 bits: the error of the k-part split of a
    random value is below 2^(-8k) of it."""
    x = np.random.default_rng(5).uniform(0.5, 2.0, 1000)
    for k in (1, 2, 3):
        assert np.max(np.abs(_split_bf16(x, k) - x) / x) <= 2.0 ** (-8 * k)


@pytest.mark.parametrize("shape", O.SHAPES)
def test_split_bf16_and_bf16_preconditioner(shape):
    """The split-BF16 operators and BF16 in a preconditioner role, on the same
    P = 6 elements.  Refinement contraction rho(I - H~^-1 H) for H~ the
    two- and three-part BF16 splits of H; and, for H~ = H rounded to BF16 used
    only as a preconditioner (an exact solve with it inside CG on H), whether
    it stays positive definite and the condition number of H~^-1 H against
    that of the Jacobi-scaled H (CG iterations grow as its square root)."""
    P, Q = 6, 8
    mesh = W.quadrant_mesh(32)
    idx = np.random.default_rng(0).choice(len(mesh[shape]), 4, replace=False)
    maps = mesh[shape].take(idx)
    H = O.Element(shape, P, Q, W.jacobian(maps, O.reference_points(shape, Q), curved=True)).helmholtz(1.0)
    rho = {2: [], 3: []}
    spd, kap_bf16, kap_jac = [], [], []
    for He in H:
        for k in rho:
            G = np.eye(len(He)) - np.linalg.solve(_split_bf16(He, k), He)
            rho[k].append(float(np.max(np.abs(np.linalg.eigvals(G)))))
        Hb = _split_bf16(He, 1)
        Hb = 0.5 * (Hb + Hb.T)
        spd.append(bool(np.linalg.eigvalsh(Hb).min() > 0))
        if spd[-1]:
            ev = np.linalg.eigvals(np.linalg.solve(Hb, He)).real
            kap_bf16.append(float(ev.max() / ev.min()) if ev.min() > 0 else np.inf)
        d = 1.0 / np.sqrt(np.diag(He))
        ej = np.linalg.eigvalsh(d[:, None] * He * d[None, :])
        kap_jac.append(float(ej.max() / ej.min()))
    print(f"{shape}: rho bf16x2 max {max(rho[2]):.2e}, bf16x3 max {max(rho[3]):.2e}; BF16 matrix SPD on "
          f"{sum(spd)}/{len(spd)} elements, cond(H_bf16^-1 H) {kap_bf16}, cond Jacobi {min(kap_jac):.2e}.."
          f"{max(kap_jac):.2e}")
    assert max(rho[3]) < 1e-2                 # three parts: FP32-like contraction
    assert max(rho[3]) < max(rho[2])          # each part helps
    assert not all(spd)                       # rounded to BF16, H loses definiteness
