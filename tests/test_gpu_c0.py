"""C0-assembled Helmholtz problem on a structured hexahedral grid (curved by
the mesh map, homogeneous Dirichlet data) through the C ABI, against the
oracle's sparse assembly of its dense elemental matrices.

Bars: the assembled action to the FP64 operator bar (1e-12 of the max-norm);
the solve, to a relative residual of 1e-13, within 1e-9 (max-norm, relative) of
the oracle's sparse direct solution; and the discrete solution at the
quadrature points within the spectral-convergence error of the analytic one.
On the 4^3 grid at P = 4, cond(A^T H A) = 6.9e5 (3.2e3 after Jacobi scaling),
so a residual r bounds the forward error by 6.9e5 r; at r = 7.5e-13 the
measured errors were 3.0e-10 (FP64 inner) and 3.0e-9 (FP32 inner), hence the
tolerance of 1e-13.  The oracle's own forward error is about 3.5e-11.
"""
import numpy as np
import pytest

from oracle import shp_assembly as A
from oracle import shp_assembly_tet as AT
from oracle import shp_oracle as O
from paper_2604_04644_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
LAM = 1.0


@pytest.fixture(scope="module")
def shp():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2604_04644_amd import shp as S
    S.lib()
    return S


def say(msg):
    print(msg, flush=True)


def grid_plan(shp, n, P):
    maps = W.affine_hex_grid(n)
    plan = shp.Plan([("hex", P, len(maps), "curved")])
    plan.set_geometry(0, W.jacobian_torch(maps, shp.quadrature("hex", P + 2)[0], True, torch.device("cuda")))
    return maps, plan, plan.c0_hex_grid(n, n, n)


def oracle_system(maps, n, P):
    xi = O.reference_points("hex", P + 2)
    jac = W.jacobian(maps, xi, curved=True)
    l2g, ng = A.hex_grid_map(n, n, n, P)
    H = A.assemble(A.element_matrices(P, jac, "helmholtz", LAM), l2g, ng)
    f = (LAM + 3 * np.pi ** 2) * W.manufactured_u(W.coords(maps, xi, curved=True))
    b = A.assemble_vector(O.apply_op("iprod", "hex", P, P + 2, jac, f), l2g, ng)
    return H, b


@pytest.mark.parametrize("n,P", [(3, 1), (3, 3), (2, 5)])
def test_c0_action_vs_oracle(shp, n, P):
    say(f"[c0] assembled action n={n} P={P}")
    maps, plan, c0 = grid_plan(shp, n, P)
    H, _ = oracle_system(maps, n, P)
    assert H.shape[0] == c0["n_global"]
    x = W.coeffs(1, c0["n_global"], 900 + P)[0]
    y = plan.c0_apply(c0, torch.from_numpy(x).cuda(), lam=LAM).cpu().numpy()
    ref = H @ x
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    if n == 3 and P == 1:                # host or mis-sized vectors never reach a kernel
        with pytest.raises(ValueError):
            plan.c0_apply(c0, torch.from_numpy(x))
        with pytest.raises(ValueError):
            plan.c0_apply(c0, torch.from_numpy(x[:-1]).cuda())
        with pytest.raises(ValueError):
            plan.c0_assemble(c0, torch.zeros(3, dtype=torch.float64, device="cuda"))


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_c0_solve_vs_oracle(shp, inner):
    n, P = 4, 4
    say(f"[c0] assembled solve n={n} P={P} inner={inner}")
    maps, plan, c0 = grid_plan(shp, n, P)
    H, b = oracle_system(maps, n, P)
    xo = A.solve(H, b)
    x, st = plan.c0_solve(c0, torch.from_numpy(b).cuda(), lam=LAM, inner=inner, tol=1e-13)
    say(f"    {st}")
    assert st["converged"]
    e = np.abs(x.cpu().numpy() - xo).max() / np.abs(xo).max()
    say(f"    error vs oracle {e:.2e}")
    assert e <= 1e-9


def test_c0_converges_to_manufactured(shp):
    """GPU solutions for P = 2, 4, 6 on the 4^3 curved grid, evaluated at the
    quadrature points, approach u = sin(pi x) sin(pi y) sin(pi z) spectrally."""
    n = 4
    errs = []
    for P in (2, 4, 6):
        say(f"[c0] convergence P={P}")
        maps, plan, c0 = grid_plan(shp, n, P)
        xi = shp.quadrature("hex", P + 2)[0]
        f = W.manufactured_u_torch(maps, xi, torch.device("cuda")) * (LAM + 3 * np.pi ** 2)
        b = plan.c0_assemble(c0, plan.apply(-1, "iprod", f.reshape(-1).contiguous()))
        x, st = plan.c0_solve(c0, b, lam=LAM, inner="fp32", tol=1e-11)
        assert st["converged"]
        l2g = c0["l2g"]
        xl = torch.where(l2g >= 0, x[l2g.clamp(min=0)], torch.zeros((), dtype=x.dtype, device=x.device))
        u = plan.apply(-1, "bwd", xl.contiguous()).cpu().numpy()
        e = float(np.abs(u - W.manufactured_u_torch(maps, xi, "cpu").numpy().ravel()).max())
        say(f"    P={P}: max error vs u {e:.2e}, {st['inner_iters']} iterations")
        errs.append(e)
    assert errs[0] > 30 * errs[1] > 900 * errs[2], errs


# ---- conforming tetrahedral mesh: orientation-aware map with sign changes ----

def tet_plan(shp, n, P):
    maps, V = W.conforming_tet_mesh(n)
    plan = shp.Plan([("tet", P, len(maps), "curved")])
    plan.set_geometry(0, W.jacobian_torch(maps, shp.quadrature("tet", P + 2)[0], True, torch.device("cuda")))
    return maps, V, plan, plan.c0_tet_mesh(V)


def tet_oracle_system(maps, V, P):
    xi = O.reference_points("tet", P + 2)
    jac = W.jacobian(maps, xi, curved=True)
    l2g, ng, _, _ = AT.tet_map(V, P)
    H = AT.assemble(AT.element_matrices(P, jac, "helmholtz", LAM), l2g, ng)
    f = (LAM + 3 * np.pi ** 2) * W.manufactured_u(W.coords(maps, xi, curved=True))
    b = AT.assemble_vector(O.apply_op("iprod", "tet", P, P + 2, jac, f), l2g, ng)
    return H, b, l2g


@pytest.mark.parametrize("n,P", [(2, 1), (2, 3), (2, 5), (3, 4)])
def test_c0_tet_action_vs_oracle(shp, n, P):
    """Assembled action on the curved conforming tet mesh (the map carries
    sign changes from P = 3 on), the gather of a global vector into signed
    local copies, and the signed assembly of a local vector."""
    say(f"[c0 tet] assembled action n={n} P={P}")
    maps, V, plan, c0 = tet_plan(shp, n, P)
    H, _, l2g = tet_oracle_system(maps, V, P)
    assert H.shape[0] == c0["n_global"]
    x = W.coeffs(1, c0["n_global"], 950 + P)[0]
    xt = torch.from_numpy(x).cuda()
    y = plan.c0_apply(c0, xt, lam=LAM).cpu().numpy()
    ref = H @ x
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    xl = plan.c0_gather(c0, xt).cpu().numpy()
    assert np.array_equal(xl, AT.scatter(x, l2g).ravel())
    v = W.coeffs(len(V), O.num_modes("tet", P), 960 + P)
    vg = plan.c0_assemble(c0, torch.from_numpy(v.ravel().copy()).cuda()).cpu().numpy()
    vref = AT.assemble_vector(v, l2g, c0["n_global"])
    assert np.abs(vg - vref).max() <= 1e-14 * max(np.abs(vref).max(), 1.0)


@pytest.mark.parametrize("inner", ["fp64", "fp32"])
def test_c0_tet_solve_vs_oracle(shp, inner):
    n, P = 3, 4
    say(f"[c0 tet] assembled solve n={n} P={P} inner={inner}")
    maps, V, plan, c0 = tet_plan(shp, n, P)
    H, b, _ = tet_oracle_system(maps, V, P)
    xo = AT.solve(H, b)
    x, st = plan.c0_solve(c0, torch.from_numpy(b).cuda(), lam=LAM, inner=inner, tol=1e-13)
    say(f"    {st}")
    assert st["converged"]
    e = np.abs(x.cpu().numpy() - xo).max() / np.abs(xo).max()
    say(f"    error vs oracle {e:.2e}")
    assert e <= 1e-9
