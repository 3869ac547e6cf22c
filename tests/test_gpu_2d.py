"""GPU parity of the 2D operators (quadrilaterals and triangles) against the
2D FP64 oracle, through the C ABI.  Bar: 1e-12 relative in the max norm."""
import numpy as np
import pytest

from oracle import shp_oracle2d as O2
from paper_2604_04644_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12
OPS = ["bwd", "iprod", "physderiv", "iprod_deriv", "mass", "laplacian", "helmholtz"]


@pytest.fixture(scope="module")
def shp():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2604_04644_amd import shp as S
    S.lib()
    return S


def say(msg):
    print(msg, flush=True)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def op_input(op, ne, NP, NQ, seed):
    if op in ("iprod", "physderiv"):
        return W.point_values(ne, NQ, seed)
    if op == "iprod_deriv":
        return W.point_values(ne, NQ, seed, ncomp=2)
    return W.coeffs(ne, NP, seed)


def plan2d(shp, mesh, P, geom="curved", pts="gj"):
    plan = shp.Plan([(s, P, len(mesh[s]), geom, pts) for s in O2.SHAPES2])
    jo = {}
    for b, s in enumerate(O2.SHAPES2):
        if geom == "curved":
            xi, _ = shp.quadrature(s, P + 2, pts)
            plan.set_geometry(b, torch.from_numpy(W.jacobian2d(mesh[s], xi, True)).cuda())
            jo[s] = W.jacobian2d(mesh[s], O2.reference_points(s, P + 2, pts), True)
        else:
            plan.set_geometry(b, torch.from_numpy(W.affine_jacobian2d(mesh[s])).cuda())
            jo[s] = W.affine_jacobian2d(mesh[s])
    return plan, jo


@pytest.mark.parametrize("P", list(range(1, 11)))
def test_2d_whole_mesh_vs_oracle(shp, P):
    """Every operator on a curved quad/triangle mesh (8^2 cells: 32
    quadrilaterals, 64 triangles) in one launch: equal to the per-block
    launches bit for bit and to the oracle on every element."""
    say(f"[2d] whole mesh P={P}")
    mesh = W.quad_tri_mesh(8)
    plan, jo = plan2d(shp, mesh, P)
    nc, npnt = plan.totals()
    for k, op in enumerate(OPS):
        if op in ("iprod", "physderiv"):
            x = W.point_values(1, npnt, 800 + k)[0]
        elif op == "iprod_deriv":
            x = W.point_values(1, npnt, 800 + k, ncomp=2).reshape(2, npnt)
        else:
            x = W.coeffs(1, nc, 800 + k)[0]
        y = plan.apply(-1, op, torch.from_numpy(np.ascontiguousarray(x)).cuda(), lam=1.4).cpu().numpy()
        worst = 0.0
        for b, s in enumerate(O2.SHAPES2):
            co, po = plan.offsets(b)
            ne, NP, NQ = len(mesh[s]), plan.n_modes[b], plan.n_points[b]
            if op in ("iprod", "physderiv"):
                xb = x[po:po + ne * NQ].reshape(ne, NQ)
            elif op == "iprod_deriv":
                xb = x[:, po:po + ne * NQ].reshape(2, ne, NQ)
            else:
                xb = x[co:co + ne * NP].reshape(ne, NP)
            if op == "bwd":
                ym = y[po:po + ne * NQ].reshape(ne, NQ)
            elif op == "physderiv":
                ym = y.reshape(2, -1)[:, po:po + ne * NQ].reshape(2, ne, NQ)
            else:
                ym = y[co:co + ne * NP].reshape(ne, NP)
            yb = plan.apply(b, op, torch.from_numpy(np.ascontiguousarray(xb)).cuda(), lam=1.4).cpu().numpy()
            assert np.array_equal(ym, yb.reshape(ym.shape)), (op, s)
            ref = O2.apply_op(op, s, P, P + 2, jo[s], xb, lam=1.4)
            e = rel(ym.reshape(ref.shape), ref)
            worst = max(worst, e)
            assert e <= TOL, (op, s, e)
        say(f"    {op:12s} worst rel={worst:.2e}")


@pytest.mark.parametrize("geom,pts", [("affine", "gj"), ("curved", "radau")])
def test_2d_affine_and_radau(shp, geom, pts):
    """Affine elements (constant d x/d xi) and Gauss-Radau points in the
    triangle's collapsed direction, every operator, on ragged blocks."""
    say(f"[2d] {geom} {pts}")
    P = 5
    mesh = W.quad_tri_mesh(6)
    mesh = {s: mesh[s].take(np.arange(len(mesh[s]) - 3)) for s in O2.SHAPES2}
    plan, jo = plan2d(shp, mesh, P, geom, pts)
    for b, s in enumerate(O2.SHAPES2):
        ne, NP, NQ = len(mesh[s]), plan.n_modes[b], plan.n_points[b]
        for k, op in enumerate(OPS):
            x = op_input(op, ne, NP, NQ, 820 + k)
            y = plan.apply(b, op, torch.from_numpy(np.ascontiguousarray(x)).cuda(), lam=0.6).cpu().numpy()
            ref = O2.apply_op(op, s, P, P + 2, jo[s], x, lam=0.6, pts=pts)
            assert rel(y.reshape(ref.shape), ref) <= TOL, (s, op)


def test_2d_limits(shp):
    """Operations the 2D blocks do not have report UNSUPPORTED; a mirrored
    triangle (negative determinant) is reported as bad geometry."""
    say("[2d] limits")
    mesh = W.quad_tri_mesh(4)
    plan, _ = plan2d(shp, mesh, 3)
    nc, _ = plan.totals()
    x = torch.zeros(nc, dtype=torch.float64, device="cuda")
    with pytest.raises(shp.ShpError) as ei:
        plan.apply(-1, "helmholtz", x, strategy="sumfac")
    assert ei.value.code == -2
    with pytest.raises(shp.ShpError) as ei:
        plan.tune(-1, "helmholtz", x)
    assert ei.value.code == -2
    with pytest.raises(shp.ShpError) as ei:
        plan.helmholtz_diag(1.0)
    assert ei.value.code == -2
    jac = W.jacobian2d(mesh["tri"], shp.quadrature("tri", 5)[0], True)
    jac[3, 0:2, :] *= -1.0
    bad = shp.Plan([("tri", 3, len(mesh["tri"]), "curved")])
    with pytest.raises(shp.ShpError) as ei:
        bad.set_geometry(0, torch.from_numpy(jac).cuda())
    assert ei.value.code == -3
