"""GPU parity of the whole-mesh advection-diffusion-reaction action (the
collocated Helmholtz action plus b . grad u tested with the basis) through the
C ABI, against the oracle's lambda M + L + C formed by explicit quadrature.
Bar: max-norm error relative to the oracle's max-norm <= 1e-12 in FP64.  The
velocity is U[-1,1] at every point (seeded)."""
import numpy as np
import pytest

from oracle import shp_oracle as O
from paper_2604_04644_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-12


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


def _plan(shp, ncell, P):
    mesh = W.quadrant_mesh(ncell)
    plan = shp.Plan([(s, P, len(mesh[s]), "curved") for s in O.SHAPES])
    for b, s in enumerate(O.SHAPES):
        xi, _ = shp.quadrature(s, P + 2)
        plan.set_geometry(b, torch.from_numpy(np.ascontiguousarray(W.jacobian(mesh[s], xi, curved=True))).cuda())
    return mesh, plan


@pytest.mark.parametrize("P", [1, 3, 4, 6])
def test_adr_whole_mesh_vs_oracle(shp, P):
    say(f"[adr] whole mesh P={P}")
    mesh, plan = _plan(shp, 4, P)
    nc, npnt = plan.totals()
    x = W.coeffs(1, nc, 800 + P)[0]
    vel = W.point_values(1, npnt, 810 + P, ncomp=3).reshape(3, npnt)
    adv = plan.advection_factors(torch.from_numpy(np.ascontiguousarray(vel)).cuda())
    y = plan.apply_adr(torch.from_numpy(x).cuda(), adv, lam=1.3).cpu().numpy()
    for b, s in enumerate(O.SHAPES):
        co, po = plan.offsets(b)
        ne, NP, NQ = len(mesh[s]), plan.n_modes[b], plan.n_points[b]
        jo = W.jacobian(mesh[s], O.reference_points(s, P + 2), curved=True)
        ref = O.apply_op("adr", s, P, P + 2, jo, x[co:co + ne * NP].reshape(ne, NP), lam=1.3,
                         vel=vel[:, po:po + ne * NQ].reshape(3, ne, NQ))
        e = rel(y[co:co + ne * NP].reshape(ne, NP), ref)
        say(f"    {s:6s} rel={e:.2e}")
        assert e <= TOL, (s, P, e)


def test_adr_zero_velocity_is_helmholtz(shp):
    say("[adr] zero velocity equals the Helmholtz action")
    _, plan = _plan(shp, 2, 4)
    nc, npnt = plan.totals()
    x = torch.from_numpy(W.coeffs(1, nc, 820)[0]).cuda()
    adv = plan.advection_factors(torch.zeros(3 * npnt, dtype=torch.float64, device="cuda"))
    assert float(adv.abs().max()) == 0.0
    y = plan.apply_adr(x, adv, lam=0.9).cpu().numpy()
    yh = plan.apply(-1, "helmholtz", x, lam=0.9).cpu().numpy()
    assert rel(y, yh) <= 1e-15
    with pytest.raises(ValueError):      # host memory never reaches a kernel
        plan.apply_adr(x, adv.cpu())
    with pytest.raises(ValueError):
        plan.apply_adr(x, adv, out=torch.empty(nc, dtype=torch.float64))


def test_adr_rejects_mixed_orders(shp):
    say("[adr] mixed P rejected")
    plan = shp.Plan([("hex", 2, 3, "curved"), ("tet", 3, 3, "curved")])
    for b, (s, P) in enumerate((("hex", 2), ("tet", 3))):
        xi, _ = shp.quadrature(s, P + 2)
        plan.set_geometry(b, torch.from_numpy(W.jacobian(W.shape_batch(s, 3), xi, curved=True)).cuda())
    nc, npnt = plan.totals()
    adv = torch.zeros(3 * npnt, dtype=torch.float64, device="cuda")
    with pytest.raises(shp.ShpError) as ei:
        plan.apply_adr(torch.zeros(nc, dtype=torch.float64, device="cuda"), adv)
    assert ei.value.code == -2


def test_adr_affine_and_radau_blocks(shp):
    """Affine blocks (per-point factors from a constant Jacobian) and blocks on
    Gauss-Radau-Jacobi points in one whole-mesh launch."""
    say("[adr] affine and Radau blocks")
    P = 3
    blocks = [("hex", P, 7, "affine", "gj"), ("prism", P, 9, "curved", "radau"), ("pyr", P, 11, "affine", "radau"),
              ("tet", P, 13, "curved", "gj")]
    plan = shp.Plan(blocks)
    maps, jos = {}, {}
    for b, (s, _, n, geom, pts) in enumerate(blocks):
        maps[s] = W.shape_batch(s, n)
        if geom == "affine":
            jac = W.affine_jacobian(maps[s])
            jos[s] = jac
        else:
            jac = W.jacobian(maps[s], shp.quadrature(s, P + 2, pts)[0], curved=True)
            jos[s] = W.jacobian(maps[s], O.reference_points(s, P + 2, pts), curved=True)
        plan.set_geometry(b, torch.from_numpy(np.ascontiguousarray(jac)).cuda())
    nc, npnt = plan.totals()
    x = W.coeffs(1, nc, 830)[0]
    vel = W.point_values(1, npnt, 831, ncomp=3).reshape(3, npnt)
    adv = plan.advection_factors(torch.from_numpy(np.ascontiguousarray(vel)).cuda())
    y = plan.apply_adr(torch.from_numpy(x).cuda(), adv, lam=0.6).cpu().numpy()
    for b, (s, _, ne, geom, pts) in enumerate(blocks):
        co, po = plan.offsets(b)
        NP, NQ = plan.n_modes[b], plan.n_points[b]
        ref = O.apply_op("adr", s, P, P + 2, jos[s], x[co:co + ne * NP].reshape(ne, NP), lam=0.6, pts=pts,
                         vel=vel[:, po:po + ne * NQ].reshape(3, ne, NQ))
        e = rel(y[co:co + ne * NP].reshape(ne, NP), ref)
        say(f"    {s:6s} {geom:6s} {pts:5s} rel={e:.2e}")
        assert e <= TOL, (s, e)
