"""GPU parity of libshp with Gauss-Radau-Jacobi points in the collapsed
directions (the node eta = -1 included), through the C ABI, against the FP64
oracle on its own Radau rule (Golub's modified Jacobi matrix).  Same bar as the
Gauss-Jacobi cases: max-norm error relative to the oracle's max-norm <= 1e-12
in FP64.  Every case prints its name before touching the GPU."""
import numpy as np
import pytest

from oracle import shp_oracle as O
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
        return W.point_values(ne, NQ, seed, ncomp=3)
    return W.coeffs(ne, NP, seed)


@pytest.mark.parametrize("shape,P", [(s, P) for s in ("prism", "pyr", "tet") for P in (1, 3, 4, 7)])
def test_radau_block_ops_vs_oracle(shp, shape, P):
    """All seven operators (collocated), the non-collocated Laplacian and
    Helmholtz, and for P <= 4 the local matrices, on a ragged curved batch."""
    ne = 29 if P <= 4 else 11
    say(f"[radau] block ops shape={shape} P={P} n_elem={ne}")
    maps = W.shape_batch(shape, ne)
    NP, NQ = O.num_modes(shape, P), (P + 2) ** 3
    plan = shp.Plan([(shape, P, ne, "curved", "radau")])
    xi, _ = shp.quadrature(shape, P + 2, "radau")
    plan.set_geometry(0, torch.from_numpy(np.ascontiguousarray(W.jacobian(maps, xi, curved=True))).cuda())
    jo = W.jacobian(maps, O.reference_points(shape, P + 2, "radau"), curved=True)
    for k, op in enumerate(OPS):
        x = op_input(op, ne, NP, NQ, 900 + k)
        ref = O.apply_op(op, shape, P, P + 2, jo, x, lam=1.3, chunk=8, pts="radau")
        xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        strategies = ["sumfac_coll"]
        if op in ("laplacian", "helmholtz"):
            strategies.append("sumfac")
        if op in ("mass", "laplacian", "helmholtz") and P <= 4:
            strategies.append("localmat")
        for st in strategies:
            y = plan.apply(0, op, xt, lam=1.3, strategy=st).cpu().numpy()
            e = rel(y.reshape(ref.shape), ref)
            say(f"    {op:12s} {st:12s} rel={e:.2e}")
            assert e <= TOL, (shape, P, op, st, e)


@pytest.mark.parametrize("shape", ("prism", "pyr", "tet"))
def test_radau_affine_vs_oracle(shp, shape):
    """Affine blocks: the sum-factorised Helmholtz and the 7-matrix local-matrix
    form built on the Radau rule."""
    P, ne = 3, 37
    say(f"[radau] affine shape={shape} P={P}")
    maps = W.shape_batch(shape, ne)
    plan = shp.Plan([(shape, P, ne, "affine", "radau")])
    plan.set_geometry(0, torch.from_numpy(np.ascontiguousarray(W.affine_jacobian(maps))).cuda())
    jo = W.affine_jacobian(maps)
    x = W.coeffs(ne, plan.n_modes[0], 950)
    ref = O.apply_op("helmholtz", shape, P, P + 2, jo, x, lam=2.5, pts="radau")
    xt = torch.from_numpy(x).cuda()
    for st in ("sumfac_coll", "localmat"):
        e = rel(plan.apply(0, "helmholtz", xt, lam=2.5, strategy=st).cpu().numpy(), ref)
        say(f"    helmholtz {st:12s} rel={e:.2e}")
        assert e <= TOL, (shape, st, e)


def test_radau_whole_mesh_mixed_points(shp):
    """One whole-mesh launch over blocks with both point sets (each block's own
    tables), FP64 and the FP32-contraction path, against the oracle per block."""
    P = 4
    mesh = W.quadrant_mesh(2)
    blocks = [(s, P, len(mesh[s]), "curved", "radau" if s in ("prism", "tet") else "gj") for s in O.SHAPES]
    say(f"[radau] whole mesh P={P} blocks={[(b[0], b[2], b[4]) for b in blocks]}")
    plan = shp.Plan(blocks)
    for b, (s, _, _, _, pts) in enumerate(blocks):
        xi, _ = shp.quadrature(s, P + 2, pts)
        plan.set_geometry(b, torch.from_numpy(np.ascontiguousarray(W.jacobian(mesh[s], xi, curved=True))).cuda())
    nc, _ = plan.totals()
    x = W.coeffs(1, nc, 960)[0].astype(np.float32).astype(np.float64)  # exact in FP32 too
    xt = torch.from_numpy(x).cuda()
    y = plan.apply(-1, "helmholtz", xt, lam=1.0).cpu().numpy()
    y32 = plan.apply_prec("helmholtz", xt.float(), lam=1.0, prec="fp32").double().cpu().numpy()
    for b, (s, _, ne, _, pts) in enumerate(blocks):
        co, _ = plan.offsets(b)
        NP = plan.n_modes[b]
        jo = W.jacobian(mesh[s], O.reference_points(s, P + 2, pts), curved=True)
        ref = O.apply_op("helmholtz", s, P, P + 2, jo, x[co:co + ne * NP].reshape(ne, NP), lam=1.0, pts=pts)
        e = rel(y[co:co + ne * NP].reshape(ne, NP), ref)
        e32 = rel(y32[co:co + ne * NP].reshape(ne, NP), ref)
        say(f"    {s:6s} {pts:6s} fp64 rel={e:.2e} fp32 rel={e32:.2e}")
        assert e <= TOL, (s, pts, e)
        assert e32 <= 5e-6, (s, pts, e32)
