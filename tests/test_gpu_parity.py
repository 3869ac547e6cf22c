"""GPU parity of libshp against the FP64 oracle, through the C ABI.

Every case prints its name before touching the GPU.  The bar is the max-norm
error relative to the max-norm of the oracle's result, <= 1e-12 in FP64 (the
two differ only by summation order; a dense-matrix check of the collocated
form measured <= 8e-14).  Inputs: the library's quadrature points feed the GPU geometry, the
oracle's own points feed the oracle's geometry; coefficients and point data are
U[-1,1] from seeded generators.
"""
import os

import numpy as np
import pytest

import oracle_pool as OP
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


def gpu_geometry(shp, maps, shape, P, curved):
    xi, _ = shp.quadrature(shape, P + 2)
    if curved:
        jac = W.jacobian(maps, xi, curved=True)
    else:
        jac = W.affine_jacobian(maps)
    return torch.from_numpy(np.ascontiguousarray(jac)).cuda()


def oracle_geometry(maps, shape, P, curved):
    if curved:
        return W.jacobian(maps, O.reference_points(shape, P + 2), curved=True)
    return W.affine_jacobian(maps)


CASES = [(s, P) for s in O.SHAPES for P in (1, 2, 3, 4, 5, 6, 7, 8, 10)]


@pytest.mark.parametrize("shape,P", CASES)
def test_block_ops_vs_oracle(shp, shape, P):
    """All seven operators on a ragged batch of curved elements."""
    ne = 37 if P <= 6 else (9 if P <= 8 else 4)
    say(f"[parity] block ops shape={shape} P={P} n_elem={ne}")
    maps = W.shape_batch(shape, ne)
    NP, NQ = O.num_modes(shape, P), (P + 2) ** 3
    plan = shp.Plan([(shape, P, ne, "curved")])
    plan.set_geometry(0, gpu_geometry(shp, maps, shape, P, True))
    jo = oracle_geometry(maps, shape, P, True)
    for k, op in enumerate(OPS):
        x = op_input(op, ne, NP, NQ, 100 + k)
        ref = O.apply_op(op, shape, P, P + 2, jo, x, lam=1.0, chunk=8)
        y = plan.apply(0, op, torch.from_numpy(np.ascontiguousarray(x)).cuda(), lam=1.0)
        torch.cuda.synchronize()
        e = rel(y.cpu().numpy().reshape(ref.shape), ref)
        say(f"    {op:12s} rel={e:.2e}")
        assert e <= TOL, (shape, P, op, e)


@pytest.mark.parametrize("shape,P", [(s, P) for s in O.SHAPES for P in (1, 2, 4, 6, 9)])
def test_noncollocated_vs_oracle(shp, shape, P):
    """Alg. 5 (sum-factorised B and d_d B, strategy 'sumfac') for the Laplacian and
    Helmholtz actions, and its agreement with the collocated form (eq. helm1)."""
    ne = 23 if P <= 6 else 4
    say(f"[parity] non-collocated shape={shape} P={P}")
    maps = W.shape_batch(shape, ne)
    plan = shp.Plan([(shape, P, ne, "curved")])
    plan.set_geometry(0, gpu_geometry(shp, maps, shape, P, True))
    jo = oracle_geometry(maps, shape, P, True)
    for k, op in enumerate(("laplacian", "helmholtz")):
        x = W.coeffs(ne, plan.n_modes[0], 400 + k)
        ref = O.apply_op(op, shape, P, P + 2, jo, x, lam=0.7, chunk=8)
        xt = torch.from_numpy(x).cuda()
        y = plan.apply(0, op, xt, lam=0.7, strategy="sumfac").cpu().numpy()
        yc = plan.apply(0, op, xt, lam=0.7, strategy="sumfac_coll").cpu().numpy()
        e = rel(y, ref)
        say(f"    {op:12s} rel={e:.2e} vs collocated {rel(y, yc):.2e}")
        assert e <= TOL, (shape, P, op, e)
        assert rel(y, yc) <= TOL


@pytest.mark.parametrize("shape,P", [(s, P) for s in O.SHAPES for P in (1, 2, 3, 4)])
@pytest.mark.parametrize("curved", [True, False])
def test_localmat_vs_oracle(shp, shape, P, curved):
    """The local-matrix strategy on FP64 MFMA, every operator (BwdTrans as one
    GEMM, IProduct, PhysDeriv with dense collocation derivatives,
    IProductDeriv, mass, Laplacian, Helmholtz) on a ragged batch (not a
    multiple of the 16-element tile nor of the 4-wave work-group), curved and
    affine blocks."""
    ne = 37
    say(f"[parity] local matrix shape={shape} P={P} curved={curved}")
    maps = W.shape_batch(shape, ne)
    NP, NQ = O.num_modes(shape, P), (P + 2) ** 3
    plan = shp.Plan([(shape, P, ne, "curved" if curved else "affine")])
    plan.set_geometry(0, gpu_geometry(shp, maps, shape, P, curved))
    jo = oracle_geometry(maps, shape, P, curved)
    for k, op in enumerate(OPS):
        x = op_input(op, ne, NP, NQ, 500 + k)
        ref = O.apply_op(op, shape, P, P + 2, jo, x, lam=1.7)
        y = plan.apply(0, op, torch.from_numpy(np.ascontiguousarray(x)).cuda(), lam=1.7, strategy="localmat").cpu().numpy()
        e = rel(y.reshape(ref.shape), ref)
        say(f"    {op:12s} rel={e:.2e}")
        assert e <= TOL, (shape, P, op, e)


@pytest.mark.parametrize("shape", ["hex", "tet"])
def test_localmat_transforms_large_block(shp, shape):
    """The local-matrix transforms on a curved P = 4 block of 65549 elements
    (4097 tiles, a ragged last one): there BwdTrans takes one wave per tile,
    the launch form that smaller blocks split among up to 8 waves.  Every
    transform against the oracle on sampled elements (the first 40, the last
    21, 24 random ones)."""
    ne, P = 65549, 4
    say(f"[parity] local-matrix transforms, large block shape={shape} P={P} n_elem={ne}")
    maps = W.shape_batch(shape, ne)
    NP, NQ = O.num_modes(shape, P), (P + 2) ** 3
    plan = shp.Plan([(shape, P, ne, "curved")])
    plan.set_geometry(0, gpu_geometry(shp, maps, shape, P, True))
    rng = np.random.default_rng(705)
    idx = np.unique(np.concatenate([np.arange(40), np.arange(ne - 21, ne), rng.integers(0, ne, 24)]))
    jo = oracle_geometry(maps.take(idx), shape, P, True)
    for k, op in enumerate(("bwd", "iprod", "physderiv", "iprod_deriv")):
        x = op_input(op, ne, NP, NQ, 700 + k)
        y = plan.apply(0, op, torch.from_numpy(np.ascontiguousarray(x)).cuda(), strategy="localmat").cpu().numpy()
        if op == "iprod_deriv":
            ref = O.apply_op(op, shape, P, P + 2, jo, x[:, idx])
            got = y.reshape(ne, NP)[idx]
        elif op == "physderiv":
            ref = O.apply_op(op, shape, P, P + 2, jo, x[idx])
            got = y.reshape(3, ne, NQ)[:, idx]
        else:
            ref = O.apply_op(op, shape, P, P + 2, jo, x[idx])
            got = y.reshape(ne, -1)[idx]
        e = rel(got, ref)
        say(f"    {op:12s} rel={e:.2e}")
        assert e <= TOL, (shape, op, e)


def test_localmat_whole_mesh_and_limits(shp):
    say("[parity] local matrix whole mesh and limits")
    mesh, plan = _mixed_plan(shp, 4, 2)
    nc, _ = plan.totals()
    x = W.coeffs(1, nc, 41)[0]
    y = plan.apply(-1, "helmholtz", torch.from_numpy(x).cuda(), strategy="localmat").cpu().numpy()
    for b, s in enumerate(O.SHAPES):
        co, _ = plan.offsets(b)
        ne, NP = len(mesh[s]), plan.n_modes[b]
        ref = O.apply_op("helmholtz", s, 2, 4, oracle_geometry(mesh[s], s, 2, True), x[co:co + ne * NP].reshape(ne, NP))
        assert rel(y[co:co + ne * NP].reshape(ne, NP), ref) <= TOL
    # the transforms over the whole mesh equal the per-block launches, and
    # BwdTrans (one GEMM per block) equals the oracle
    u = plan.apply(-1, "bwd", torch.from_numpy(x).cuda(), strategy="localmat").cpu().numpy()
    for b, s in enumerate(O.SHAPES):
        co, po = plan.offsets(b)
        ne, NP, NQ = len(mesh[s]), plan.n_modes[b], plan.n_points[b]
        ref = O.apply_op("bwd", s, 2, 4, oracle_geometry(mesh[s], s, 2, True), x[co:co + ne * NP].reshape(ne, NP))
        assert rel(u[po:po + ne * NQ].reshape(ne, NQ), ref) <= TOL
    nc, npnt = plan.totals()
    f3 = torch.from_numpy(np.ascontiguousarray(W.point_values(1, 3 * npnt, 43)[0])).cuda()
    g = plan.apply(-1, "iprod_deriv", f3, strategy="localmat").cpu().numpy()
    gs = plan.apply(-1, "iprod_deriv", f3, strategy="sumfac_coll").cpu().numpy()
    assert rel(g, gs) <= TOL
    maps = W.shape_batch("hex", 3)
    p5 = shp.Plan([("hex", 5, 3, "curved")])
    p5.set_geometry(0, gpu_geometry(shp, maps, "hex", 5, True))
    with pytest.raises(shp.ShpError) as ei:      # dense reference matrices only up to P = 4
        p5.apply(0, "helmholtz", torch.zeros(3, p5.n_modes[0], dtype=torch.float64, device="cuda"),
                 strategy="localmat")
    assert ei.value.code == -2


def test_noncollocated_whole_mesh(shp):
    say("[parity] non-collocated whole mesh")
    mesh, plan = _mixed_plan(shp, 4, 3)
    nc, _ = plan.totals()
    x = torch.from_numpy(W.coeffs(1, nc, 31)[0]).cuda()
    y = plan.apply(-1, "helmholtz", x, strategy="sumfac").cpu().numpy()
    for b, s in enumerate(O.SHAPES):
        co, _ = plan.offsets(b)
        ne, NP = len(mesh[s]), plan.n_modes[b]
        xb = x.cpu().numpy()[co:co + ne * NP].reshape(ne, NP)
        yb = plan.apply(b, "helmholtz", torch.from_numpy(xb).cuda(), strategy="sumfac").cpu().numpy()
        assert np.array_equal(y[co:co + ne * NP].reshape(ne, NP), yb)
        ref = O.apply_op("helmholtz", s, 3, 5, oracle_geometry(mesh[s], s, 3, True), xb)
        assert rel(yb, ref) <= TOL


@pytest.mark.parametrize("shape", O.SHAPES)
def test_affine_blocks_vs_oracle(shp, shape):
    P, ne = 3, 21
    say(f"[parity] affine shape={shape} P={P}")
    maps = W.shape_batch(shape, ne)
    NP, NQ = O.num_modes(shape, P), (P + 2) ** 3
    plan = shp.Plan([(shape, P, ne, "affine")])
    plan.set_geometry(0, gpu_geometry(shp, maps, shape, P, False))
    jo = oracle_geometry(maps, shape, P, False)
    for k, op in enumerate(OPS):
        x = op_input(op, ne, NP, NQ, 200 + k)
        ref = O.apply_op(op, shape, P, P + 2, jo, x, lam=2.5)
        y = plan.apply(0, op, torch.from_numpy(np.ascontiguousarray(x)).cuda(), lam=2.5)
        e = rel(y.cpu().numpy().reshape(ref.shape), ref)
        assert e <= TOL, (shape, op, e)


@pytest.mark.parametrize("shape,P", [(s, P) for s in O.SHAPES for P in (1, 2, 3, 4)])
def test_affine_localmat_vs_oracle(shp, shape, P):
    """Affine local matrices (7 reference matrices, 7 coefficients per element,
    FP64 MFMA) for mass, Laplacian and Helmholtz on a ragged batch (the last
    16-element tile and the last work-group partial) against the oracle, and
    against the affine sum-factorisation of the same block."""
    ne = 83
    say(f"[parity] affine local matrices shape={shape} P={P} n_elem={ne}")
    maps = W.shape_batch(shape, ne)
    NP = O.num_modes(shape, P)
    plan = shp.Plan([(shape, P, ne, "affine")])
    plan.set_geometry(0, gpu_geometry(shp, maps, shape, P, False))
    jo = oracle_geometry(maps, shape, P, False)
    for k, op in enumerate(("mass", "laplacian", "helmholtz")):
        x = W.coeffs(ne, NP, 700 + k)
        xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        ref = O.apply_op(op, shape, P, P + 2, jo, x, lam=2.5)
        y = plan.apply(0, op, xt, lam=2.5, strategy="localmat").cpu().numpy()
        e = rel(y.reshape(ref.shape), ref)
        assert e <= TOL, (shape, op, e)
        ys = plan.apply(0, op, xt, lam=2.5, strategy="sumfac_coll").cpu().numpy()
        assert rel(y, ys) <= TOL, (shape, op)


def test_affine_localmat_whole_mesh(shp):
    """Whole-mesh local matrices over affine blocks of every shape equal the
    per-block launches bitwise (the same kernel per block)."""
    say("[parity] affine local matrices, whole mesh")
    P = 2
    blocks = [(s, P, n, "affine") for s, n in zip(O.SHAPES, (5, 17, 33, 40))]
    plan = shp.Plan(blocks)
    maps = {}
    for b, (s, _, n, _) in enumerate(blocks):
        maps[s] = W.shape_batch(s, n)
        plan.set_geometry(b, gpu_geometry(shp, maps[s], s, P, False))
    nc, _ = plan.totals()
    x = torch.from_numpy(W.coeffs(1, nc, 710)[0]).cuda()
    y = plan.apply(-1, "helmholtz", x, strategy="localmat").cpu().numpy()
    for b, (s, _, n, _) in enumerate(blocks):
        co, _ = plan.offsets(b)
        NP = plan.n_modes[b]
        yb = plan.apply(b, "helmholtz", x[co:co + n * NP].view(n, NP).contiguous(), strategy="localmat")
        assert np.array_equal(y[co:co + n * NP], yb.cpu().numpy().ravel()), s


def test_affine_hex_grid_64_P2_helmholtz(shp):
    """64 affine hexes of side 1/4, P=2, Q=4, lambda=1, seed 0."""
    say("[parity] 64 affine hexahedra (4^3 grid), P=2")
    maps = W.affine_hex_grid(4)
    P = 2
    x = W.coeffs(64, 27, W.SEED_CFG1)
    plan = shp.Plan([("hex", P, 64, "affine")])
    plan.set_geometry(0, torch.from_numpy(W.affine_jacobian(maps)).cuda())
    y = plan.apply(0, "helmholtz", torch.from_numpy(x).cuda(), lam=1.0).cpu().numpy()
    ref = O.apply_op("helmholtz", "hex", P, 4, W.affine_jacobian(maps), x, lam=1.0)
    assert rel(y, ref) <= TOL


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4])
def test_whole_mesh_variants_agree(shp, variant):
    """Every launch variant of the whole-mesh Helmholtz launch gives the same bits."""
    say(f"[parity] whole-mesh variant={variant}")
    mesh, plan = _mixed_plan(shp, 4, 4)
    nc, _ = plan.totals()
    x = torch.from_numpy(W.coeffs(1, nc, 21)[0]).cuda()
    plan.set_tiling(-1, "helmholtz", 1, 64, 3 if variant >= 3 else 0)
    base = plan.apply(-1, "helmholtz", x).cpu().numpy()
    for E, NT in ((1, 64), (2, 128), (4, 256), (3, 192), (7, 256)):
        plan.set_tiling(-1, "helmholtz", E, NT, variant)
        y = plan.apply(-1, "helmholtz", x).cpu().numpy()
        assert np.array_equal(y, base), (E, NT, variant)


def _mixed_plan(shp, ncell, P):
    mesh = W.quadrant_mesh(ncell)
    blocks = [(s, P, len(mesh[s]), "curved") for s in O.SHAPES]
    plan = shp.Plan(blocks)
    for b, s in enumerate(O.SHAPES):
        plan.set_geometry(b, gpu_geometry(shp, mesh[s], s, P, True))
    return mesh, plan


def _whole_mesh_input(op, nc, npnt, seed):
    if op in ("iprod", "physderiv"):
        return W.point_values(1, npnt, seed)[0]
    if op == "iprod_deriv":
        return W.point_values(1, npnt, seed, ncomp=3).reshape(3, npnt)
    return W.coeffs(1, nc, seed)[0]


def _block_slices(op, plan, b, ne, x, y):
    """Block b's part of a whole-mesh input x and output y."""
    co, po = plan.offsets(b)
    NP, NQ = plan.n_modes[b], plan.n_points[b]
    if op in ("iprod", "physderiv"):
        xb = x[po:po + ne * NQ].reshape(ne, NQ)
    elif op == "iprod_deriv":
        xb = x[:, po:po + ne * NQ].reshape(3, ne, NQ)
    else:
        xb = x[co:co + ne * NP].reshape(ne, NP)
    if op == "bwd":
        yb = y[po:po + ne * NQ].reshape(ne, NQ)
    elif op == "physderiv":
        yb = y.reshape(3, -1)[:, po:po + ne * NQ].reshape(3, ne, NQ)
    else:
        yb = y[co:co + ne * NP].reshape(ne, NP)
    return xb, yb


@pytest.mark.parametrize("P", list(range(1, 11)))
def test_whole_mesh_launch(shp, P):
    """One mixed-shape launch over the 4^3-cell mesh (16 hexes, 32 prisms, 96
    pyramids, 96 tets) equals the per-block launches bitwise and the oracle on
    every element to the FP64 bar, for every operator and order (at P = 6 and 7
    the whole-mesh Helmholtz tile holds two elements, the per-block tiles one)."""
    say(f"[parity] whole-mesh launch P={P}")
    mesh, plan = _mixed_plan(shp, 4, P)
    nc, npnt = plan.totals()
    for k, op in enumerate(OPS):
        x = _whole_mesh_input(op, nc, npnt, 300 + k)
        xt = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        y = plan.apply(-1, op, xt, lam=1.0).cpu().numpy()
        worst = 0.0
        for b, s in enumerate(O.SHAPES):
            ne = len(mesh[s])
            xb, ym = _block_slices(op, plan, b, ne, x, y)
            yb = plan.apply(b, op, torch.from_numpy(np.ascontiguousarray(xb)).cuda(), lam=1.0).cpu().numpy()
            assert np.array_equal(ym, yb.reshape(ym.shape)), (op, s)
            ref = OP.apply_op(op, s, P, mesh[s], xb, lam=1.0)
            e = rel(ym.reshape(ref.shape), ref)
            worst = max(worst, e)
            assert e <= TOL, (op, s, e)
        say(f"    {op:12s} every element, worst shape rel={worst:.2e}")


@pytest.mark.parametrize("P,E,NT,variant", [(7, 2, 512, 0), (7, 2, 256, 2), (5, 4, 256, 0), (8, 1, 512, 0)])
def test_whole_mesh_tuned_shapes(shp, P, E, NT, variant):
    """Whole-mesh Helmholtz launch shapes the tuner picks (P = 7: two elements on
    512 threads without prefetch) give the same bits as the default shape and
    match the oracle on every element."""
    say(f"[parity] whole-mesh tuned launch P={P} E={E} threads={NT} variant={variant}")
    mesh, plan = _mixed_plan(shp, 4, P)
    nc, _ = plan.totals()
    x = W.coeffs(1, nc, 350 + P)[0]
    xt = torch.from_numpy(x).cuda()
    base = plan.apply(-1, "helmholtz", xt, lam=0.5).cpu().numpy()
    plan.set_tiling(-1, "helmholtz", E, NT, variant)
    y = plan.apply(-1, "helmholtz", xt, lam=0.5).cpu().numpy()
    assert np.array_equal(y, base)
    for b, s in enumerate(O.SHAPES):
        ne = len(mesh[s])
        xb, yb = _block_slices("helmholtz", plan, b, ne, x, y)
        ref = OP.apply_op("helmholtz", s, P, mesh[s], xb, lam=0.5)
        assert rel(yb, ref) <= TOL, s


@pytest.mark.parametrize("shape", O.SHAPES)
def test_tilings_agree_bitwise(shp, shape):
    """Every launch shape computes each element with the same arithmetic."""
    P, ne = 4, 53
    say(f"[parity] tilings shape={shape}")
    maps = W.shape_batch(shape, ne)
    plan = shp.Plan([(shape, P, ne, "curved")])
    plan.set_geometry(0, gpu_geometry(shp, maps, shape, P, True))
    x = torch.from_numpy(W.coeffs(ne, plan.n_modes[0], 9)).cuda()
    base = {}
    plan.set_tiling(0, "helmholtz", 1, 64, 0)
    base[0] = plan.apply(0, "helmholtz", x).cpu().numpy()
    plan.set_tiling(0, "helmholtz", 1, 64, 3)
    base[3] = plan.apply(0, "helmholtz", x).cpu().numpy()
    # the two families (separate stages; fused stages) differ by summation order only
    assert rel(base[3], base[0]) < 1e-14
    ref = O.apply_op("helmholtz", shape, P, P + 2, oracle_geometry(maps, shape, P, True), x.cpu().numpy())
    assert rel(base[3], ref) <= TOL
    for E, NT, pe in ((1, 64, 0), (2, 128, 0), (5, 256, 0), (8, 512, 0), (3, 192, 0),
                      (1, 64, 1), (2, 128, 1), (4, 256, 1), (8, 512, 1), (3, 192, 1), (6, 256, 1),
                      (1, 64, 2), (2, 128, 2), (4, 256, 2), (8, 512, 2), (3, 192, 2), (6, 256, 2),
                      (1, 64, 3), (2, 128, 3), (4, 256, 3), (7, 512, 3), (3, 192, 3), (5, 320, 3),
                      (1, 64, 4), (2, 128, 4), (4, 256, 4), (7, 256, 4), (3, 192, 4), (5, 320, 4)):
        plan.set_tiling(0, "helmholtz", E, NT, pe)
        y = plan.apply(0, "helmholtz", x).cpu().numpy()
        assert np.array_equal(y, base[3 if pe >= 3 else 0]), (E, NT, pe)


def test_bad_geometry_is_reported(shp):
    say("[parity] bad geometry error path")
    maps = W.shape_batch("tet", 6)
    jac = gpu_geometry(shp, maps, "tet", 2, True)
    jac[3, 0:3, :] *= -1.0         # reflect element 3 (negate row 0 of dx/dxi): det < 0
    plan = shp.Plan([("tet", 2, 6, "curved")])
    with pytest.raises(shp.ShpError) as ei:
        plan.set_geometry(0, jac)
    assert ei.value.code == -3
    x = torch.zeros(6, plan.n_modes[0], dtype=torch.float64, device="cuda")
    with pytest.raises(shp.ShpError):
        plan.apply(0, "helmholtz", x)


def test_empty_block(shp):
    say("[parity] empty block")
    plan = shp.Plan([("hex", 3, 0, "curved"), ("tet", 3, 5, "curved")])
    maps = W.shape_batch("tet", 5)
    plan.set_geometry(0, torch.zeros(0, 9, 125, dtype=torch.float64, device="cuda"))
    plan.set_geometry(1, gpu_geometry(shp, maps, "tet", 3, True))
    x = torch.from_numpy(W.coeffs(1, plan.totals()[0], 3)[0]).cuda()
    y = plan.apply(-1, "helmholtz", x).cpu().numpy()
    ref = O.apply_op("helmholtz", "tet", 3, 5, oracle_geometry(maps, "tet", 3, True),
                     x.cpu().numpy().reshape(5, -1))
    assert rel(y.reshape(ref.shape), ref) <= TOL


@pytest.fixture(scope="module")
def mesh32_p4(shp):
    say("[parity] building the 32^3 mixed mesh at P=4")
    return _mixed_plan(shp, 32, 4)


@pytest.mark.parametrize("op", ["helmholtz", "bwd", "iprod", "physderiv"])
def test_mixed_mesh_32_P4_every_element(shp, mesh32_p4, op):
    """The mixed P=4 mesh (32^3 cells, 122,880 curved elements) in one launch,
    checked against the oracle on every element (the oracle runs in worker
    processes on the host's cores)."""
    say(f"[parity] 32^3-cell mixed mesh P=4, every element, op={op}")
    P = 4
    mesh, plan = mesh32_p4
    nc, npnt = plan.totals()
    seeds = W.SEED_MIXED
    if op in ("iprod", "physderiv"):
        parts = [W.point_values(len(mesh[s]), (P + 2) ** 3, seeds[s]).ravel() for s in O.SHAPES]
    else:
        parts = [W.coeffs(len(mesh[s]), plan.n_modes[b], seeds[s]).ravel() for b, s in enumerate(O.SHAPES)]
    x = np.concatenate(parts)
    y = plan.apply(-1, op, torch.from_numpy(x).cuda(), lam=1.0).cpu().numpy()
    for b, s in enumerate(O.SHAPES):
        ne = len(mesh[s])
        xb, yb = _block_slices(op, plan, b, ne, x, y)
        ref = OP.apply_op(op, s, P, mesh[s], xb, lam=1.0)
        e = rel(yb, ref)
        say(f"    {s:5s} all {ne} elements rel={e:.2e}")
        assert e <= TOL, (s, e)
