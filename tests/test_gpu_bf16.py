"""Split-BF16 affine local-matrix actions and the solve with BF16 inner
actions, through the C ABI, against the FP64 oracle.

The kernel forms y_e = sum_k A_k (c_{e,k} x_e) as one contraction over
kappa = (k, n) of K = 7 N_P terms (N_P for the mass).  The matrices are split
into bfloat16 parts rounded to nearest (each the rounding of what the previous
parts leave: relative error 2^-9, 2^-18, 2^-27 after one, two, three parts);
the B values c_k x_n, rounded to FP32, are split by truncation (2^-8, 2^-16
after one and two parts; three parts hold the FP32 value exactly).  The part
products of order below the part count are accumulated in FP32.  Per product
a b the dropped terms are, relative to |a b|:
  three parts (SHP_BF16):   a1 b2 (2^-25), a2 b1 (2^-26), a2 b2 and the
                            matrix remainder (2^-27): about 7e-8;
  two parts (SHP_BF16X3):   a1 b1 (2^-17), b's remainder (2^-16) and a's
                            (2^-18): about 2.5e-5 at worst, 1e-5 typically.
On top come FP32 roundings of c_k and of c_k x_n (2^-24 each) and the FP32
accumulation of K terms, about sqrt(K) 2^-24 of sum |a b| for rounding errors
of random sign (K <= 875 here: 1.8e-6; K 2^-24 = 5e-5 is the worst case).
The bars are on the error relative to the max-norm of the scale
s_e = sum_k |c_{e,k}| |A_k| |x_e|, which the oracle forms from its own dense
mass and stiffness blocks (the coefficients c come from J alone):
  three parts: 2e-6   (the FP32 accumulation term, with margin);
  two parts:   3e-5   (the dropped first-order products, with margin).
The oracle acts on the same FP32-rounded coefficients.
"""
import numpy as np
import pytest

from oracle import shp_oracle as O
from paper_2604_04644_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BAR = {"bf16": 2e-6, "bf16x3": 3e-5}
RESID_TOL = {1e-6: 1e-9, 1e-10: 2e-13}
LAM = 2.5


@pytest.fixture(scope="module")
def shp():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2604_04644_amd import shp as S
    S.lib()
    return S


def say(msg):
    print(msg, flush=True)


def scale(shape, P, jac, x, op, lam):
    """s_e = |H_e|-type bound sum_k |c_k| |A_k| |x_e| from the oracle's own
    dense matrices: A_0 the mass of the reference map, A_ab the xi-space
    stiffness blocks (recovered from Laplacians of maps with chosen J^-1 J^-T)."""
    Q = P + 2
    J = np.asarray(jac, dtype=np.float64).reshape(-1, 3, 3)
    det = np.linalg.det(J)
    Ji = np.linalg.inv(J)
    G = det[:, None, None] * np.einsum("eai,ebi->eab", Ji, Ji)
    ref = np.eye(3).reshape(1, 9)
    A0 = O.Element(shape, P, Q, ref).mass()[0]                # |J| = 1 for the identity map
    # the Laplacian of a map with G = |J| J^-1 J^-T is sum_ab G_ab S_ab; the
    # identity and three axis scalings give the S_aa, shears the S_ab + S_ba
    blocks = {}
    L_id = O.Element(shape, P, Q, ref).laplacian()[0]
    diag = []
    for a in range(3):
        Jd = np.eye(3)
        Jd[a, a] = 0.5                                          # G_aa = |J| / 0.25, others |J|
        Ga = np.linalg.det(Jd) * np.linalg.inv(Jd) @ np.linalg.inv(Jd).T
        La = O.Element(shape, P, Q, Jd.reshape(1, 9)).laplacian()[0]
        diag.append((Ga, La))
    # solve for S_aa from L_id = sum S_aa and La = sum_b Ga_bb S_bb
    Mat = np.array([[1.0, 1.0, 1.0]] + [[Ga[b, b] for b in range(3)] for Ga, _ in diag])
    rhs = [L_id] + [La for _, La in diag]
    sol = np.linalg.lstsq(Mat, np.stack([r.ravel() for r in rhs]), rcond=None)[0]
    for a in range(3):
        blocks[(a, a)] = sol[a].reshape(L_id.shape)
    for a in range(3):
        for b in range(a + 1, 3):
            Js = np.eye(3)
            Js[a, b] = 0.5                                      # shear: G_ab != 0
            Gs = np.linalg.det(Js) * np.linalg.inv(Js) @ np.linalg.inv(Js).T
            Ls = O.Element(shape, P, Q, Js.reshape(1, 9)).laplacian()[0]
            rest = Ls - sum(Gs[c, c] * blocks[(c, c)] for c in range(3))
            blocks[(a, b)] = rest / Gs[a, b]                    # S_ab + S_ba
    ax = np.abs(x)
    s = np.zeros_like(x)
    if op in ("mass", "helmholtz"):
        w = det * (lam if op == "helmholtz" else 1.0)
        s += np.abs(w)[:, None] * (ax @ np.abs(A0).T)
    if op in ("laplacian", "helmholtz"):
        for (a, b), Sab in blocks.items():
            s += np.abs(G[:, a, b])[:, None] * (ax @ np.abs(Sab).T)
    return s


def affine_plan(shp, blocks):
    """Plan of affine blocks [(shape, P, maps)] with geometry set."""
    plan = shp.Plan([(s, P, len(m), "affine") for s, P, m in blocks])
    for b, (s, P, m) in enumerate(blocks):
        plan.set_geometry(b, torch.from_numpy(np.ascontiguousarray(W.affine_jacobian(m))).cuda())
    return plan


@pytest.mark.parametrize("shape,P", [(s, P) for s in O.SHAPES for P in (1, 2, 3, 4)])
@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
def test_bf16_action_vs_oracle(shp, shape, P, prec):
    """Mass, Laplacian and Helmholtz of one affine block on a ragged batch
    (83 elements: the last 16-element tile and the last wave partial) in split
    BF16 against the oracle on the FP32-rounded coefficients."""
    ne = 83
    say(f"[bf16] {prec} shape={shape} P={P} n_elem={ne}")
    maps = W.shape_batch(shape, ne)
    NP = O.num_modes(shape, P)
    plan = affine_plan(shp, [(shape, P, maps)])
    jac = W.affine_jacobian(maps)
    worst = 0.0
    for k, op in enumerate(("mass", "laplacian", "helmholtz")):
        x = W.coeffs(ne, NP, 900 + k).astype(np.float32)
        y = plan.apply_prec(op, torch.from_numpy(x).cuda(), lam=LAM, prec=prec, blk=0).cpu().numpy()
        assert y.dtype == np.float32
        x64 = x.astype(np.float64)
        ref = O.apply_op(op, shape, P, P + 2, jac, x64, lam=LAM)
        s = scale(shape, P, jac, x64, op, LAM)
        # the scale bounds the result itself (a check of the decomposition)
        assert np.all(np.abs(ref) <= s * (1 + 1e-9) + 1e-300), (shape, op)
        e = float(np.abs(y.astype(np.float64) - ref).max() / s.max())
        worst = max(worst, e)
        assert e <= BAR[prec], (shape, op, e)
    say(f"    worst {worst:.2e} of the scale")


@pytest.mark.parametrize("shape,P", [(s, P) for s in O.SHAPES for P in (1, 2, 3, 4)])
def test_fp32_localmat_vs_oracle(shp, shape, P):
    """The affine local matrices in FP32 on the FP32 matrix cores (matrices
    and coefficients rounded to FP32, FP32 accumulation): the error of the FP32
    roundings (2^-24 of each matrix entry, coefficient and product) and of the
    accumulation over K = 7 N_P terms, under the three-part BF16 bar; whole
    mesh and single block launches agree."""
    ne = 83
    say(f"[fp32 localmat] shape={shape} P={P} n_elem={ne}")
    maps = W.shape_batch(shape, ne)
    NP = O.num_modes(shape, P)
    plan = affine_plan(shp, [(shape, P, maps)])
    jac = W.affine_jacobian(maps)
    worst = 0.0
    for k, op in enumerate(("mass", "laplacian", "helmholtz")):
        x = W.coeffs(ne, NP, 920 + k).astype(np.float32)
        xt = torch.from_numpy(x).cuda()
        y = plan.apply_prec(op, xt, lam=LAM, prec="fp32", blk=0, strategy="localmat").cpu().numpy()
        yw = plan.apply_prec(op, xt.reshape(-1), lam=LAM, prec="fp32", strategy="localmat").cpu().numpy()
        assert np.array_equal(y.ravel(), yw.ravel())
        x64 = x.astype(np.float64)
        ref = O.apply_op(op, shape, P, P + 2, jac, x64, lam=LAM)
        s = scale(shape, P, jac, x64, op, LAM)
        e = float(np.abs(y.astype(np.float64) - ref).max() / s.max())
        worst = max(worst, e)
        assert e <= BAR["bf16"], (shape, op, e)
    say(f"    worst {worst:.2e} of the scale")


@pytest.mark.parametrize("shape,P", [(s, P) for s in O.SHAPES for P in (1, 3, 4)])
def test_affine_localmat_wide_launch(shp, shape, P):
    """Affine blocks large enough that the local-matrix launches take their
    wide form (two 16-element tiles per wave sharing every A fragment, a
    tile's row blocks split among waves): 33013 elements, a ragged last
    tile.  FP64 and FP32 Helmholtz against the oracle on sampled elements
    (the first 40, the last 21, 24 random ones), and the first 37 elements
    bit for bit equal to a 37-element launch (one tile per wave)."""
    ne, ns = 33013, 37
    say(f"[localmat wide] shape={shape} P={P} n_elem={ne}")
    maps = W.shape_batch(shape, ne)
    NP = O.num_modes(shape, P)
    jac = np.ascontiguousarray(W.affine_jacobian(maps))
    plan = shp.Plan([(shape, P, ne, "affine")])
    plan.set_geometry(0, torch.from_numpy(jac).cuda())
    small = shp.Plan([(shape, P, ns, "affine")])
    small.set_geometry(0, torch.from_numpy(np.ascontiguousarray(jac[:ns])).cuda())
    rng = np.random.default_rng(941)
    idx = np.unique(np.concatenate([np.arange(40), np.arange(ne - 21, ne), rng.integers(0, ne, 24)]))
    x = W.coeffs(ne, NP, 940)
    for prec, bar in (("fp64", 1e-12), ("fp32", BAR["bf16"])):
        xs = x if prec == "fp64" else x.astype(np.float32)
        xt = torch.from_numpy(np.ascontiguousarray(xs)).cuda()
        if prec == "fp64":
            y = plan.apply(0, "helmholtz", xt, lam=LAM, strategy="localmat")
            ys = small.apply(0, "helmholtz", xt[:ns].contiguous(), lam=LAM, strategy="localmat")
        else:
            y = plan.apply_prec("helmholtz", xt, lam=LAM, prec="fp32", blk=0, strategy="localmat")
            ys = small.apply_prec("helmholtz", xt[:ns].contiguous(), lam=LAM, prec="fp32", blk=0, strategy="localmat")
        y, ys = y.cpu().numpy().reshape(ne, NP), ys.cpu().numpy().reshape(ns, NP)
        assert np.array_equal(y[:ns], ys), (shape, P, prec)
        x64 = xs[idx].astype(np.float64)
        ref = O.apply_op("helmholtz", shape, P, P + 2, jac[idx], x64, lam=LAM)
        s = scale(shape, P, jac[idx], x64, "helmholtz", LAM)
        e = float(np.abs(y[idx].astype(np.float64) - ref).max() / s.max())
        say(f"    {prec} {e:.2e} of the scale")
        assert e <= bar, (shape, P, prec, e)


def test_fp64_localmat_mesh_launch_equals_blocks(shp):
    """The FP64 and FP32 affine local matrices over the whole mesh (one launch over
    every block of one order, each with its own tiles per wave) equal the
    per-block launches bit for bit, for the mass, Laplacian and Helmholtz;
    block sizes that are not multiples of the tile pair nor of the 4-wave
    work-group, and small enough that the per-block launches take one tile
    per wave."""
    say("[localmat] FP64 affine whole mesh == per block")
    sizes = (("hex", 4, 37), ("prism", 4, 17), ("pyr", 4, 33), ("tet", 4, 70))
    blocks = [(s, P, W.shape_batch(s, n)) for s, P, n in sizes]
    plan = affine_plan(shp, blocks)
    nc, _ = plan.totals()
    x = torch.from_numpy(W.coeffs(1, nc, 960)[0]).cuda()
    x32 = x.float()
    for op in ("mass", "laplacian", "helmholtz"):
        yw = plan.apply(-1, op, x, lam=LAM, strategy="localmat").cpu().numpy()
        yw32 = plan.apply_prec(op, x32, lam=LAM, prec="fp32", strategy="localmat").cpu().numpy()
        for b in range(len(sizes)):
            co, _ = plan.offsets(b)
            n = len(blocks[b][2]) * plan.n_modes[b]
            yb = plan.apply(b, op, x[co:co + n].contiguous(), lam=LAM, strategy="localmat").cpu().numpy()
            assert np.array_equal(yw[co:co + n], yb.ravel()), (op, sizes[b])
            yb32 = plan.apply_prec(op, x32[co:co + n].contiguous(), lam=LAM, prec="fp32", blk=b,
                                   strategy="localmat").cpu().numpy()
            assert np.array_equal(yw32[co:co + n], yb32.ravel()), ("fp32", op, sizes[b])


@pytest.mark.parametrize("orders", ["one", "mixed"])
def test_bf16_whole_mesh_equals_blocks(shp, orders):
    """blk = -1 over affine blocks of every shape equals the per-block launches
    bit for bit, in both split widths: one launch over all blocks when they
    share P (block sizes not multiples of the 4-wave work-group), one launch
    per block when the orders differ."""
    say(f"[bf16] whole mesh == per block ({orders} order)")
    sizes = (("hex", 2, 5), ("prism", 3, 17), ("pyr", 4, 33), ("tet", 1, 40), ("tet", 4, 21)) if orders == "mixed" \
        else (("hex", 4, 37), ("prism", 4, 17), ("pyr", 4, 33), ("tet", 4, 70))
    blocks = [(s, P, W.shape_batch(s, n)) for s, P, n in sizes]
    plan = affine_plan(shp, blocks)
    nc, _ = plan.totals()
    x = torch.from_numpy(W.coeffs(1, nc, 910)[0].astype(np.float32)).cuda()
    for prec in ("bf16", "bf16x3"):
        y = plan.apply_prec("helmholtz", x, lam=LAM, prec=prec).cpu().numpy()
        for b, (s, P, m) in enumerate(blocks):
            co, _ = plan.offsets(b)
            NP = plan.n_modes[b]
            yb = plan.apply_prec("helmholtz", x[co:co + len(m) * NP].contiguous(), lam=LAM, prec=prec, blk=b)
            assert np.array_equal(y[co:co + len(m) * NP], yb.cpu().numpy().ravel()), (prec, s, P)


def test_bf16_rejects(shp):
    """Curved blocks, P > 4 and other operators are refused."""
    say("[bf16] refusals")
    maps = W.shape_batch("hex", 4)
    plan = shp.Plan([("hex", 3, 4, "curved")])
    xi, _ = shp.quadrature("hex", 5)
    plan.set_geometry(0, torch.from_numpy(W.jacobian(maps, xi, curved=True)).cuda())
    x = torch.zeros(4 * 64, dtype=torch.float32, device="cuda")
    with pytest.raises(shp.ShpError) as ei:
        plan.apply_prec("helmholtz", x, prec="bf16")
    assert ei.value.code == -2
    plan5 = affine_plan(shp, [("hex", 5, maps)])
    with pytest.raises(shp.ShpError) as ei:
        plan5.apply_prec("helmholtz", torch.zeros(4 * 216, dtype=torch.float32, device="cuda"), prec="bf16")
    assert ei.value.code == -2
    with pytest.raises(shp.ShpError) as ei:
        plan5.solve(torch.ones(4 * 216, dtype=torch.float64, device="cuda"), inner="bf16")
    assert ei.value.code == -2


@pytest.fixture(scope="module")
def affine_problem(shp):
    """The 4^3-cell mixed mesh with affine elements at P = 4, the manufactured
    right-hand side and the oracle's Cholesky solution per element."""
    P = 4
    say("[bf16] building the affine 4^3 mixed mesh at P=4 and the oracle solution")
    mesh = W.quadrant_mesh(4)
    plan = affine_plan(shp, [(s, P, mesh[s]) for s in O.SHAPES])
    b, xref = {}, {}
    for s in O.SHAPES:
        jac = W.affine_jacobian(mesh[s])
        xi = O.reference_points(s, P + 2)
        f = (1.0 + 3 * np.pi ** 2) * W.manufactured_u(W.coords(mesh[s], xi, curved=False))
        b[s] = O.apply_op("iprod", s, P, P + 2, jac, f, lam=1.0)
        xref[s] = O.helmholtz_solve(s, P, P + 2, jac, b[s], lam=1.0)
    return mesh, plan, np.concatenate([b[s].ravel() for s in O.SHAPES]), xref


def test_fp32_auto_follows_plan_choice(shp, affine_problem):
    """The FP32 whole-mesh action with SHP_AUTO is the FP32 sum-factorisation
    by default and the FP32 local matrices once they are the plan's
    whole-mesh choice, bit for bit (what the FP32-inner solves call)."""
    mesh, plan, b, xref = affine_problem
    nc, _ = plan.totals()
    x = torch.from_numpy(W.coeffs(1, nc, 950)[0].astype(np.float32)).cuda()
    y_sf = plan.apply_prec("helmholtz", x, lam=LAM, prec="fp32", strategy="sumfac_coll").cpu().numpy()
    y_lm = plan.apply_prec("helmholtz", x, lam=LAM, prec="fp32", strategy="localmat").cpu().numpy()
    y_auto = plan.apply_prec("helmholtz", x, lam=LAM, prec="fp32", strategy="auto").cpu().numpy()
    assert np.array_equal(y_auto, y_sf)
    plan.set_auto_strategy(-1, "helmholtz", "localmat")
    try:
        y_auto = plan.apply_prec("helmholtz", x, lam=LAM, prec="fp32", strategy="auto").cpu().numpy()
    finally:
        plan.set_auto_strategy(-1, "helmholtz", "sumfac_coll")
    assert np.array_equal(y_auto, y_lm)
    assert not np.array_equal(y_lm, y_sf)


@pytest.mark.parametrize("inner", ["bf16", "bf16x3", "fp32", "fp64-localmat", "fp32-localmat"])
@pytest.mark.parametrize("target", [1e-6, 1e-10])
def test_bf16_solve_vs_oracle(shp, affine_problem, inner, target):
    """Jacobi-PCG with split-BF16 inner actions and FP64 reliable updates on
    the affine mesh reaches both error targets against the oracle's solution
    (max over elements of ||x_e - x*_e|| / ||x*_e||); the FP32
    sum-factorisation inner actions on the same problem for comparison; and
    the FP64 PCG and the FP32-inner PCG whose actions take the local matrices
    as the plan's whole-mesh choice."""
    mesh, plan, b, xref = affine_problem
    say(f"[bf16] solve inner={inner} target={target:g}")
    lm = inner.endswith("-localmat")
    if lm:
        plan.set_auto_strategy(-1, "helmholtz", "localmat")
    try:
        x, st = plan.solve(torch.from_numpy(b).cuda(), lam=1.0, inner=inner.split("-")[0], tol=RESID_TOL[target],
                           max_outer=80, max_inner=20000)
    finally:
        if lm:
            plan.set_auto_strategy(-1, "helmholtz", "sumfac_coll")
    x = x.cpu().numpy()
    worst = 0.0
    for bi, s in enumerate(O.SHAPES):
        co, _ = plan.offsets(bi)
        ne, NP = len(mesh[s]), plan.n_modes[bi]
        xs = x[co:co + ne * NP].reshape(ne, NP)
        err = float((np.linalg.norm(xs - xref[s], axis=1) / np.linalg.norm(xref[s], axis=1)).max())
        worst = max(worst, err)
    say(f"    outer {st['outer_iters']} inner {st['inner_iters']} residual {st['rel_residual']:.2e} error {worst:.2e}")
    assert st["converged"]
    assert worst <= target, worst
