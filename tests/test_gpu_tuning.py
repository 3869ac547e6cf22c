"""GPU tests of the autotuner: every accepted candidate passes the parity gate,
SHP_AUTO uses the choice, and the JSON-lines cache round-trips."""
import os

import numpy as np
import pytest

from oracle import shp_oracle as O
from paper_2604_04644_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def shp():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2604_04644_amd import shp as S
    S.lib()
    return S


def _plan(shp, shape, P, ne):
    maps = W.shape_batch(shape, ne)
    plan = shp.Plan([(shape, P, ne, "curved")])
    xi, _ = shp.quadrature(shape, P + 2)
    plan.set_geometry(0, torch.from_numpy(W.jacobian(maps, xi, curved=True)).cuda())
    return maps, plan


@pytest.mark.parametrize("shape,P", [("hex", 3), ("tet", 4)])
def test_tune_block(shp, shape, P, tmp_path):
    print(f"[tune] block shape={shape} P={P}", flush=True)
    maps, plan = _plan(shp, shape, P, 700)
    x = torch.from_numpy(W.coeffs(700, plan.n_modes[0], 3)).cuda()
    res, recs = plan.tune(0, "helmholtz", x, reps=5, quick=True)
    assert res["n_candidates"] == len(recs) > 4
    assert res["n_rejected"] == 0
    assert {r["strategy"] for r in recs} == {"sumfac", "sumfac_coll", "localmat"}
    assert res["ms"] == pytest.approx(min(r["ms"] for r in recs if r["passed"]))
    # AUTO applies the tuned choice, bit for bit
    y_auto = plan.apply(0, "helmholtz", x, strategy="auto").cpu().numpy()
    y_pick = plan.apply(0, "helmholtz", x, strategy=res["strategy"]).cpu().numpy()
    assert np.array_equal(y_auto, y_pick)
    ref = O.apply_op("helmholtz", shape, P, P + 2,
                     W.jacobian(maps, O.reference_points(shape, P + 2), curved=True), x.cpu().numpy())
    assert np.abs(y_auto - ref).max() <= 1e-12 * np.abs(ref).max()
    # cache round trip into a fresh plan
    path = str(tmp_path / "tune.jsonl")
    plan.save_tuning(path)
    _, plan2 = _plan(shp, shape, P, 700)
    assert plan2.load_tuning(path) == 1
    assert plan2.get_tiling(0, "helmholtz", res["strategy"]) == (res["elems_per_wg"], res["threads"], res["variant"])


def test_tune_whole_mesh_and_corrupt_cache(shp, tmp_path):
    print("[tune] whole mesh", flush=True)
    mesh = W.quadrant_mesh(8)
    P = 3
    plan = shp.Plan([(s, P, len(mesh[s]), "curved") for s in O.SHAPES])
    for b, s in enumerate(O.SHAPES):
        xi, _ = shp.quadrature(s, P + 2)
        plan.set_geometry(b, torch.from_numpy(W.jacobian(mesh[s], xi, curved=True)).cuda())
    nc, _ = plan.totals()
    x = torch.from_numpy(W.coeffs(1, nc, 8)[0]).cuda()
    res, recs = plan.tune(-1, "helmholtz", x, reps=3, quick=True)
    assert res["n_rejected"] == 0 and len(recs) > 4
    path = str(tmp_path / "c.jsonl")
    with open(path, "w") as f:
        f.write("not json\n{\"kind\":\"block\",\"device\":\"x\"}\n")
        f.write('{"kind":"mixed","device":"zz","prec":"fp64","op":6,"blocks":"bad","strategy":2,"E":999,"NT":7,"variant":9}\n')
    plan.save_tuning(path)
    assert plan.load_tuning(path) == 1       # only the valid mixed entry applies
