"""Order/strategy sweep: tune the Helmholtz action for every shape, order P and
batch size and record the best launch time of each strategy.

Each configuration is one block of ``n_elem`` curved or affine elements of one shape
(``n_elem`` chosen so the batch holds about 2^k DOF), tuned by libshp's
exhaustive tuner (quick candidate set); for each strategy the fastest accepted
candidate is one dataset row.  Rows are JSON lines:

    {"shape", "P", "Q", "n_elem", "dof", "curved", "strategy", "ms", "gdofs",
     "elems_per_wg", "threads", "variant"}

    python -m paper_2604_04644_amd.sweep --out timings.jsonl [--P 1-10] [--kmin 14 --kmax 22] [--geom curved|affine]
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

SHAPES = ("hex", "prism", "pyr", "tet")


def _range(spec: str):
    if "-" in spec:
        a, b = spec.split("-")
        return list(range(int(a), int(b) + 1))
    return [int(v) for v in spec.split(",")]


def sweep(out_path: str, Ps, ks, shapes=SHAPES, reps: int = 5, seed: int = 1000, log=print, geom: str = "curved"):
    import torch

    from . import shp, workloads as W
    dev = torch.device("cuda")
    rows = 0
    t0 = time.time()
    with open(out_path, "a") as f:
        for shape in shapes:
            for P in Ps:
                npm = shp.num_modes(shape, P)
                xi, _ = shp.quadrature(shape, P + 2)
                for k in ks:
                    ne = max(1, int(round(2.0 ** k / npm)))
                    maps = W.shape_batch(shape, ne)
                    plan = shp.Plan([(shape, P, ne, geom)])
                    if geom == "curved":
                        plan.set_geometry(0, W.jacobian_torch(maps, xi, True, dev))
                    else:
                        plan.set_geometry(0, torch.from_numpy(W.affine_jacobian(maps)).to(dev))
                    x = torch.from_numpy(W.coeffs(ne, npm, seed + P)).to(dev)
                    _, recs = plan.tune(0, "helmholtz", x, reps=reps, quick=True)
                    best = {}
                    for r in recs:
                        if r["passed"] and (r["strategy"] not in best or r["ms"] < best[r["strategy"]]["ms"]):
                            best[r["strategy"]] = r
                    for st, r in best.items():
                        row = {"shape": shape, "P": P, "Q": P + 2, "n_elem": ne, "dof": ne * npm, "curved": int(geom == "curved"),
                               "strategy": st, "ms": r["ms"], "gdofs": ne * npm / (r["ms"] * 1e-3) / 1e9,
                               "elems_per_wg": r["elems_per_wg"], "threads": r["threads"], "variant": r["variant"]}
                        f.write(json.dumps(row) + "\n")
                        rows += 1
                    f.flush()
                    del plan, x
                log(f"sweep {geom} {shape} P={P}: {rows} rows, {time.time() - t0:.0f} s")
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--P", default="1-10")
    ap.add_argument("--kmin", type=float, default=14)
    ap.add_argument("--kmax", type=float, default=22)
    ap.add_argument("--nk", type=int, default=12)
    ap.add_argument("--shapes", default=",".join(SHAPES))
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--geom", choices=("curved", "affine"), default="curved")
    a = ap.parse_args()
    ks = list(np.linspace(a.kmin, a.kmax, a.nk))
    n = sweep(a.out, _range(a.P), ks, shapes=a.shapes.split(","), reps=a.reps,
              log=lambda m: print(m, file=sys.stderr, flush=True), geom=a.geom)
    print(json.dumps({"rows": n, "out": a.out}))


if __name__ == "__main__":
    main()
