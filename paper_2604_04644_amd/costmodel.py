"""MLP cost model that predicts the fastest strategy, trained on the GPU.

The network (libshp's shp_mlp_* kernels: forward, backward and Adam written in
HIP) maps a configuration -- shape one-hot, P, Q, log2 of the batch size, the
mapping type and a strategy one-hot -- to the standardised log launch time per
DOF.  The model's choice for a configuration is the strategy with the smallest
prediction; exhaustive tuning (Plan.tune) stays the fallback and the measure
of its regret.  Timings come from paper_2604_04644_amd.sweep.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
from collections import defaultdict

import numpy as np

from . import shp as _shp

SHAPES = ("hex", "prism", "pyr", "tet")
STRATS = ("localmat", "sumfac", "sumfac_coll")
NIN = 11
DATA = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "timings_mi355x.jsonl")


def load_rows(path: str = DATA):
    with open(path) as f:
        return [json.loads(l) for l in f if l.strip()]


def featurize(rows) -> np.ndarray:
    X = np.zeros((len(rows), NIN), dtype=np.float32)
    for i, r in enumerate(rows):
        X[i, SHAPES.index(r["shape"])] = 1.0
        X[i, 4] = r["P"] / 10.0
        X[i, 5] = r["Q"] / 12.0
        X[i, 6] = math.log2(r["n_elem"]) / 22.0
        X[i, 7] = float(r.get("curved", 1))
        X[i, 8 + STRATS.index(r["strategy"])] = 1.0
    return X


def log_time_per_dof(rows) -> np.ndarray:
    return np.array([math.log(r["ms"] * 1e-3 / r["dof"]) for r in rows])


def _fp(t):
    return ctypes.c_void_p(t.data_ptr())


def save_model(path: str, members, source: str = ""):
    """Write a cost model file that libshp loads (shp_plan_load_model): one
    JSON header line, then every member's FP32 parameters."""
    params = [m.params.detach().cpu().numpy().astype("<f4") for m in members]
    head = {"format": "shp-mlp", "version": 1, "nin": NIN, "nh": 64, "n_params": int(params[0].size),
            "members": len(params), "mu": members[0].mu, "sigma": members[0].sigma,
            "target": "standardised log(launch seconds per DOF)",
            "features": "shape one-hot(hex,prism,pyr,tet), P/10, Q/12, log2(n_elem)/22, curved, "
                        "strategy one-hot(localmat,sumfac,sumfac_coll)",
            "source": source}
    with open(path, "wb") as f:
        f.write((json.dumps(head) + "\n").encode())
        for q in params:
            f.write(q.tobytes())


class CostModel:
    """The network's parameters live in a torch float32 tensor on the GPU."""

    def __init__(self, seed: int = 0, device="cuda"):
        import torch
        self.torch = torch
        L = _shp.lib()
        self._bind(L)
        n = ctypes.c_int()
        _shp._check(L.shp_mlp_num_params(ctypes.byref(n)))
        self.nparam = n.value
        rng = np.random.default_rng(seed)
        p = np.zeros(self.nparam, dtype=np.float32)
        o = 0
        for (fan_out, fan_in) in ((64, 11), (64, 64), (1, 64)):
            p[o:o + fan_out * fan_in] = rng.normal(0, math.sqrt(2.0 / fan_in), fan_out * fan_in)
            o += fan_out * fan_in + fan_out
        self.params = torch.from_numpy(p).to(device)
        self.device = device
        self.mu, self.sigma = 0.0, 1.0
        self.history = []

    @staticmethod
    def _bind(L):
        if getattr(L, "_mlp_bound", False):
            return
        vp, i, f = ctypes.c_void_p, ctypes.c_int, ctypes.c_float
        L.shp_mlp_num_params.argtypes = [ctypes.POINTER(ctypes.c_int)]
        L.shp_mlp_work_floats.argtypes = [i, ctypes.POINTER(ctypes.c_longlong)]
        L.shp_mlp_forward.argtypes = [vp, vp, i, vp, vp, vp]
        L.shp_mlp_loss_grad.argtypes = [vp, vp, vp, i, vp, vp, vp, vp]
        L.shp_mlp_adam.argtypes = [vp, vp, vp, vp, i, f, f, f, f, vp]
        for name in ("shp_mlp_num_params", "shp_mlp_work_floats", "shp_mlp_forward", "shp_mlp_loss_grad",
                     "shp_mlp_adam"):
            getattr(L, name).restype = ctypes.c_int
        L._mlp_bound = True

    def _work(self, n):
        m = ctypes.c_longlong()
        _shp._check(_shp.lib().shp_mlp_work_floats(n, ctypes.byref(m)))
        return self.torch.empty(m.value, dtype=self.torch.float32, device=self.device)

    # --- raw kernels ------------------------------------------------------
    def forward_raw(self, X: np.ndarray, params=None) -> np.ndarray:
        t = self.torch
        p = self.params if params is None else params
        Xd = t.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(self.device)
        y = t.empty(X.shape[0], dtype=t.float32, device=self.device)
        _shp._check(_shp.lib().shp_mlp_forward(_fp(p), _fp(Xd), X.shape[0], _fp(y), _fp(self._work(X.shape[0])),
                                               _shp._stream(t)))
        return y.cpu().numpy()

    def loss_grad_raw(self, X: np.ndarray, target: np.ndarray, params=None):
        t = self.torch
        p = self.params if params is None else params
        Xd = t.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(self.device)
        Td = t.from_numpy(np.ascontiguousarray(target, dtype=np.float32)).to(self.device)
        g = t.empty(self.nparam, dtype=t.float32, device=self.device)
        loss = t.empty(1, dtype=t.float32, device=self.device)
        _shp._check(_shp.lib().shp_mlp_loss_grad(_fp(p), _fp(Xd), _fp(Td), X.shape[0], _fp(g), _fp(loss),
                                                 _fp(self._work(X.shape[0])), _shp._stream(t)))
        return float(loss.item()), g.cpu().numpy()

    # --- training and prediction -----------------------------------------
    def fit(self, rows, epochs: int = 3000, lr: float = 3e-3, log_every: int = 250):
        """Full-batch Adam on the standardised log time per DOF."""
        t = self.torch
        X = featurize(rows)
        y = log_time_per_dof(rows)
        self.mu, self.sigma = float(y.mean()), float(y.std() + 1e-12)
        target = ((y - self.mu) / self.sigma).astype(np.float32)
        n = X.shape[0]
        Xd = t.from_numpy(X).to(self.device)
        Td = t.from_numpy(target).to(self.device)
        g = t.empty(self.nparam, dtype=t.float32, device=self.device)
        m = t.zeros_like(g)
        v = t.zeros_like(g)
        loss = t.empty(1, dtype=t.float32, device=self.device)
        work = self._work(n)
        L = _shp.lib()
        s = _shp._stream(t)
        for step in range(1, epochs + 1):
            _shp._check(L.shp_mlp_loss_grad(_fp(self.params), _fp(Xd), _fp(Td), n, _fp(g), _fp(loss), _fp(work), s))
            _shp._check(L.shp_mlp_adam(_fp(self.params), _fp(g), _fp(m), _fp(v), step, lr, 0.9, 0.999, 1e-8, s))
            if step == 1 or step % log_every == 0:
                self.history.append((step, float(loss.item())))
        return self.history

    def predict_log_time(self, rows) -> np.ndarray:
        return self.forward_raw(featurize(rows)).astype(np.float64) * self.sigma + self.mu

    def choose(self, shape: str, P: int, n_elem: int, curved: int = 1, strategies=STRATS) -> str:
        cand = [{"shape": shape, "P": P, "Q": P + 2, "n_elem": n_elem, "curved": curved, "strategy": st}
                for st in strategies]
        pred = self.predict_log_time(cand)
        return cand[int(np.argmin(pred))]["strategy"]

    def save(self, path: str, source: str = ""):
        save_model(path, [self], source)


class CostEnsemble:
    """Several networks trained from different initial weights; the prediction
    is the mean of their log-time predictions, which damps the run-to-run
    variance of a single network's choice near strategy crossovers."""

    def __init__(self, seeds=(0, 1, 2), device="cuda"):
        self.members = [CostModel(seed=sd, device=device) for sd in seeds]

    def fit(self, rows, epochs: int = 3000, lr: float = 3e-3):
        return [m.fit(rows, epochs=epochs, lr=lr) for m in self.members]

    def predict_log_time(self, rows) -> np.ndarray:
        return np.mean([m.predict_log_time(rows) for m in self.members], axis=0)

    def choose(self, shape: str, P: int, n_elem: int, curved: int = 1, strategies=STRATS) -> str:
        cand = [{"shape": shape, "P": P, "Q": P + 2, "n_elem": n_elem, "curved": curved, "strategy": st}
                for st in strategies]
        return cand[int(np.argmin(self.predict_log_time(cand)))]["strategy"]

    def save(self, path: str, source: str = ""):
        save_model(path, self.members, source)


def group_configs(rows):
    g = defaultdict(dict)
    for r in rows:
        g[(r["shape"], r["P"], r["n_elem"], r.get("curved", 1))][r["strategy"]] = r
    return g


def regret(model, rows):
    """Per configuration: t(model's pick) / t(fastest measured) - 1, and the same
    for the fixed rule 'always sumfac_coll'."""
    out = []
    for (shape, P, ne, curved), byst in group_configs(rows).items():
        best = min(r["ms"] for r in byst.values())
        pick = model.choose(shape, P, ne, curved, strategies=tuple(byst))
        fixed = byst.get("sumfac_coll", min(byst.values(), key=lambda r: r["ms"]))
        out.append({"shape": shape, "P": P, "n_elem": ne, "curved": curved, "pick": pick, "best_ms": best,
                    "regret": byst[pick]["ms"] / best - 1.0, "fixed_regret": fixed["ms"] / best - 1.0})
    return out


def split_heldout(rows, held_P=(3, 7)):
    """Held-out (P, batch size) pairs: every configuration with P in held_P, and
    every other batch size of the remaining orders."""
    sizes = sorted({r["n_elem"] for r in rows})
    train, test = [], []
    by_shape_P = defaultdict(list)
    for r in rows:
        by_shape_P[(r["shape"], r["P"])].append(r)
    for (shape, P), rs in by_shape_P.items():
        ne_sorted = sorted({r["n_elem"] for r in rs})
        odd = set(ne_sorted[1::2])
        for r in rs:
            (test if (P in held_P or r["n_elem"] in odd) else train).append(r)
    return train, test


def main():
    """Train the ensemble on the committed timings and write a model file:
    python -m paper_2604_04644_amd.costmodel --out FILE [--seeds 0,1,2] [--epochs 3000]"""
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--seeds", default="0,1,2")
    ap.add_argument("--epochs", type=int, default=3000)
    ap.add_argument("--lr", type=float, default=3e-3)
    a = ap.parse_args()
    rows = load_rows()
    ens = CostEnsemble(seeds=tuple(int(v) for v in a.seeds.split(",")))
    hist = ens.fit(rows, epochs=a.epochs, lr=a.lr)
    ens.save(a.out, source=f"{os.path.basename(DATA)}: {len(rows)} rows; seeds {a.seeds}; {a.epochs} epochs of "
                           f"full-batch Adam, lr {a.lr}")
    print(json.dumps({"out": a.out, "rows": len(rows), "final_loss": [h[-1][1] for h in hist]}))


if __name__ == "__main__":
    main()
