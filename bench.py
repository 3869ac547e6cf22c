"""Benchmark: FP64 Helmholtz action y = (lambda M + L) x on the mixed-element
mesh (32^3 cells of the unit cube split by quadrant into 8192 hexes, 16384
prisms, 49152 pyramids and 49152 tets; curved by the sine perturbation; P = 4,
Q = 6; lambda = 1), one whole-mesh launch per step, inputs resident in HBM.

Prints one JSON line.  value = elemental DOFs per second (GDOF/s) of the
whole-mesh action; roofline = algorithmic HBM bytes of the launch (16 N_P + 56
N_Q bytes per element: x, y and 7 FP64 geometric factors per point) over the
launch's mean duration from HIP events on the launch stream, against the 8 TB/s
HBM3E peak; cpu_baseline = the FP64 oracle (dense elemental matrices) on a
bounded sample of the same mesh; mixed_vs_fp64 = the mixed-precision leg on the
same mesh at P = 6 (FP32 vs FP64 action, and the Helmholtz solve by FP32
Jacobi-PCG with FP64 reliable updates vs plain FP64 PCG at the residual
tolerances of the 1e-6 and 1e-10 error targets); per_shape_and_order = each
shape's block and the whole mesh at P = 2, 4, 6, 8, 10; further legs: the
advection-diffusion-reaction action, iso-parametric against precomputed
geometry, and a 2D quadrilateral/triangle mesh.  Every timed launch follows a
1 GiB write that flushes the 256 MiB Infinity Cache.

    python bench.py [--gpus 1] [--steps 50] [--warmup 5] [--no-cpu] [--no-mixed]
                    [--no-adr] [--no-iso] [--no-2d] [--no-per-shape] [--orders 2,4,...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Helmholtz action GDOF/s per shape & P, % of HBM roofline; mixed-vs-FP64 speedup at stated err"
SHAPES = ("hex", "prism", "pyr", "tet")
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def bytes_per_elem(n_modes: int, n_points: int) -> int:
    return 16 * n_modes + 56 * n_points


KERNEL_SOURCES = ("shp_kernels.hpp", "shp_layout.hpp", "shp_k_mixed_p.inc", "shp_k_mixed_p4.hip")


def kernel_source_hash() -> str:
    """sha256[:16] of the sources that define the benchmarked whole-mesh
    Helmholtz kernel at P = 4 (names and contents)."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_2604_04644_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(P: int, ncell: int):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, when it was taken on the current kernel sources; else None."""
    import re
    if (P, ncell) != (4, 32):
        return None
    path = os.path.join(ROOT, "profiles", "helmholtz_mixed_P4_hbm_traffic.md")
    try:
        txt = open(path).read()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch:\s*(\d+)", txt)
    h = re.search(r"source_sha256_16:\s*([0-9a-f]+)", txt)
    if not m or not h or h.group(1) != kernel_source_hash():
        return None
    return int(m.group(1))


def build_mesh_plan(torch, shp, W, ncell: int, P: int):
    mesh = W.quadrant_mesh(ncell)
    blocks = [(s, P, len(mesh[s]), "curved") for s in SHAPES]
    plan = shp.Plan(blocks)
    for b, s in enumerate(SHAPES):
        xi, _ = shp.quadrature(s, P + 2)
        jac = torch.from_numpy(W.jacobian(mesh[s], xi, curved=True)).cuda()
        plan.set_geometry(b, jac)
        del jac
        log(f"  geometry {s}: {len(mesh[s])} elements")
    return mesh, plan


def time_launches(torch, fn, steps: int, warmup: int, flush=None):
    """Wall time of `steps` launches, and the mean and median of their HIP-event
    durations on the current stream.  With flush (a device tensor of at least
    1 GiB) every launch is preceded, outside its events, by a write of that
    buffer, which evicts the 256 MiB Infinity Cache (MALL)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        if flush is not None:
            flush.fill_(i & 0xff)
        starts[i].record()
        fn()
        ends[i].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    return wall, float(np.mean(ev)), float(np.median(ev))


def flush_buffer(torch):
    """1 GiB device buffer whose write evicts the 256 MiB Infinity Cache."""
    return torch.empty(1 << 30, dtype=torch.uint8, device="cuda")


def copy_bandwidth(torch, flush, reps: int = 10):
    """Device-to-device copy of 1 GiB (1 GiB read + 1 GiB written) timed with
    HIP events after a cache flush: the rate a plain streaming kernel reaches."""
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    _, _, med = time_launches(torch, lambda: dst.copy_(src), reps, 2, flush=flush)
    del src, dst
    return 2.0 * (1 << 30) / (med * 1e-3) / 1e9


def flops_per_elem(shape: str, P: int) -> int:
    """Algorithmic FP64 flops of one collocated Helmholtz element action:
    2 [2 BT + 6 Q^4 + 11 Q^3] with BT the multiply-adds of one sum-factorised
    BwdTrans (the three line stages) and 6 Q^4 those of the three collocated
    derivatives and their transposes, 11 Q^3 the metric and the reaction term."""
    Q, n = P + 2, P + 1
    NP = {"hex": n ** 3, "prism": n * n * (P + 2) // 2, "pyr": (P + 1) * (P + 2) * (2 * P + 3) // 6,
          "tet": (P + 1) * (P + 2) * (P + 3) // 6}[shape]
    if shape == "hex":
        bt = n ** 3 * Q + n * n * Q * Q + n * Q ** 3
    elif shape == "tet":
        bt = NP * Q + (P + 1) * (P + 2) // 2 * Q * Q + n * Q ** 3
    else:
        bt = NP * Q + n * n * Q * Q + n * Q ** 3
    return 2 * (2 * bt + 6 * Q ** 4 + 11 * Q ** 3)


FP64_PEAK_TFS = 78.6
BF16_PEAK_TFS = 2500.0   # dense BF16 MFMA


def order_table(torch, shp, W, flush, ncell: int = 32, Ps=(2, 4, 6, 8, 10), steps: int = 20):
    """Per shape and order on the mixed mesh: each block's FP64 Helmholtz launch
    (collocated, default launch shape) and the whole-mesh launch, timed with
    HIP events after a cache flush (median of `steps`): GDOF/s, fraction of the
    8 TB/s HBM peak for the algorithmic bytes and of the 78.6 TF FP64 peak for
    the algorithmic flops."""
    out = {}
    dev = torch.device("cuda")
    mesh = W.quadrant_mesh(ncell)
    for P in Ps:
        plan = shp.Plan([(s, P, len(mesh[s]), "curved") for s in SHAPES])
        for b, s in enumerate(SHAPES):
            plan.set_geometry(b, W.jacobian_torch(mesh[s], shp.quadrature(s, P + 2)[0], True, dev))
        nc, _ = plan.totals()
        x = torch.from_numpy(np.concatenate([W.coeffs(len(mesh[s]), plan.n_modes[b], W.SEED_MIXED[s]).ravel()
                                             for b, s in enumerate(SHAPES)])).cuda()
        y = torch.empty_like(x)
        row = {}
        tot_b = tot_f = 0
        for b, s in enumerate(SHAPES):
            co, _ = plan.offsets(b)
            ne, nm = len(mesh[s]), plan.n_modes[b]
            xb = x[co:co + ne * nm].view(ne, nm)
            yb = y[co:co + ne * nm].view(ne, nm)
            _, _, med = time_launches(torch, lambda: plan.apply(b, "helmholtz", xb, out=yb), steps, 3, flush=flush)
            nb = ne * bytes_per_elem(nm, plan.n_points[b])
            nf = ne * flops_per_elem(s, P)
            tot_b += nb
            tot_f += nf
            row[s] = {"n_elem": ne, "ms": round(med, 5), "GDOF/s": round(ne * nm / (med * 1e-3) / 1e9, 3),
                      "hbm_frac": round(nb / (med * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                      "fp64_frac": round(nf / (med * 1e-3) / 1e12 / FP64_PEAK_TFS, 4)}
        _, _, med = time_launches(torch, lambda: plan.apply(-1, "helmholtz", x, out=y), steps, 3, flush=flush)
        row["whole_mesh"] = {"n_elem": int(sum(len(mesh[s]) for s in SHAPES)), "ms": round(med, 5),
                             "GDOF/s": round(nc / (med * 1e-3) / 1e9, 3),
                             "hbm_frac": round(tot_b / (med * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                             "fp64_frac": round(tot_f / (med * 1e-3) / 1e12 / FP64_PEAK_TFS, 4)}
        out[f"P{P}"] = row
        log(f"  P={P}: " + ", ".join(f"{k} {v['GDOF/s']} GDOF/s ({v['hbm_frac']:.2f} HBM)" for k, v in row.items()))
        del plan, x, y
        torch.cuda.empty_cache()
    return out


def mixed_precision_leg(torch, shp, W, ncell: int = 32, P: int = 6, lam: float = 1.0):
    """Mixed precision on the mixed mesh at P = 6: the Helmholtz action with FP32
    contractions against FP64, and the Helmholtz solve with a manufactured
    right-hand side (u = sin(pi x) sin(pi y) sin(pi z), b = IProduct((lambda +
    3 pi^2) u)) by an FP32 Jacobi-PCG with FP64 reliable updates (residual
    replacement and solution update in FP64) against the same iteration run in
    FP64, to the same FP64 relative residual."""
    log(f"mixed precision: mesh ncell={ncell} P={P}")
    mesh = W.quadrant_mesh(ncell)
    dev = torch.device("cuda")
    plan = shp.Plan([(s, P, len(mesh[s]), "curved") for s in SHAPES])
    for b, s in enumerate(SHAPES):
        plan.set_geometry(b, W.jacobian_torch(mesh[s], shp.quadrature(s, P + 2)[0], True, dev))
    nc, _ = plan.totals()
    x64 = torch.from_numpy(np.concatenate([W.coeffs(len(mesh[s]), plan.n_modes[b], W.SEED_MIXED[s]).ravel()
                                           for b, s in enumerate(SHAPES)])).cuda()
    x32 = x64.float()
    y64, y32 = torch.empty_like(x64), torch.empty_like(x32)
    _, t64, _ = time_launches(torch, lambda: plan.apply(-1, "helmholtz", x64, out=y64, lam=lam), 20, 3)
    _, t32, _ = time_launches(torch, lambda: plan.apply_prec("helmholtz", x32, out=y32, lam=lam, prec="fp32"), 20, 3)
    dev32 = float((y32.double() - y64).abs().max() / y64.abs().max())
    # the same FP32 action reading an FP32 copy of the geometric factors
    plan.set_fp32_factors(True)
    _, t32f, _ = time_launches(torch, lambda: plan.apply_prec("helmholtz", x32, out=y32, lam=lam, prec="fp32"), 20, 3)
    dev32f = float((y32.double() - y64).abs().max() / y64.abs().max())
    plan.set_fp32_factors(False)
    action = {"fp64_ms": round(t64, 5), "fp32_ms": round(t32, 5), "fp64_GDOF/s": round(nc / t64 / 1e6, 3),
              "fp32_GDOF/s": round(nc / t32 / 1e6, 3), "speedup": round(t64 / t32, 3),
              "fp32_vs_fp64_maxrel": dev32,
              "fp32_fac32_ms": round(t32f, 5), "fp32_fac32_GDOF/s": round(nc / t32f / 1e6, 3),
              "fac32_speedup": round(t64 / t32f, 3), "fp32_fac32_vs_fp64_maxrel": dev32f}
    log(f"  action: {action}")
    del x32, y32, y64
    f = torch.cat([W.manufactured_u_torch(mesh[s], shp.quadrature(s, P + 2)[0], dev).reshape(-1)
                   for s in SHAPES]) * (lam + 3 * np.pi ** 2)
    b = plan.apply(-1, "iprod", f)
    del f
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.helmholtz_diag(lam)
    torch.cuda.synchronize()
    t_diag = time.perf_counter() - t0
    solves = {}
    # residual tolerances for the error targets 1e-6 and 1e-10 against the
    # oracle on this mesh (the FP64 action's relative residual floor here is
    # about 9e-12; at a residual of 2e-11 the sampled error is below 3e-11)
    for target, tol in ((1e-6, 1e-9), (1e-10, 2e-11)):
        row = {}
        sols = {}
        for name, kw in (("fp64", dict(inner="fp64", max_outer=100, max_inner=30000)),
                         ("mixed", dict(inner="fp32", max_outer=100, max_inner=30000)),
                         ("mixed_fac32", dict(inner="fp32", max_outer=100, max_inner=30000))):
            if name == "mixed_fac32":
                plan.set_fp32_factors(True)   # (set-up outside the timed solve)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xs, st = plan.solve(b, lam=lam, tol=tol, check=False, **kw)
            torch.cuda.synchronize()
            st["s"] = round(time.perf_counter() - t0, 4)
            if name == "mixed_fac32":
                plan.set_fp32_factors(False)
            row[name] = st
            sols[name] = xs
            log(f"  solve tol={tol:g} {name}: {st}")
        row["speedup"] = round(row["fp64"]["s"] / row["mixed"]["s"], 3)
        row["speedup_fac32"] = round(row["fp64"]["s"] / row["mixed_fac32"]["s"], 3)
        row["mixed_vs_fp64_rel2"] = float((sols["mixed"] - sols["fp64"]).norm() / sols["fp64"].norm())
        row["mixed_fac32_vs_fp64_rel2"] = float((sols["mixed_fac32"] - sols["fp64"]).norm() / sols["fp64"].norm())
        row["resid_tol"] = tol
        solves[f"err_target_{target:g}"] = row
    return {"workload": f"mixed-element mesh {ncell}^3 cells, curved, P={P}, Q={P + 2}, lambda={lam}",
            "dof": int(nc), "action": action, "diag_setup_s": round(t_diag, 4), "solve": solves,
            "note": "solve: Jacobi-PCG in FP32 (mixed) or FP64 (plain), FP64 residual replacement and solution "
                    "update every decade of residual reduction; mixed_fac32: the FP32 iterations read an FP32 "
                    "copy of the geometric factors; wall time per solve including host checks; error against "
                    "the FP64 oracle is asserted by the test suite"}


def affine_leg(torch, shp, W, flush=None, dof: float = 4e6, Ps=(1, 2, 3, 4)):
    """Affine single-shape blocks of about 4M DOF (as in the per-shape order sweep): the FP64
    Helmholtz action with the local-matrix strategy (7 reference matrices on
    FP64 MFMA, 7 coefficients per element) against the collocated
    sum-factorisation (per-point factors), and the local matrices in split
    BF16 (three and two parts, FP32 vectors); GDOF/s from the median of 20
    launches, each after a cache flush (these batches fit in the 256 MiB
    Infinity Cache)."""
    out = {}
    for s in SHAPES:
        for P in Ps:
            nm = shp.num_modes(s, P)
            ne = max(1, int(round(dof / nm)))
            maps = W.shape_batch(s, ne)
            plan = shp.Plan([(s, P, ne, "affine")])
            plan.set_geometry(0, torch.from_numpy(W.affine_jacobian(maps)).cuda())
            x = torch.from_numpy(W.coeffs(ne, nm, W.seed_sweep(P))).cuda()
            y = torch.empty_like(x)
            x32, y32 = x.float(), torch.empty(x.shape, dtype=torch.float32, device=x.device)
            row = {"n_elem": ne}
            for st in ("localmat", "sumfac_coll"):
                _, _, med = time_launches(torch, lambda: plan.apply(0, "helmholtz", x, out=y, strategy=st), 20, 3,
                                          flush=flush)
                row[st] = round(ne * nm / (med * 1e-3) / 1e9, 2)
            row["localmat_speedup"] = round(row["localmat"] / row["sumfac_coll"], 3)
            _, _, med = time_launches(torch, lambda: plan.apply_prec("helmholtz", x32, out=y32, prec="fp32", blk=0,
                                                                     strategy="localmat"), 20, 3, flush=flush)
            row["localmat_fp32"] = round(ne * nm / (med * 1e-3) / 1e9, 2)
            for pr in ("bf16", "bf16x3"):
                _, _, med = time_launches(torch, lambda: plan.apply_prec("helmholtz", x32, out=y32, prec=pr, blk=0),
                                          20, 3, flush=flush)
                row[f"localmat_{pr}"] = round(ne * nm / (med * 1e-3) / 1e9, 2)
                ex = (ne + 15) // 16 * bf16_mfma_flops(s, P, 3 if pr == "bf16" else 2)
                row[f"localmat_{pr}_mfma_frac"] = round(ex / (med * 1e-3) / 1e12 / BF16_PEAK_TFS, 4)
            out[f"{s}_P{P}"] = row
            log(f"  affine {s} P={P}: {row}")
            del plan, x, y, x32, y32
    return out


def bf16_mfma_flops(shape: str, P: int, nparts: int) -> int:
    """Executed BF16 MFMA flops per 16 elements of the split-BF16 affine
    Helmholtz action: K = 7 N_P (N_P padded to 8) in steps of 32, output rows
    in blocks of 16, nparts (nparts + 1) / 2 part products, 2 16 16 32 flops
    per v_mfma_f32_16x16x32_bf16."""
    nm = {"hex": (P + 1) ** 3, "prism": (P + 1) ** 2 * (P + 2) // 2, "pyr": (P + 1) * (P + 2) * (2 * P + 3) // 6,
          "tet": (P + 1) * (P + 2) * (P + 3) // 6}[shape]
    npp = (nm + 7) // 8 * 8
    ks, mb = (7 * npp + 31) // 32, (nm + 15) // 16
    return ks * mb * (nparts * (nparts + 1) // 2) * 2 * 16 * 16 * 32


def bf16_leg(torch, shp, W, flush, ncell: int = 32, P: int = 4, lam: float = 1.0, steps: int = 20):
    """Split-BF16 MFMA contractions on the mixed mesh made affine (each element
    its affine map, no curvature), P = 4: the Helmholtz action as FP64
    collocated sum-factorisation, FP64 local matrices (FP64 MFMA), FP32
    collocated sum-factorisation, FP32 local matrices on the FP32 matrix
    cores, and split-BF16 local matrices with three
    parts (six products, "bf16") and two parts (three products, "bf16x3"),
    HIP-event medians after a cache flush; then the Jacobi-PCG with FP64
    reliable updates to the error targets 1e-6 and 1e-10 with each inner
    precision (wall time per solve)."""
    log(f"bf16: affine mesh ncell={ncell} P={P}")
    mesh = W.quadrant_mesh(ncell)
    plan = shp.Plan([(s, P, len(mesh[s]), "affine") for s in SHAPES])
    for b, s in enumerate(SHAPES):
        plan.set_geometry(b, torch.from_numpy(np.ascontiguousarray(W.affine_jacobian(mesh[s]))).cuda())
    nc, _ = plan.totals()
    x64 = torch.from_numpy(np.concatenate([W.coeffs(len(mesh[s]), plan.n_modes[b], W.SEED_MIXED[s]).ravel()
                                           for b, s in enumerate(SHAPES)])).cuda()
    x32 = x64.float()
    y64, y32 = torch.empty_like(x64), torch.empty_like(x32)
    nel = sum(len(mesh[s]) for s in SHAPES)
    useful = sum(len(mesh[s]) * 14 * plan.n_modes[b] ** 2 for b, s in enumerate(SHAPES))
    action = {}
    ref = plan.apply(-1, "helmholtz", x64, lam=lam, strategy="sumfac_coll")
    for name, fn, out in (
            ("fp64_sumfac", lambda: plan.apply(-1, "helmholtz", x64, out=y64, lam=lam, strategy="sumfac_coll"), y64),
            ("fp64_localmat", lambda: plan.apply(-1, "helmholtz", x64, out=y64, lam=lam, strategy="localmat"), y64),
            ("fp32_sumfac", lambda: plan.apply_prec("helmholtz", x32, out=y32, lam=lam, prec="fp32"), y32),
            ("fp32_localmat", lambda: plan.apply_prec("helmholtz", x32, out=y32, lam=lam, prec="fp32",
                                                      strategy="localmat"), y32),
            ("bf16", lambda: plan.apply_prec("helmholtz", x32, out=y32, lam=lam, prec="bf16"), y32),
            ("bf16x3", lambda: plan.apply_prec("helmholtz", x32, out=y32, lam=lam, prec="bf16x3"), y32)):
        _, _, med = time_launches(torch, fn, steps, 3, flush=flush)
        dev = float((out.double() - ref).abs().max() / ref.abs().max())
        row = {"ms": round(med, 5), "GDOF/s": round(nc / (med * 1e-3) / 1e9, 3), "maxrel_vs_fp64": dev}
        if name.startswith("bf16") or name.endswith("_localmat"):
            row["useful_TFLOP/s"] = round(useful / (med * 1e-3) / 1e12, 2)
        if name.startswith("bf16"):
            parts = 3 if name == "bf16" else 2
            ex = sum((len(mesh[s]) + 15) // 16 * bf16_mfma_flops(s, P, parts) for s in SHAPES)
            row["mfma_TFLOP/s"] = round(ex / (med * 1e-3) / 1e12, 1)
            row["mfma_frac"] = round(ex / (med * 1e-3) / 1e12 / BF16_PEAK_TFS, 4)
            row["hbm_frac"] = round((nc * 8 + nel * 56) / (med * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        action[name] = row
        log(f"  action {name}: {row}")
    del x32, y32, y64, ref
    f = torch.cat([W.manufactured_u_torch(mesh[s], shp.quadrature(s, P + 2)[0], torch.device("cuda"),
                                          amp=0.0).reshape(-1) for s in SHAPES]) * (lam + 3 * np.pi ** 2)
    b = plan.apply(-1, "iprod", f)
    del f
    plan.helmholtz_diag(lam)
    solves = {}
    for target, tol in ((1e-6, 1e-9), (1e-10, 2e-11)):
        row = {}
        sols = {}
        for inner in ("fp64", "fp32", "bf16", "bf16x3"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xs, st = plan.solve(b, lam=lam, tol=tol, check=False, inner=inner, max_outer=100, max_inner=30000)
            torch.cuda.synchronize()
            st["s"] = round(time.perf_counter() - t0, 4)
            row[inner] = st
            sols[inner] = xs
            log(f"  solve tol={tol:g} {inner}: {st}")
        # the FP64 and FP32-inner solves with the local matrices as the plan's
        # whole-mesh choice
        plan.set_auto_strategy(-1, "helmholtz", "localmat")
        for inner in ("fp64", "fp32"):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            xs, st = plan.solve(b, lam=lam, tol=tol, check=False, inner=inner, max_outer=100, max_inner=30000)
            torch.cuda.synchronize()
            st["s"] = round(time.perf_counter() - t0, 4)
            row[f"{inner}_localmat"] = st
            sols[f"{inner}_localmat"] = xs
            log(f"  solve tol={tol:g} {inner} with local matrices: {st}")
        plan.set_auto_strategy(-1, "helmholtz", "sumfac_coll")
        for inner in ("fp32", "bf16", "bf16x3", "fp64_localmat", "fp32_localmat"):
            row[f"speedup_{inner}"] = round(row["fp64"]["s"] / row[inner]["s"], 3)
            row[f"{inner}_vs_fp64_rel2"] = float((sols[inner] - sols["fp64"]).norm() / sols["fp64"].norm())
        row["resid_tol"] = tol
        solves[f"err_target_{target:g}"] = row
    del plan, x64, b
    return {"workload": f"mixed-element mesh {ncell}^3 cells, affine, P={P}, Q={P + 2}, lambda={lam}",
            "dof": int(nc), "action": action, "solve": solves,
            "note": "useful flops 14 N_P^2 per element (7 matrix-vector products); mfma flops as executed "
                    "(padding and part products included) against the dense BF16 peak; hbm_frac from 8 N_P + 56 "
                    "bytes per element (FP32 x and y, FP64 coefficients); solve wall time per solve"}


def iso_flops_per_elem(shape: str, P: int) -> int:
    """Algorithmic FP64 flops of the iso-parametric Helmholtz element action:
    the collocated action, plus per coordinate the sum-factorised BwdTrans and
    the three collocated derivatives (BT + 3 Q^4 multiply-adds), plus about 85
    flops per point for the determinant, the inverse and the metric."""
    Q, n = P + 2, P + 1
    NP = {"hex": n ** 3, "prism": n * n * (P + 2) // 2, "pyr": (P + 1) * (P + 2) * (2 * P + 3) // 6,
          "tet": (P + 1) * (P + 2) * (P + 3) // 6}[shape]
    if shape == "hex":
        bt = n ** 3 * Q + n * n * Q * Q + n * Q ** 3
    elif shape == "tet":
        bt = NP * Q + (P + 1) * (P + 2) // 2 * Q * Q + n * Q ** 3
    else:
        bt = NP * Q + n * n * Q * Q + n * Q ** 3
    return flops_per_elem(shape, P) + 2 * 3 * (bt + 3 * Q ** 4) + 85 * Q ** 3


def iso_leg(torch, shp, W, flush, ncell: int = 32, Ps=(4, 6), steps: int = 20):
    """The mixed mesh made iso-parametric (each element's map a polynomial of
    degree P in its own basis: the curved mesh's vertex positions on the vertex
    modes, seeded perturbations of 2 % of the element size on the others),
    FP64 Helmholtz action with the geometry rebuilt in the launch (40 N_P bytes
    per element: x, y and 3 coordinate coefficients per mode), against the
    action that streams the 7 precomputed factors per point of the curved mesh
    (16 N_P + 56 Q^3 bytes per element).  HIP events after a cache flush,
    median of `steps`."""
    out = {}
    mesh = W.quadrant_mesh(ncell)
    dev = torch.device("cuda")
    for P in Ps:
        row = {}
        iso = shp.Plan([(s, P, len(mesh[s]), "isoparam") for s in SHAPES])
        for b, s in enumerate(SHAPES):
            idx, vxi = shp.vertex_modes(s, P)
            X = W.iso_coords(mesh[s], idx, vxi, iso.n_modes[b], 40 + b)
            iso.set_geometry(b, torch.from_numpy(X).to(dev))
            del X
        nc, _ = iso.totals()
        x = torch.from_numpy(np.concatenate([W.coeffs(len(mesh[s]), iso.n_modes[b], W.SEED_MIXED[s]).ravel()
                                             for b, s in enumerate(SHAPES)])).to(dev)
        y = torch.empty_like(x)
        _, _, t_iso = time_launches(torch, lambda: iso.apply(-1, "helmholtz", x, out=y), steps, 3, flush=flush)
        del iso
        torch.cuda.empty_cache()
        pre = shp.Plan([(s, P, len(mesh[s]), "curved") for s in SHAPES])
        for b, s in enumerate(SHAPES):
            pre.set_geometry(b, W.jacobian_torch(mesh[s], shp.quadrature(s, P + 2)[0], True, dev))
        _, _, t_pre = time_launches(torch, lambda: pre.apply(-1, "helmholtz", x, out=y), steps, 3, flush=flush)
        del pre
        torch.cuda.empty_cache()
        nm = {s: shp.num_modes(s, P) for s in SHAPES}
        b_iso = sum(len(mesh[s]) * 40 * nm[s] for s in SHAPES)
        b_pre = sum(len(mesh[s]) * bytes_per_elem(nm[s], (P + 2) ** 3) for s in SHAPES)
        f_iso = sum(len(mesh[s]) * iso_flops_per_elem(s, P) for s in SHAPES)
        row = {"dof": int(nc), "iso_ms": round(t_iso, 5), "precomputed_ms": round(t_pre, 5),
               "iso_GDOF/s": round(nc / (t_iso * 1e-3) / 1e9, 3), "precomputed_GDOF/s": round(nc / (t_pre * 1e-3) / 1e9, 3),
               "iso_vs_precomputed": round(t_pre / t_iso, 3),
               "iso_bytes": int(b_iso), "precomputed_bytes": int(b_pre),
               "iso_hbm_frac": round(b_iso / (t_iso * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
               "iso_flops": int(f_iso), "iso_fp64_frac": round(f_iso / (t_iso * 1e-3) / 1e12 / FP64_PEAK_TFS, 4)}
        out[f"P{P}"] = row
        log(f"  iso-parametric P={P}: {row}")
        del x, y
    return out


def leg_2d(torch, shp, W, flush, cases=((512, 2), (512, 4), (256, 8)), steps: int = 20):
    """The 2D operators: a curved quadrilateral/triangle mesh of the unit
    square (ncell^2 cells, quadrilaterals left of x = 1/2, two triangles per
    cell right of it), FP64 Helmholtz action in one launch, HIP events after a
    cache flush (median of `steps`); algorithmic bytes 16 N_P + 32 Q^2 per
    element (x, y and 4 factors per point)."""
    out = {}
    dev = torch.device("cuda")
    for ncell, P in cases:
        mesh = W.quad_tri_mesh(ncell)
        shapes = ("quad", "tri")
        plan = shp.Plan([(s, P, len(mesh[s]), "curved") for s in shapes])
        for b, s in enumerate(shapes):
            plan.set_geometry(b, torch.from_numpy(W.jacobian2d(mesh[s], shp.quadrature(s, P + 2)[0], True)).to(dev))
        nc, _ = plan.totals()
        x = torch.from_numpy(W.coeffs(1, nc, 90 + P)[0]).to(dev)
        y = torch.empty_like(x)
        _, _, med = time_launches(torch, lambda: plan.apply(-1, "helmholtz", x, out=y), steps, 3, flush=flush)
        nb = sum(len(mesh[s]) * (16 * plan.n_modes[b] + 32 * (P + 2) ** 2) for b, s in enumerate(shapes))
        row = {"cells": ncell, "elements": {s: len(mesh[s]) for s in shapes}, "dof": int(nc), "ms": round(med, 5),
               "GDOF/s": round(nc / (med * 1e-3) / 1e9, 3), "algorithmic_bytes": int(nb),
               "hbm_frac": round(nb / (med * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        out[f"P{P}"] = row
        log(f"  2D P={P}: {row}")
        del plan, x, y
        torch.cuda.empty_cache()
    return out


OP_BYTES = {  # algorithmic HBM bytes per element (N_P modes, N_Q points)
    "bwd": lambda nm, nq: 8 * nm + 8 * nq,
    "iprod": lambda nm, nq: 8 * nq + 8 * nq + 8 * nm,            # f and jw in, y out
    "physderiv": lambda nm, nq: 8 * nq + 72 * nq + 24 * nq,      # u and 9 metric terms in, 3 fields out
    "iprod_deriv": lambda nm, nq: 24 * nq + 80 * nq + 8 * nm,    # 3 fields, 9 metric terms and jw in
    "mass": lambda nm, nq: 16 * nm + 8 * nq,
}


def ops_leg(torch, shp, W, flush, plan, mesh, P: int, steps: int = 20):
    """The other operators on the same mesh (curved, P as the headline): every
    operator as one whole-mesh call with the collocated sum-factorisation and
    with the local matrices (FP64 MFMA; P <= 4), HIP-event medians after a
    cache flush, and the fraction of 8 TB/s of each operator's algorithmic
    bytes."""
    nc, npnt = plan.totals()
    dev = torch.device("cuda")
    out = {}
    for op in OP_BYTES:
        nb = sum(len(mesh[s]) * OP_BYTES[op](plan.n_modes[b], plan.n_points[b]) for b, s in enumerate(SHAPES))
        nin = {"bwd": nc, "mass": nc, "iprod": npnt, "physderiv": npnt, "iprod_deriv": 3 * npnt}[op]
        x = torch.from_numpy(np.ascontiguousarray(W.point_values(1, nin, 77)[0])).to(dev)
        row = {"bytes": int(nb)}
        for st in ("sumfac_coll", "localmat") if P <= 4 else ("sumfac_coll",):
            _, _, med = time_launches(torch, lambda: plan.apply(-1, op, x, strategy=st), steps, 3, flush=flush)
            row[st] = {"ms": round(med, 5), "GDOF/s": round(nc / (med * 1e-3) / 1e9, 3),
                       "hbm_frac": round(nb / (med * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        out[op] = row
        log(f"  operator {op}: {row}")
        del x
    return out


def adr_leg(torch, plan, mesh, x, y, helm_ms: float, steps: int = 20):
    """The advection-diffusion-reaction action (Helmholtz plus b . grad u tested
    with the basis) on the same mesh, velocity U[-1,1] at every point: launch
    time, GDOF/s and HBM rate of its algorithmic bytes (16 N_P + 80 Q^3 per
    element: x, y, 7 factors and 3 advection factors per point)."""
    nc, npnt = plan.totals()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(17)
    vel = torch.rand(3 * npnt, generator=gen, dtype=torch.float64, device="cuda") * 2.0 - 1.0
    adv = plan.advection_factors(vel)
    del vel
    _, m, _ = time_launches(torch, lambda: plan.apply_adr(x, adv, out=y, lam=1.0), steps, 3)
    nbytes = sum(len(mesh[s]) * (16 * plan.n_modes[b] + 80 * plan.n_points[b]) for b, s in enumerate(SHAPES))
    gbs = nbytes / (m * 1e-3) / 1e9
    row = {"workload": "advection-diffusion-reaction action, same mesh, velocity U[-1,1] per point, lambda=1",
           "launch_ms": round(m, 5), "GDOF/s": round(nc / (m * 1e-3) / 1e9, 3), "achieved_GB/s": round(gbs, 1),
           "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "algorithmic_bytes": int(nbytes),
           "vs_helmholtz_launch": round(m / helm_ms, 3)}
    log(f"  adr: {row}")
    del adv
    return row


def c0_leg(torch, shp, W, shape: str = "hex", n: int = 32, P: int = 4, lam: float = 1.0):
    """The C0-assembled problem on the unit cube in n^3 cubes curved by the
    mesh map, homogeneous Dirichlet data: hexahedra (one per cube, aligned
    axes) or the conforming tetrahedral mesh (six per cube; the map carries
    sign changes of odd edge and face modes).  The assembled action (gather,
    elemental action, scatter-sum) against the elemental action alone, and the
    assembled solve of -lap u + lambda u = f for u = sin(pi x) sin(pi y)
    sin(pi z), FP32 PCG with FP64 reliable updates against FP64 PCG."""
    log(f"c0: {n}^3 cubes, curved {shape}, P={P}")
    dev = torch.device("cuda")
    if shape == "hex":
        maps = W.affine_hex_grid(n)
    else:
        maps, verts = W.conforming_tet_mesh(n)
    xi = shp.quadrature(shape, P + 2)[0]
    plan = shp.Plan([(shape, P, len(maps), "curved")])
    plan.set_geometry(0, W.jacobian_torch(maps, xi, True, dev))
    c0 = plan.c0_hex_grid(n, n, n) if shape == "hex" else plan.c0_tet_mesh(verts)
    nc, _ = plan.totals()
    ng = c0["n_global"]
    xg = torch.from_numpy(W.coeffs(1, ng, 17)[0]).cuda()
    yg = torch.empty_like(xg)
    xl = torch.from_numpy(W.coeffs(1, nc, 18)[0]).cuda()
    yl = torch.empty_like(xl)
    _, _, t_c0 = time_launches(torch, lambda: plan.c0_apply(c0, xg, lam=lam, out=yg), 20, 3)
    _, _, t_el = time_launches(torch, lambda: plan.apply(-1, "helmholtz", xl, out=yl, lam=lam), 20, 3)
    f = W.manufactured_u_torch(maps, xi, dev) * (lam + 3 * np.pi ** 2)
    b = plan.c0_assemble(c0, plan.apply(-1, "iprod", f.reshape(-1).contiguous()))
    u_exact = W.manufactured_u_torch(maps, xi, dev).reshape(-1)
    solves = {}
    for name, inner in (("fp64", "fp64"), ("mixed", "fp32")):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st = plan.c0_solve(c0, b, lam=lam, inner=inner, tol=1e-10, check=False)
        torch.cuda.synchronize()
        st["s"] = round(time.perf_counter() - t0, 4)
        u = plan.apply(-1, "bwd", plan.c0_gather(c0, x))
        st["max_err_vs_u"] = float((u - u_exact).abs().max())
        solves[name] = st
        log(f"  c0 solve {name}: {st}")
    out = {"workload": f"{n}^3 cubes, {len(maps)} {shape} elements curved by the mesh map, P={P}, "
                       f"Dirichlet boundary, lambda={lam}",
           "global_dof": int(ng), "local_dof": int(nc),
           "assembled_action_ms": round(t_c0, 5), "elemental_action_ms": round(t_el, 5),
           "assembled_action_GDOF/s_global": round(ng / t_c0 / 1e6, 3), "solve_resid_tol": 1e-10,
           "solve": solves, "speedup": round(solves["fp64"]["s"] / solves["mixed"]["s"], 3)}
    log(f"  c0: {out}")
    return out


def _oracle_piece(args):
    """One worker's share of the CPU baseline: the oracle's Helmholtz action on
    a slice of elements, formation of the dense H_e (explicit quadrature) and
    its application timed apart.  The Jacobian is evaluated first, untimed."""
    shape, P, x0, A, seed = args
    from oracle import shp_oracle as O
    from paper_2604_04644_amd import workloads as W
    maps = W.ElementMaps(shape, x0, A)
    jac = W.jacobian(maps, O.reference_points(shape, P + 2), curved=True)
    x = W.coeffs(len(maps), O.num_modes(shape, P), seed)
    t_form = t_apply = 0.0
    for e0 in range(0, len(maps), 64):
        e1 = min(len(maps), e0 + 64)
        t0 = time.perf_counter()
        H = O.Element(shape, P, P + 2, jac[e0:e1]).helmholtz(1.0)
        t1 = time.perf_counter()
        np.einsum("emn,en->em", H, x[e0:e1])
        t2 = time.perf_counter()
        t_form += t1 - t0
        t_apply += t2 - t1
    return len(maps), len(maps) * O.num_modes(shape, P), t_form, t_apply


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(mesh, P: int, frac: int = 3, frac_1t: int = 128, workers: int = 16):
    """The oracle's Helmholtz action (form each dense H_e by explicit quadrature,
    then y = H_e x) on a fixed random sample of every shape's elements (1/frac
    of each block), spread over `workers` single-threaded processes; and the
    same on a 1/frac_1t sample in one process.  value = sample DOF over the
    parallel run's wall time (formation and application); the CPU seconds of
    each part are reported apart."""
    import multiprocessing as mp
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    nw = max(1, min(workers, avail))
    rng = np.random.default_rng(5)
    jobs, jobs_1t = [], []
    for s in SHAPES:
        perm = rng.permutation(len(mesh[s]))
        idx = np.sort(perm[:max(1, len(mesh[s]) // frac)])
        for k, part in enumerate(np.array_split(idx, 4 * nw)):
            if len(part):
                jobs.append((s, P, mesh[s].x0[part], mesh[s].A[part], 11 + k))
        idx1 = np.sort(perm[:max(1, len(mesh[s]) // frac_1t)])
        jobs_1t.append((s, P, mesh[s].x0[idx1], mesh[s].A[idx1], 7))
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        ctx = mp.get_context("spawn")
        with ctx.Pool(nw) as pool:
            pool.map(_oracle_piece, jobs[:nw], chunksize=1)          # workers up and warm
            t0 = time.perf_counter()
            res = pool.map(_oracle_piece, jobs, chunksize=1)
            wall = time.perf_counter() - t0
        with ctx.Pool(1) as pool:
            pool.map(_oracle_piece, jobs_1t[:1])
            t0 = time.perf_counter()
            res1 = pool.map(_oracle_piece, jobs_1t)
            wall1 = time.perf_counter() - t0
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    n = sum(r[0] for r in res)
    dof = sum(r[1] for r in res)
    t_form = sum(r[2] for r in res)
    t_apply = sum(r[3] for r in res)
    dof1 = sum(r[1] for r in res1)
    return {"value": round(dof / wall / 1e9, 8), "unit": "GDOF/s", "cores": nw, "kind": "oracle",
            "sample": f"{n} elements (a fixed random 1/{frac} of every shape's block), P={P}, in {nw} "
                      f"single-threaded processes; the oracle forms each dense H_e by explicit quadrature and "
                      f"applies it; {wall:.1f} s wall, {t_form + t_apply:.1f} CPU-s",
            "cpu_model": _cpu_model(), "host_cpus": avail,
            "formation_cpu_s": round(t_form, 3), "application_cpu_s": round(t_apply, 3),
            "application_only_GDOF/s": round(dof / (t_apply / nw) / 1e9, 8),
            "one_thread_GDOF/s": round(dof1 / wall1 / 1e9, 8),
            "one_thread_sample": f"{sum(r[0] for r in res1)} elements (1/{frac_1t} of every block), {wall1:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--ncell", type=int, default=32)
    ap.add_argument("--P", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-per-shape", action="store_true",
                    help="skip the per-shape x order table (P = 2, 4, 6, 8, 10 on the same mesh)")
    ap.add_argument("--orders", default="2,4,6,8,10", help="orders of the per-shape table")
    ap.add_argument("--strategies", action="store_true",
                    help="also time collocated vs non-collocated Helmholtz per shape (block launches)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg (P=6 mesh)")
    ap.add_argument("--no-adr", action="store_true", help="skip the advection-diffusion-reaction action")
    ap.add_argument("--no-ops", action="store_true",
                    help="skip the other operators (BwdTrans, IProduct, PhysDeriv, IProductDeriv, mass)")
    ap.add_argument("--no-bf16", action="store_true",
                    help="skip the split-BF16 leg (affine mesh, P=4: actions and solves per inner precision)")
    ap.add_argument("--no-2d", action="store_true", help="skip the 2D quadrilateral/triangle leg")
    ap.add_argument("--no-iso", action="store_true",
                    help="skip the iso-parametric leg (geometry rebuilt in the launch, P = 4 and 6)")
    ap.add_argument("--c0", action="store_true",
                    help="also run the C0-assembled Helmholtz problem, P=4: 32^3 curved hexahedra and the "
                         "conforming tetrahedral mesh of 16^3 cubes")
    ap.add_argument("--affine", action="store_true",
                    help="also time affine blocks per shape and P=1..4: local matrices on MFMA vs sum-factorisation")
    ap.add_argument("--mixed-ncell", type=int, default=32)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (HBM counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU: the elemental action needs no exchange between GPUs, and multi-GPU "
              "runs are not part of this build (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2604_04644_amd import shp, workloads as W
    if not torch.cuda.is_available():
        print("no HIP device visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if a.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 5 copies of 1073741824 bytes (read 1 GiB, write 1 GiB each)")
        return
    P = a.P
    log(f"bench: mixed mesh ncell={a.ncell} P={P}")
    mesh, plan = build_mesh_plan(torch, shp, W, a.ncell, P)
    nc, npnt = plan.totals()
    x = torch.from_numpy(np.concatenate([W.coeffs(len(mesh[s]), plan.n_modes[b], W.SEED_MIXED[s]).ravel()
                                         for b, s in enumerate(SHAPES)])).cuda()
    y = torch.empty_like(x)
    fn = lambda: plan.apply(-1, "helmholtz", x, out=y, lam=1.0)
    log(f"  timing {a.steps} steps after {a.warmup} warm-up")
    wall, ev_mean_ms, ev_med_ms = time_launches(torch, fn, a.steps, a.warmup)
    ms = wall / a.steps * 1e3
    dof = nc
    value = dof / (wall / a.steps) / 1e9
    flush = flush_buffer(torch)
    _, fl_mean_ms, fl_med_ms = time_launches(torch, fn, a.steps, 1, flush=flush)
    copy_gbs = copy_bandwidth(torch, flush)
    nbytes = sum(len(mesh[s]) * bytes_per_elem(plan.n_modes[b], plan.n_points[b]) for b, s in enumerate(SHAPES))
    nflops = sum(len(mesh[s]) * flops_per_elem(s, P) for s in SHAPES)
    achieved = nbytes / (fl_mean_ms * 1e-3) / 1e9
    log(f"  {ms:.3f} ms/step, launch {ev_mean_ms:.3f} ms (median {ev_med_ms:.3f}); with the cache flushed "
        f"{fl_mean_ms:.3f} ms (median {fl_med_ms:.3f}); {value:.2f} GDOF/s, {achieved:.0f} GB/s; "
        f"copy {copy_gbs:.0f} GB/s")
    adr = None if a.no_adr else adr_leg(torch, plan, mesh, x, y, ev_mean_ms)
    ops = None if a.no_ops else ops_leg(torch, shp, W, flush, plan, mesh, P)
    strategies = None
    if a.strategies:
        strategies = {}
        for b, s in enumerate(SHAPES):
            co, _ = plan.offsets(b)
            ne = len(mesh[s])
            xb = x[co:co + ne * plan.n_modes[b]].view(ne, -1)
            yb = torch.empty_like(xb)
            row = {}
            for st in ("sumfac_coll", "sumfac"):
                _, m, _ = time_launches(torch, lambda: plan.apply(b, "helmholtz", xb, out=yb, strategy=st), 20, 3)
                row[st] = {"ms": round(m, 5), "GDOF/s": round(ne * plan.n_modes[b] / (m * 1e-3) / 1e9, 3)}
            row["coll_speedup"] = round(row["sumfac"]["ms"] / row["sumfac_coll"]["ms"], 3)
            strategies[s] = row
            log(f"  {s}: {row}")
    c0 = None
    if a.c0:
        c0 = {"hex": c0_leg(torch, shp, W, "hex", 32), "tet": c0_leg(torch, shp, W, "tet", 16)}
    affine = None
    if a.affine:
        affine = affine_leg(torch, shp, W, flush)
    del plan, x, y
    torch.cuda.empty_cache()
    per_shape = None
    if not a.no_per_shape:
        log("  per-shape x order table")
        per_shape = order_table(torch, shp, W, flush, a.ncell, tuple(int(v) for v in a.orders.split(",")))
    two_d = None
    if not a.no_2d:
        log("  2D leg")
        two_d = leg_2d(torch, shp, W, flush)
    iso = None
    if not a.no_iso:
        log("  iso-parametric leg")
        iso = iso_leg(torch, shp, W, flush, a.ncell)
    del flush
    torch.cuda.empty_cache()
    bf16 = None
    if not a.no_bf16:
        flush = flush_buffer(torch)
        bf16 = bf16_leg(torch, shp, W, flush, a.ncell)
        del flush
        torch.cuda.empty_cache()
    mixed = None
    if not a.no_mixed:
        mixed = mixed_precision_leg(torch, shp, W, a.mixed_ncell)
    cpu = None
    if not a.no_cpu:
        log("  cpu baseline (oracle, bounded sample)")
        cpu = cpu_baseline(mesh, P)
    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"mixed-element mesh {a.ncell}^3 cells (hex/prism/pyr/tet quadrants), curved, "
                               f"P={P}, Q={P + 2}, FP64 Helmholtz action, lambda=1, one whole-mesh launch",
                   "elements": int(sum(len(mesh[s]) for s in SHAPES)), "dof": int(dof),
                   "elements_per_shape": {s: len(mesh[s]) for s in SHAPES}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(P, a.ncell),
                     "algorithmic_bytes": int(nbytes), "launch_ms": round(fl_mean_ms, 5),
                     "launch_ms_median": round(fl_med_ms, 5), "timing": "HIP events on the launch stream, "
                     "Infinity Cache flushed (1 GiB written) before each launch",
                     "launch_ms_unflushed": round(ev_mean_ms, 5),
                     "copy_GB/s": round(copy_gbs, 1), "frac_of_copy": round(achieved / copy_gbs, 4),
                     "algorithmic_flops": int(nflops),
                     "fp64_frac": round(nflops / (fl_mean_ms * 1e-3) / 1e12 / FP64_PEAK_TFS, 4)},
        "cpu_baseline": cpu,
        "mixed_vs_fp64": mixed,
    }
    if per_shape is not None:
        out["per_shape_and_order"] = per_shape
    if strategies is not None:
        out["collocated_vs_noncollocated"] = strategies
    if affine is not None:
        out["affine_localmat_vs_sumfac"] = affine
    if c0 is not None:
        out["c0_assembled"] = c0
    if adr is not None:
        out["adr_action"] = adr
    if ops is not None:
        out["other_operators"] = ops
    if iso is not None:
        out["isoparametric_vs_precomputed"] = iso
    if bf16 is not None:
        out["bf16_split_affine"] = bf16
    if two_d is not None:
        out["quad_tri_2d"] = two_d
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
