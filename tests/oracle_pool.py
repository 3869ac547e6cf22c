"""The FP64 oracle over large element batches, spread over worker processes.

Test infrastructure: each worker evaluates the oracle (oracle.shp_oracle.apply_op,
unchanged) on a contiguous slice of the batch; the slices are joined in element
order, so the result is the one apply_op gives on the whole batch.  Workers
take the element maps, not the Jacobians, and evaluate the mesh map's Jacobian
at the oracle's own points themselves, so only small arrays cross process
boundaries.  The pool uses the "spawn" start method: the workers never touch
the GPU and do not inherit the parent's HIP state.
"""
from __future__ import annotations

import atexit
import multiprocessing as mp
import os

import numpy as np

_POOL = None
_POOL_N = 0


def _pool(workers: int):
    """One pool of worker processes for the whole test session (started on
    first use: starting processes costs about a second each time)."""
    global _POOL, _POOL_N
    if _POOL is None or _POOL_N != workers:
        if _POOL is not None:
            _POOL.terminate()
        # one BLAS thread per worker: the workers already fill the cores
        keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
        saved = {k: os.environ.get(k) for k in keys}
        os.environ.update({k: "1" for k in keys})
        try:
            _POOL = mp.get_context("spawn").Pool(workers)
        finally:
            for k, v in saved.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
        _POOL_N = workers
        atexit.register(_POOL.terminate)
    return _POOL


def n_workers(limit: int = 16) -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(limit, n))


def _work(args):
    op, shape, P, x0, A, curved, x, lam, pts, X = args
    from oracle import shp_oracle as O
    from paper_2604_04644_amd import workloads as W
    Q = P + 2
    if X is not None:
        jac = O.isoparametric_jacobian(shape, P, Q, X, pts)
        chunk = max(1, min(64, int(4e8 // (8 * 4 * Q ** 3 * O.num_modes(shape, P)))))
        return O.apply_op(op, shape, P, Q, jac, x, lam=lam, chunk=chunk, pts=pts)
    maps = W.ElementMaps(shape, x0, A)
    if curved:
        jac = W.jacobian(maps, O.reference_points(shape, Q, pts), curved=True)
    else:
        jac = W.affine_jacobian(maps)
    chunk = max(1, min(64, int(4e8 // (8 * 4 * Q ** 3 * O.num_modes(shape, P)))))
    return O.apply_op(op, shape, P, Q, jac, x, lam=lam, chunk=chunk, pts=pts)


def apply_op(op: str, shape: str, P: int, maps, x, lam: float = 1.0, curved: bool = True, pts: str = "gj",
             workers: int | None = None, pieces_per_worker: int = 4, X=None):
    """oracle.apply_op(op, shape, P, P + 2, jac(maps), x) with the batch split
    over worker processes.  x: [n_elem][..] (coefficients or point values) or
    [3][n_elem][N_Q] for iprod_deriv.  With X (iso-parametric coordinate
    coefficients [n_elem][3][N_P]) the Jacobian is the oracle's
    isoparametric_jacobian of X and maps only gives the element count."""
    x = np.asarray(x, dtype=np.float64)
    ne = len(maps) if X is None else X.shape[0]
    workers = workers or n_workers()
    npiece = max(1, min(ne, workers * pieces_per_worker))
    bounds = np.linspace(0, ne, npiece + 1).astype(int)
    jobs = []
    for a, b in zip(bounds[:-1], bounds[1:]):
        if b <= a:
            continue
        xs = x[:, a:b] if op == "iprod_deriv" else x[a:b]
        if X is None:
            jobs.append((op, shape, P, maps.x0[a:b], maps.A[a:b], curved, np.ascontiguousarray(xs), lam, pts, None))
        else:
            jobs.append((op, shape, P, None, None, curved, np.ascontiguousarray(xs), lam, pts,
                         np.ascontiguousarray(X[a:b])))
    if workers == 1 or len(jobs) == 1:
        outs = [_work(j) for j in jobs]
    else:
        outs = _pool(workers).map(_work, jobs, chunksize=1)
    return np.concatenate(outs, axis=1 if op == "physderiv" else 0)
