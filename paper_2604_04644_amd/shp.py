"""Python binding of libshp (include/shp.h): argument marshalling only.

Every operator runs in the HIP kernels of libshp.so; this module passes torch
tensor device pointers and the current HIP stream through the C ABI.  There is
no fallback: if the library or a GPU is missing, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libshp.so")

SHAPES = {"hex": 0, "prism": 1, "pyr": 2, "tet": 3, "quad": 4, "tri": 5}
SHAPES_2D = ("quad", "tri")
GEOM = {"affine": 0, "curved": 1, "isoparam": 2}
POINTS = {"gj": 0, "radau": 1}
OPS = {"bwd": 0, "iprod": 1, "physderiv": 2, "iprod_deriv": 3, "mass": 4, "laplacian": 5, "helmholtz": 6}
STRATEGY = {"auto": 0, "sumfac": 1, "sumfac_coll": 2, "localmat": 3}
PREC = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3}
ERRORS = {0: "OK", -1: "INVALID_ARG", -2: "UNSUPPORTED", -3: "BAD_GEOMETRY", -4: "WORKSPACE",
          -5: "STATE", -6: "DEVICE", -7: "NOT_CONVERGED"}

# exported symbols with their argument types
_SIGS = {
    "shp_num_modes": [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
    "shp_num_points": [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
    "shp_quadrature": [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p],
    "shp_plan_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p, ctypes.c_int],
    "shp_vertex_modes": [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)],
    "shp_plan_workspace_bytes": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "shp_plan_bind_workspace": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "shp_plan_set_geometry": [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p],
    "shp_block_offsets": [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                          ctypes.POINTER(ctypes.c_int64)],
    "shp_apply": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_double, ctypes.c_void_p],
    "shp_set_tiling": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                       ctypes.c_int],
    "shp_get_tiling": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
    "shp_plan_destroy": [ctypes.c_void_p],
    "shp_tune": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                 ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                 ctypes.POINTER(ctypes.c_int), ctypes.c_void_p],
    "shp_set_auto_strategy": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int],
    "shp_tune_cache_save": [ctypes.c_void_p, ctypes.c_char_p],
    "shp_tune_cache_load": [ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)],
    "shp_apply_prec": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                       ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p],
    "shp_solve_workspace_bytes": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "shp_advection_factors": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "shp_apply_adr": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                      ctypes.c_void_p],
    "shp_c0_hex_sizes": [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                         ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
    "shp_c0_hex_map": [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                       ctypes.c_void_p],
    "shp_plan_set_fp32_factors": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "shp_c0_tet_sizes": [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                         ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)],
    "shp_c0_tet_map": [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                       ctypes.c_void_p],
    "shp_c0_gather": [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "shp_c0_apply": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p],
    "shp_c0_assemble": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                        ctypes.c_void_p],
    "shp_c0_solve_workspace_bytes": [ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)],
    "shp_c0_helmholtz_solve": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                               ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                               ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t,
                               ctypes.c_void_p, ctypes.c_void_p],
    "shp_helmholtz_diag": [ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                           ctypes.c_void_p],
    "shp_plan_set_model": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                           ctypes.c_void_p],
    "shp_plan_load_model": [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_void_p],
    "shp_model_choose": [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_void_p,
                         ctypes.c_void_p],
    "shp_helmholtz_solve": [ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                            ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p],
}

_lib = None


class TuneResult(ctypes.Structure):
    _fields_ = [("strategy", ctypes.c_int), ("elems_per_wg", ctypes.c_int), ("threads", ctypes.c_int),
                ("variant", ctypes.c_int), ("ms", ctypes.c_double), ("n_candidates", ctypes.c_int),
                ("n_rejected", ctypes.c_int)]


class TuneRecord(ctypes.Structure):
    _fields_ = [("strategy", ctypes.c_int), ("elems_per_wg", ctypes.c_int), ("threads", ctypes.c_int),
                ("variant", ctypes.c_int), ("ms", ctypes.c_double), ("passed", ctypes.c_int)]


STRATEGY_NAME = {v: k for k, v in {"auto": 0, "sumfac": 1, "sumfac_coll": 2, "localmat": 3}.items()}


class SolveStats(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int), ("inner_iters", ctypes.c_int), ("converged", ctypes.c_int),
                ("rel_residual", ctypes.c_double)]


class ShpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _BlockDesc(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int), ("P", ctypes.c_int), ("Q", ctypes.c_int),
                ("n_elem", ctypes.c_int64), ("geom", ctypes.c_int), ("pts", ctypes.c_int)]


def lib() -> ctypes.CDLL:
    """Load libshp.so (built in-tree by paper_2604_04644_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2604_04644_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.shp_last_error.argtypes = []
        L.shp_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(code: int):
    if code != 0:
        raise ShpError(code, lib().shp_last_error().decode())


def num_modes(shape: str, P: int) -> int:
    n = ctypes.c_int()
    _check(lib().shp_num_modes(SHAPES[shape], P, ctypes.byref(n)))
    return n.value


def num_points(shape: str, Q: int) -> int:
    n = ctypes.c_int()
    _check(lib().shp_num_points(SHAPES[shape], Q, ctypes.byref(n)))
    return n.value


def quadrature(shape: str, Q: int, pts: str = "gj"):
    """Reference points xi [Q^3, 3] and weights [Q^3] (numpy, host) of point set
    pts ("gj" or "radau" in the collapsed directions)."""
    import numpy as np
    dim = 2 if shape in SHAPES_2D else 3
    Q3 = Q ** dim
    xi = np.empty((dim, Q3))
    w = np.empty(Q3)
    _check(lib().shp_quadrature(SHAPES[shape], Q, POINTS[pts], xi.ctypes.data, w.ctypes.data))
    return np.ascontiguousarray(xi.T), w


def vertex_modes(shape: str, P: int):
    """Mode indices of the vertex modes and the reference coordinates xi
    [n_vertices, 3] of the vertex where each is one (numpy, host)."""
    import numpy as np
    idx = np.zeros(8, dtype=np.int32)
    xi = np.zeros((8, 3))
    n = ctypes.c_int()
    _check(lib().shp_vertex_modes(SHAPES[shape], P, idx.ctypes.data, xi.ctypes.data, ctypes.byref(n)))
    return idx[:n.value].tolist(), xi[:n.value].copy()


def _stream(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def c0_tet_map(verts, P: int):
    """Host call of shp_c0_tet_map: (l2g, row_ptr, col, n_global) as int64
    numpy arrays for the tetrahedra with vertex ids verts [n_elem][4]."""
    import numpy as np
    v = np.ascontiguousarray(verts, dtype=np.int64)
    if v.ndim != 2 or v.shape[1] != 4:
        raise ValueError("verts must be [n_elem][4]")
    ng, nl, nent = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().shp_c0_tet_sizes(len(v), v.ctypes.data, int(P), ctypes.byref(ng), ctypes.byref(nl),
                                  ctypes.byref(nent)))
    l2g = np.empty(nl.value, dtype=np.int64)
    rp = np.empty(ng.value + 1, dtype=np.int64)
    col = np.empty(max(nent.value, 1), dtype=np.int64)
    _check(lib().shp_c0_tet_map(len(v), v.ctypes.data, int(P), l2g.ctypes.data, rp.ctypes.data, col.ctypes.data))
    return l2g, rp, col, ng.value   # col holds max(n_entries, 1) values


class Plan:
    """A plan over blocks [(shape, P, n_elem, geom[, pts])], with its workspace
    held as a torch uint8 tensor on the current device.  geom defaults to
    "curved", pts (the collapsed directions' points) to "gj".  model: a cost
    model file to load (see load_model); by default the file named by the
    environment variable SHP_MODEL_PATH, if it is set."""

    def __init__(self, blocks: Sequence, device=None, model=None):
        import torch
        self._torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("libshp needs a HIP device; none is visible")
        self.blocks = [(b[0], int(b[1]), int(b[2]), b[3] if len(b) > 3 else "curved") for b in blocks]
        self.points = [b[4] if len(b) > 4 else "gj" for b in blocks]
        arr = (_BlockDesc * len(self.blocks))()
        for i, (sh, P, ne, geom) in enumerate(self.blocks):
            arr[i] = _BlockDesc(SHAPES[sh], P, P + 2, ne, GEOM[geom], POINTS[self.points[i]])
        h = ctypes.c_void_p()
        _check(lib().shp_plan_create(ctypes.byref(h), ctypes.cast(arr, ctypes.c_void_p), len(self.blocks)))
        self._h = h
        nb = ctypes.c_size_t()
        _check(lib().shp_plan_workspace_bytes(self._h, ctypes.byref(nb)))
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        _check(lib().shp_plan_bind_workspace(self._h, ctypes.c_void_p(self._ws_ptr), nb.value, _stream(torch)))
        self.n_modes = [num_modes(sh, P) for sh, P, _, _ in self.blocks]
        self.dim = 2 if self.blocks[0][0] in SHAPES_2D else 3
        self.n_points = [(P + 2) ** self.dim for _, P, _, _ in self.blocks]
        if model is not None or os.environ.get("SHP_MODEL_PATH"):
            self.load_model(model)

    # ---------------------------------------------------------------
    def load_model(self, path=None):
        """Load a cost model file (path, else $SHP_MODEL_PATH): SHP_AUTO then
        uses its per-block choice for the Laplacian and Helmholtz actions."""
        _check(lib().shp_plan_load_model(self._h, None if path is None else str(path).encode(),
                                         _stream(self._torch)))

    def set_model(self, params, mu: float, sigma: float):
        """Copy a model's parameters (float32 device tensor [members][n_params]
        or [n_params]) into the plan."""
        t = self._torch
        if params.dtype != t.float32 or not params.is_cuda or not params.is_contiguous():
            raise ValueError("params must be a contiguous float32 device tensor")
        members = params.shape[0] if params.dim() == 2 else 1
        _check(lib().shp_plan_set_model(self._h, ctypes.c_void_p(params.data_ptr()), members, float(mu),
                                        float(sigma), _stream(t)))

    def model_choose(self, blk: int, op: str = "helmholtz"):
        """The loaded model's strategy for (blk, op) and its predicted launch
        times in ms {strategy: ms} (inf where the block has no such strategy)."""
        import numpy as np
        st = ctypes.c_int()
        pred = np.empty(3)
        _check(lib().shp_model_choose(self._h, blk, OPS[op], ctypes.byref(st), ctypes.c_void_p(pred.ctypes.data),
                                      _stream(self._torch)))
        return STRATEGY_NAME[st.value], dict(zip(("localmat", "sumfac", "sumfac_coll"), pred.tolist()))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.shp_plan_destroy(h)
            self._h = None

    # ---------------------------------------------------------------
    def set_geometry(self, blk: int, jac):
        """jac: float64 device tensor [n][9][Q^3] (curved), [n][9] (affine) or
        the coordinate coefficients [n][3][N_P] (isoparam)."""
        t = self._torch
        self.__dict__.pop("_diag", None)
        sh, P, ne, geom = self.blocks[blk]
        if self.dim == 2:
            want = {"curved": (ne, 4, (P + 2) ** 2), "affine": (ne, 4)}[geom]
        else:
            want = {"curved": (ne, 9, (P + 2) ** 3), "affine": (ne, 9), "isoparam": (ne, 3, self.n_modes[blk])}[geom]
        if tuple(jac.shape) != want or jac.dtype != t.float64 or not jac.is_cuda or not jac.is_contiguous():
            raise ValueError(f"jac must be a contiguous float64 device tensor of shape {want}")
        _check(lib().shp_plan_set_geometry(self._h, blk, ctypes.c_void_p(jac.data_ptr()), _stream(t)))

    def offsets(self, blk: int):
        c, p = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().shp_block_offsets(self._h, blk, ctypes.byref(c), ctypes.byref(p)))
        return c.value, p.value

    def totals(self):
        nc = sum(b[2] * m for b, m in zip(self.blocks, self.n_modes))
        npnt = sum(b[2] * q for b, q in zip(self.blocks, self.n_points))
        return nc, npnt

    def _out_shape(self, blk: int, op: str):
        if blk >= 0:
            ne = self.blocks[blk][2]
            nm, nq = self.n_modes[blk], self.n_points[blk]
            return {"bwd": (ne, nq), "physderiv": (self.dim, ne, nq)}.get(op, (ne, nm))
        nc, npnt = self.totals()
        return {"bwd": (npnt,), "physderiv": (self.dim, npnt)}.get(op, (nc,))

    def _in_numel(self, blk: int, op: str):
        if blk >= 0:
            ne = self.blocks[blk][2]
            nm, nq = self.n_modes[blk], self.n_points[blk]
        else:
            nm, nq, ne = None, None, None
            nc, npnt = self.totals()
            return {"iprod": npnt, "physderiv": npnt, "iprod_deriv": self.dim * npnt}.get(op, nc)
        return {"iprod": ne * nq, "physderiv": ne * nq, "iprod_deriv": self.dim * ne * nq}.get(op, ne * nm)

    def apply(self, blk: int, op: str, x, out=None, lam: float = 1.0, strategy: str = "auto"):
        """y = op(x) for block blk (or the whole mesh, blk = -1); strategy
        "auto" runs the tuned or set choice, else the cost model's (when one is
        loaded), else the collocated sum-factorisation."""
        t = self._torch
        if x.dtype != t.float64 or not x.is_cuda or not x.is_contiguous():
            raise ValueError("x must be a contiguous float64 device tensor")
        if x.numel() != self._in_numel(blk, op):
            raise ValueError(f"x has {x.numel()} values, {op} on block {blk} takes {self._in_numel(blk, op)}")
        if out is None:
            out = t.empty(self._out_shape(blk, op), dtype=t.float64, device=x.device)
        elif out.dtype != t.float64 or not out.is_cuda or not out.is_contiguous() or out.numel() != int(
                t.Size(self._out_shape(blk, op)).numel()):
            raise ValueError("bad output tensor")
        _check(lib().shp_apply(self._h, blk, OPS[op], STRATEGY[strategy], ctypes.c_void_p(x.data_ptr()),
                               ctypes.c_void_p(out.data_ptr()), float(lam), _stream(t)))
        return out

    def apply_prec(self, op: str, x, out=None, lam: float = 1.0, prec: str = "fp32", blk: int = -1,
                   strategy: str | None = None):
        """The action of op with contractions in prec: "fp32" (whole-mesh
        collocated Laplacian/Helmholtz; with strategy "localmat" the affine
        local matrices on the FP32 matrix cores; with "auto" those when they
        are the plan's whole-mesh choice), "bf16" / "bf16x3" (split-BF16 affine
        local matrices: mass, Laplacian, Helmholtz of block blk or, blk = -1,
        every block) or "fp64"; x and out are float32 device tensors (float64
        for fp64)."""
        t = self._torch
        if prec not in PREC:
            raise ShpError(-1, f"unknown precision {prec}")
        dt = t.float64 if prec == "fp64" else t.float32
        if strategy is None:
            strategy = "localmat" if prec.startswith("bf16") else "sumfac_coll"
        if x.dtype != dt or not x.is_cuda or not x.is_contiguous():
            raise ValueError(f"x must be a contiguous {dt} device tensor")
        if x.numel() != self._in_numel(blk, op):
            raise ValueError(f"x has {x.numel()} values, {op} on block {blk} takes {self._in_numel(blk, op)}")
        if out is None:
            out = t.empty(self._out_shape(blk, op), dtype=dt, device=x.device)
        elif out.dtype != dt or not out.is_cuda or not out.is_contiguous() or out.numel() != x.numel():
            raise ValueError("bad output tensor")
        _check(lib().shp_apply_prec(self._h, int(blk), OPS[op], STRATEGY[strategy], PREC[prec],
                                    ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), float(lam),
                                    _stream(t)))
        return out

    def set_fp32_factors(self, enable: bool = True):
        """Attach (or detach) an FP32 copy of the geometric factors, held by
        this Plan, for the FP32 actions and the FP32 inner iterations of the
        solve.  Call after every block's geometry is set."""
        t = self._torch
        if not enable:
            _check(lib().shp_plan_set_fp32_factors(self._h, None, _stream(t)))
            self._fac32 = None
            return None
        _, npnt = self.totals()
        buf = t.empty(7 * npnt, dtype=t.float32, device=self.device)
        _check(lib().shp_plan_set_fp32_factors(self._h, ctypes.c_void_p(buf.data_ptr()), _stream(t)))
        self._fac32 = buf
        return buf

    def advection_factors(self, vel):
        """Advection factors [3 * total points] (float64, device) from the
        velocity at the points, vel [3][total points] float64 on the device."""
        t = self._torch
        _, npnt = self.totals()
        if vel.dtype != t.float64 or not vel.is_cuda or not vel.is_contiguous() or vel.numel() != 3 * npnt:
            raise ValueError(f"vel must be a contiguous float64 device tensor of {3 * npnt} values")
        adv = t.empty(3 * npnt, dtype=t.float64, device=vel.device)
        _check(lib().shp_advection_factors(self._h, ctypes.c_void_p(vel.data_ptr()), ctypes.c_void_p(adv.data_ptr()),
                                           _stream(t)))
        return adv

    def apply_adr(self, x, adv, out=None, lam: float = 1.0):
        """Whole-mesh advection-diffusion-reaction action (FP64)."""
        t = self._torch
        nc, npnt = self.totals()
        if x.dtype != t.float64 or not x.is_cuda or not x.is_contiguous() or x.numel() != nc:
            raise ValueError(f"x must be a contiguous float64 device tensor of {nc} values")
        if adv.dtype != t.float64 or not adv.is_cuda or not adv.is_contiguous() or adv.numel() != 3 * npnt:
            raise ValueError("bad advection factors")
        if out is None:
            out = t.empty_like(x)
        elif out.dtype != t.float64 or not out.is_cuda or not out.is_contiguous() or out.numel() != nc:
            raise ValueError("bad output tensor")
        _check(lib().shp_apply_adr(self._h, ctypes.c_void_p(adv.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), float(lam), _stream(t)))
        return out

    def _solve_ws(self, device):
        nb = ctypes.c_size_t()
        _check(lib().shp_solve_workspace_bytes(self._h, ctypes.byref(nb)))
        ws = getattr(self, "_sws", None)
        if ws is None or ws.numel() < nb.value + 256:
            ws = self._sws = self._torch.empty(nb.value + 256, dtype=self._torch.uint8, device=device)
        return ctypes.c_void_p((ws.data_ptr() + 255) // 256 * 256), nb.value

    def helmholtz_diag(self, lam: float = 1.0):
        """diag(lam M + L) of every element in the whole-mesh layout (FP64,
        device), cached per lam until the geometry changes."""
        t = self._torch
        cache = self.__dict__.setdefault("_diag", {})
        if lam not in cache:
            nc, _ = self.totals()
            d = t.empty(nc, dtype=t.float64, device=self.device)
            ws, nb = self._solve_ws(self.device)
            _check(lib().shp_helmholtz_diag(self._h, float(lam), ctypes.c_void_p(d.data_ptr()), ws, nb, _stream(t)))
            cache[lam] = d
        return cache[lam]

    def solve(self, b, x=None, lam: float = 1.0, inner: str = "fp32", tol: float = 1e-10, max_outer: int = 100,
              max_inner: int = 50000, inner_tol: float = 0.1, check: bool = True):
        """Solve (lam M + L) x = b on every element: Jacobi-PCG in `inner`
        precision with FP64 reliable updates every `inner_tol` reduction of the
        residual (at most `max_outer` of them, `max_inner` iterations in all).
        Returns (x, stats)."""
        t = self._torch
        nc, _ = self.totals()
        if b.dtype != t.float64 or not b.is_cuda or not b.is_contiguous() or b.numel() != nc:
            raise ValueError("b must be a contiguous float64 device tensor of all coefficients")
        if x is None:
            x = t.zeros_like(b)
        elif x.dtype != t.float64 or not x.is_cuda or not x.is_contiguous() or x.numel() != nc:
            raise ValueError("bad initial guess")
        diag = self.helmholtz_diag(lam)
        ws, nb = self._solve_ws(b.device)
        st = SolveStats()
        code = lib().shp_helmholtz_solve(self._h, float(lam), ctypes.c_void_p(diag.data_ptr()),
                                         ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()), PREC[inner],
                                         float(tol), int(max_outer), int(max_inner), float(inner_tol), ws, nb,
                                         ctypes.byref(st), _stream(t))
        stats = {"outer_iters": st.outer_iters, "inner_iters": st.inner_iters, "converged": bool(st.converged),
                 "rel_residual": st.rel_residual}
        if code != 0 and (check or code != -7):
            _check(code)
        return x, stats

    # ---------------------------------------------------------------
    def c0_hex_grid(self, n0: int, n1: int, n2: int):
        """Local-to-global map of the plan's single hex block as an n0 x n1 x n2
        grid (homogeneous Dirichlet data); returns a C0 handle dict with the
        device arrays l2g, row_ptr, col and the global size."""
        import numpy as np
        t = self._torch
        (sh, P, ne, _), = self.blocks
        if sh != "hex" or ne != n0 * n1 * n2:
            raise ValueError("the plan must hold the grid's hexahedra as its only block")
        ng, nl, nent = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().shp_c0_hex_sizes(n0, n1, n2, P, ctypes.byref(ng), ctypes.byref(nl), ctypes.byref(nent)))
        l2g = np.empty(nl.value, dtype=np.int64)
        rp = np.empty(ng.value + 1, dtype=np.int64)
        col = np.empty(max(nent.value, 1), dtype=np.int64)
        _check(lib().shp_c0_hex_map(n0, n1, n2, P, l2g.ctypes.data, rp.ctypes.data, col.ctypes.data))
        dev = self.device
        return {"n_global": ng.value, "l2g": t.from_numpy(l2g).to(dev), "row_ptr": t.from_numpy(rp).to(dev),
                "col": t.from_numpy(col).to(dev)}

    def c0_tet_mesh(self, verts):
        """Local-to-global map of the plan's single tet block on a conforming
        mesh with vertex ids verts [n_elem][4] (local order rule of
        shp_c0_tet_map; homogeneous Dirichlet data on the boundary faces);
        returns a C0 handle dict like c0_hex_grid."""
        t = self._torch
        (sh, P, ne, _), = self.blocks
        if sh != "tet" or ne != len(verts):
            raise ValueError("the plan must hold the mesh's tetrahedra as its only block")
        l2g, rp, col, ng = c0_tet_map(verts, P)
        dev = self.device
        return {"n_global": ng, "l2g": t.from_numpy(l2g).to(dev), "row_ptr": t.from_numpy(rp).to(dev),
                "col": t.from_numpy(col).to(dev)}

    def c0_gather(self, c0, xg):
        """The local coefficients A xg of a global vector (signed copies, 0 on
        the Dirichlet boundary)."""
        t = self._torch
        nc, _ = self.totals()
        ng = c0["n_global"]
        if xg.dtype != t.float64 or not xg.is_cuda or not xg.is_contiguous() or xg.numel() != ng:
            raise ValueError(f"xg must be a contiguous float64 device tensor of {ng} values")
        out = t.empty(nc, dtype=t.float64, device=xg.device)
        _check(lib().shp_c0_gather(ctypes.c_void_p(c0["l2g"].data_ptr()), nc, ctypes.c_void_p(xg.data_ptr()),
                                   ctypes.c_void_p(out.data_ptr()), _stream(t)))
        return out

    def c0_assemble(self, c0, vl):
        """A^T vl for a local vector (all coefficients of the block)."""
        t = self._torch
        nc, _ = self.totals()
        if vl.dtype != t.float64 or not vl.is_cuda or not vl.is_contiguous() or vl.numel() != nc:
            raise ValueError(f"vl must be a contiguous float64 device tensor of {nc} values")
        out = t.empty(c0["n_global"], dtype=t.float64, device=vl.device)
        _check(lib().shp_c0_assemble(ctypes.c_void_p(c0["row_ptr"].data_ptr()), ctypes.c_void_p(c0["col"].data_ptr()),
                                     c0["n_global"], ctypes.c_void_p(vl.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                     _stream(t)))
        return out

    def c0_apply(self, c0, xg, lam: float = 1.0, out=None):
        """Assembled FP64 Helmholtz action A^T H A xg."""
        t = self._torch
        nc, _ = self.totals()
        ng = c0["n_global"]
        if xg.dtype != t.float64 or not xg.is_cuda or not xg.is_contiguous() or xg.numel() != ng:
            raise ValueError(f"xg must be a contiguous float64 device tensor of {ng} values")
        if out is None:
            out = t.empty(ng, dtype=t.float64, device=xg.device)
        elif out.dtype != t.float64 or not out.is_cuda or not out.is_contiguous() or out.numel() != ng:
            raise ValueError("bad output tensor")
        work = t.empty(2 * nc, dtype=t.float64, device=xg.device)
        _check(lib().shp_c0_apply(self._h, ctypes.c_void_p(c0["l2g"].data_ptr()),
                                  ctypes.c_void_p(c0["row_ptr"].data_ptr()), ctypes.c_void_p(c0["col"].data_ptr()),
                                  c0["n_global"], ctypes.c_void_p(xg.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                  float(lam), ctypes.c_void_p(work.data_ptr()), _stream(t)))
        return out

    def c0_solve(self, c0, b, x=None, lam: float = 1.0, inner: str = "fp32", tol: float = 1e-10,
                 max_outer: int = 100, max_inner: int = 50000, inner_tol: float = 0.1, check: bool = True):
        """Solve A^T H A x = b (assembled, Dirichlet DOFs dropped) with the
        mixed-precision PCG.  Returns (x, stats)."""
        t = self._torch
        ng = c0["n_global"]
        if b.dtype != t.float64 or not b.is_cuda or not b.is_contiguous() or b.numel() != ng:
            raise ValueError("b must be a contiguous float64 device tensor of the global DOFs")
        if x is None:
            x = t.zeros_like(b)
        elif x.dtype != t.float64 or not x.is_cuda or not x.is_contiguous() or x.numel() != ng:
            raise ValueError("bad initial guess")
        nb = ctypes.c_size_t()
        _check(lib().shp_c0_solve_workspace_bytes(self._h, ng, ctypes.byref(nb)))
        ws = t.empty(nb.value + 256, dtype=t.uint8, device=b.device)
        st = SolveStats()
        code = lib().shp_c0_helmholtz_solve(
            self._h, ctypes.c_void_p(c0["l2g"].data_ptr()), ctypes.c_void_p(c0["row_ptr"].data_ptr()),
            ctypes.c_void_p(c0["col"].data_ptr()), ng, float(lam), ctypes.c_void_p(b.data_ptr()),
            ctypes.c_void_p(x.data_ptr()), PREC[inner], float(tol), int(max_outer), int(max_inner), float(inner_tol),
            ctypes.c_void_p((ws.data_ptr() + 255) // 256 * 256), nb.value, ctypes.byref(st), _stream(t))
        stats = {"outer_iters": st.outer_iters, "inner_iters": st.inner_iters, "converged": bool(st.converged),
                 "rel_residual": st.rel_residual}
        if code != 0 and (check or code != -7):
            _check(code)
        return x, stats

    def set_tiling(self, blk: int, op: str, E: int, NT: int, persistent: int = 1, strategy: str = "sumfac_coll"):
        _check(lib().shp_set_tiling(self._h, blk, OPS[op], STRATEGY[strategy], E, NT, persistent))

    def get_tiling(self, blk: int, op: str, strategy: str = "sumfac_coll"):
        E, NT, pe = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().shp_get_tiling(self._h, blk, OPS[op], STRATEGY[strategy], ctypes.byref(E), ctypes.byref(NT),
                                    ctypes.byref(pe)))
        return E.value, NT.value, pe.value

    # ---------------------------------------------------------------
    def tune(self, blk: int, op: str, x, lam: float = 1.0, reps: int = 10, quick: bool = False,
             max_records: int = 4096):
        """Exhaustive tuning of (blk, op) on input x; returns (result dict, list of
        candidate records).  SHP_AUTO then uses the choice."""
        t = self._torch
        if x.dtype != t.float64 or not x.is_cuda or not x.is_contiguous() or x.numel() != self._in_numel(blk, op):
            raise ValueError(f"x must be a contiguous float64 device tensor of {self._in_numel(blk, op)} values")
        out = t.empty(self._out_shape(blk, op), dtype=t.float64, device=x.device)
        ref = t.empty_like(out)
        res = TuneResult()
        recs = (TuneRecord * max_records)()
        nrec = ctypes.c_int()
        _check(lib().shp_tune(self._h, blk, OPS[op], ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                              ctypes.c_void_p(ref.data_ptr()), float(lam), int(reps), int(quick), ctypes.byref(res),
                              ctypes.cast(recs, ctypes.c_void_p), max_records, ctypes.byref(nrec), _stream(t)))
        result = {"strategy": STRATEGY_NAME[res.strategy], "elems_per_wg": res.elems_per_wg,
                  "threads": res.threads, "variant": res.variant, "ms": res.ms,
                  "n_candidates": res.n_candidates, "n_rejected": res.n_rejected}
        records = [{"strategy": STRATEGY_NAME[r.strategy], "elems_per_wg": r.elems_per_wg, "threads": r.threads,
                    "variant": r.variant, "ms": r.ms, "passed": bool(r.passed)} for r in recs[:nrec.value]]
        return result, records

    def set_auto_strategy(self, blk: int, op: str, strategy: str):
        _check(lib().shp_set_auto_strategy(self._h, blk, OPS[op], STRATEGY[strategy]))

    def save_tuning(self, path: str):
        _check(lib().shp_tune_cache_save(self._h, path.encode()))

    def load_tuning(self, path: str) -> int:
        n = ctypes.c_int()
        _check(lib().shp_tune_cache_load(self._h, path.encode(), ctypes.byref(n)))
        return n.value
