"""CPU tests of the C ABI: the library loads, exports every declared symbol,
and validates its arguments before any HIP call (so error paths run without a
GPU).  Host-side reference data (quadrature points and weights) are compared
with the oracle's independent construction."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import shp_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shp.h")


@pytest.fixture(scope="module")
def L():
    from paper_2604_04644_amd import shp
    if not os.path.exists(shp.LIB_PATH):
        pytest.skip("libshp.so not built")
    return shp.lib()


def declared_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(shp_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(L):
    syms = declared_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(L, s), s


def test_num_modes_and_points(L):
    from paper_2604_04644_amd import shp
    for shape in O.SHAPES:
        for P in range(1, 11):
            assert shp.num_modes(shape, P) == O.num_modes(shape, P)
        assert shp.num_points(shape, 6) == 216


@pytest.mark.parametrize("pts", ["gj", "radau"])
@pytest.mark.parametrize("shape", O.SHAPES)
@pytest.mark.parametrize("Q", [3, 4, 6, 8, 12])
def test_quadrature_matches_oracle(L, shape, Q, pts):
    """Library rule (Newton on Jacobi polynomials; Radau: -1 plus the shifted
    Gauss-Jacobi zeros and the closed-form end weight) vs the oracle's
    Golub-Welsch (Radau: Golub's modified Jacobi matrix)."""
    from paper_2604_04644_amd import shp
    xi, w = shp.quadrature(shape, Q, pts)
    eta, wo, _ = O.quadrature(shape, Q, pts)
    assert np.abs(xi - O.collapse(shape, eta)).max() < 2e-15
    assert np.abs(w - wo).max() < 1e-14 * max(1.0, np.abs(wo).max())


def _code(L, f, *args):
    return f(*args)


def test_error_paths_without_device(L):
    from paper_2604_04644_amd import shp
    n = ctypes.c_int()
    assert L.shp_num_modes(7, 3, ctypes.byref(n)) == -1          # bad shape
    assert L.shp_num_modes(0, 11, ctypes.byref(n)) == -2         # P out of range
    assert L.shp_num_modes(0, 0, ctypes.byref(n)) == -2
    assert L.shp_num_modes(0, 3, None) == -1                     # null output
    assert L.shp_quadrature(0, 6, 0, None, None) == -1
    assert "null" in L.shp_last_error().decode()
    buf9 = (ctypes.c_double * 648)()
    assert L.shp_quadrature(3, 6, 2, ctypes.cast(buf9, ctypes.c_void_p), None) == -1  # bad point set
    assert "point set" in L.shp_last_error().decode()

    def plan(descs):
        arr = (shp._BlockDesc * len(descs))(*[shp._BlockDesc(*d) for d in descs])
        h = ctypes.c_void_p()
        rc = L.shp_plan_create(ctypes.byref(h), ctypes.cast(arr, ctypes.c_void_p), len(descs))
        return rc, h

    assert plan([(0, 4, 5, 10, 1)])[0] == -2                     # Q != P+2
    assert plan([(0, 11, 13, 10, 1)])[0] == -2                   # P > 10
    assert plan([(9, 4, 6, 10, 1)])[0] == -1                     # bad shape
    assert plan([(0, 4, 6, -1, 1)])[0] == -1                     # negative count
    assert plan([(0, 4, 6, 10, 5)])[0] == -1                     # bad geom
    assert plan([(3, 4, 6, 10, 1, 2)])[0] == -1                  # bad point set
    rc, h = plan([(0, 4, 6, 10, 1), (3, 4, 6, 7, 1)])
    assert rc == 0
    nb = ctypes.c_size_t()
    assert L.shp_plan_workspace_bytes(h, ctypes.byref(nb)) == 0
    # hex: 10 elements * 16 factors * 216 points * 8 bytes at least
    assert nb.value >= (10 + 7) * 16 * 216 * 8
    # apply / geometry before a workspace is bound
    buf = (ctypes.c_double * 8)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert L.shp_apply(h, 0, 6, 2, p, p, 1.0, None) == -5
    assert L.shp_plan_set_geometry(h, 0, p, None) == -5
    # bad arguments
    assert L.shp_apply(h, 5, 6, 2, p, p, 1.0, None) == -1        # block index
    assert L.shp_apply(h, 0, 9, 2, p, p, 1.0, None) == -1        # operator
    assert L.shp_apply(h, 0, 6, 7, p, p, 1.0, None) == -1        # strategy
    assert L.shp_apply(h, 0, 6, 2, None, p, 1.0, None) == -1     # null input
    assert L.shp_apply(h, 0, 6, 2, p, p, float("nan"), None) == -1
    assert L.shp_apply_adr(h, None, p, p, 1.0, None) == -1        # null advection factors
    assert L.shp_apply_adr(h, p, p, p, float("inf"), None) == -1
    assert L.shp_apply_adr(h, p, p, p, 1.0, None) == -5           # no workspace yet
    assert L.shp_advection_factors(h, None, p, None) == -1
    assert L.shp_advection_factors(h, p, p, None) == -5
    # workspace validation (no device call is reached)
    assert L.shp_plan_bind_workspace(h, None, nb.value, None) == -4
    assert L.shp_plan_bind_workspace(h, ctypes.c_void_p(256 * 1000 + 8), nb.value, None) == -4
    assert L.shp_plan_bind_workspace(h, ctypes.c_void_p(256 * 1000), nb.value - 1, None) == -4
    # tiling validation
    assert L.shp_set_tiling(h, 0, 6, 2, 0, 256, 1) == -1
    assert L.shp_set_tiling(h, 0, 6, 2, 4, 100, 1) == -1
    assert L.shp_set_tiling(h, 0, 6, 2, 4, 128, 7) == -1
    assert L.shp_set_tiling(h, 0, 6, 2, 64, 256, 1) == -2        # LDS overflow at P=4
    assert L.shp_set_tiling(h, 0, 6, 2, 4, 128, 0) == 0
    E, NT, pe = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    assert L.shp_get_tiling(h, 0, 6, 2, ctypes.byref(E), ctypes.byref(NT), ctypes.byref(pe)) == 0
    assert (E.value, NT.value, pe.value) == (4, 128, 0)
    assert L.shp_set_tiling(h, 0, 6, 2, 0, 0, 0) == 0            # back to default
    assert L.shp_get_tiling(h, -1, 6, 2, ctypes.byref(E), ctypes.byref(NT), ctypes.byref(pe)) == 0
    assert (E.value, NT.value, pe.value) == (4, 256, 2)          # 40 KiB LDS budget at P=4
    rc6, h6 = plan([(0, 6, 8, 10, 1), (3, 6, 8, 7, 1)])
    assert rc6 == 0
    assert L.shp_get_tiling(h6, 1, 6, 2, ctypes.byref(E), ctypes.byref(NT), ctypes.byref(pe)) == 0
    # tet block at P=6: the Helmholtz tile's LDS head holds only its per-lane
    # tables, so 40 KiB holds two elements (4 point buffers of 8^3 doubles each)
    assert (E.value, NT.value, pe.value) == (2, 256, 2)
    assert L.shp_get_tiling(h6, -1, 6, 2, ctypes.byref(E), ctypes.byref(NT), ctypes.byref(pe)) == 0
    assert (E.value, NT.value, pe.value) == (2, 256, 2)          # whole mesh: 64 KiB, two elements
    assert L.shp_plan_destroy(h6) == 0
    c, q = ctypes.c_int64(), ctypes.c_int64()
    assert L.shp_block_offsets(h, 1, ctypes.byref(c), ctypes.byref(q)) == 0
    assert (c.value, q.value) == (10 * 125, 10 * 216)
    # precision and solver validation (no device call is reached)
    assert L.shp_apply_prec(h, -1, 6, 2, 2, p, p, 1.0, None) == -2    # BF16: local matrices only
    assert L.shp_apply_prec(h, -1, 6, 3, 2, p, p, 1.0, None) == -2    # BF16 on curved blocks
    assert L.shp_apply_prec(h, 0, 6, 3, 3, p, p, 1.0, None) == -2     # BF16x3 on a curved block
    assert L.shp_apply_prec(h, -1, 1, 3, 2, p, p, 1.0, None) == -2    # BF16 inner product
    assert L.shp_apply_prec(h, -1, 6, 3, 1, p, p, 1.0, None) == -2    # FP32 local matrices, curved blocks
    assert L.shp_apply_prec(h, -1, 6, 2, 5, p, p, 1.0, None) == -1    # bad precision
    assert L.shp_apply_prec(h, -1, 4, 2, 1, p, p, 1.0, None) == -2    # FP32 mass
    assert L.shp_apply_prec(h, 0, 6, 2, 1, p, p, 1.0, None) == -2     # FP32 per block
    assert L.shp_apply_prec(h, -1, 6, 1, 1, p, p, 1.0, None) == -2    # FP32 non-collocated
    assert L.shp_apply_prec(h, -1, 6, 2, 1, p, p, 1.0, None) == -5    # no workspace
    sb = ctypes.c_size_t()
    assert L.shp_solve_workspace_bytes(h, ctypes.byref(sb)) == 0
    ncoef = 10 * 125 + 7 * 35
    assert sb.value >= ncoef * (2 * 8 + 4 + 5 * 8 + 4)
    st = shp.SolveStats()
    ws = ctypes.c_void_p(256 * 1000)

    def solve(lam=1.0, prec=1, tol=1e-10, mo=10, mi=100, itol=1e-3, w=ws, nbytes=sb.value):
        return L.shp_helmholtz_solve(h, lam, p, p, p, prec, tol, mo, mi, itol, w, nbytes, ctypes.byref(st), None)
    assert solve(prec=2) == -5 and solve(prec=3) == -5            # BF16 inner: no workspace bound
    assert solve(prec=4) == -1
    assert solve(lam=0.0) == -1                                   # H only semidefinite
    assert solve(tol=0.0) == -1
    assert solve(mo=0) == -1
    assert solve(w=None) == -1
    assert solve(w=ctypes.c_void_p(256 * 1000 + 64)) == -4        # misaligned
    assert solve(nbytes=sb.value - 1) == -4
    assert solve() == -5                                          # no workspace bound
    assert L.shp_helmholtz_diag(h, 1.0, None, ws, sb.value, None) == -1
    assert L.shp_helmholtz_diag(h, float("inf"), p, ws, sb.value, None) == -1
    assert L.shp_helmholtz_diag(h, 1.0, p, ws, sb.value - 8, None) == -4
    assert L.shp_helmholtz_diag(h, 1.0, p, ws, sb.value, None) == -5
    assert L.shp_plan_destroy(h) == 0
    assert L.shp_plan_destroy(None) == -1


def test_no_fallback_without_library_or_device(tmp_path):
    """The binding raises when libshp.so is missing, and a plan needs a HIP
    device: there is no CPU path."""
    import subprocess
    import sys
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_2604_04644_amd import shp\n"
        "shp.LIB_PATH = %r\n"
        "try:\n"
        "    shp.lib()\n"
        "except RuntimeError as e:\n"
        "    print('raised', 'missing' in str(e))\n"
    ) % (ROOT, str(tmp_path / "absent.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120)
    assert r.stdout.strip() == "raised True", r.stdout + r.stderr
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        from paper_2604_04644_amd import shp
        with pytest.raises(RuntimeError):
            shp.Plan([("hex", 2, 4, "curved")])


def test_model_file_validation_without_device(L, tmp_path):
    """shp_plan_load_model checks the file before any HIP call: a missing,
    truncated, mis-sized or non-finite file is INVALID_ARG; a good file on a
    plan without a workspace is STATE (the upload needs the device)."""
    import json
    import struct
    from paper_2604_04644_amd import shp
    arr = (shp._BlockDesc * 1)(shp._BlockDesc(0, 2, 4, 10, 1, 0))
    h = ctypes.c_void_p()
    assert L.shp_plan_create(ctypes.byref(h), ctypes.cast(arr, ctypes.c_void_p), 1) == 0
    L.shp_plan_load_model.argtypes = [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_void_p]
    n = 64 * 11 + 64 + 64 * 64 + 64 + 64 + 1

    def write(name, head, values):
        p = tmp_path / name
        with open(p, "wb") as f:
            f.write((json.dumps(head) + "\n").encode())
            f.write(struct.pack(f"<{len(values)}f", *values))
        return str(p).encode()

    good = {"format": "shp-mlp", "nin": 11, "nh": 64, "n_params": n, "members": 2, "mu": -20.0, "sigma": 1.5}
    ok = write("ok.bin", good, [0.01] * (2 * n))
    assert L.shp_plan_load_model(h, ok, None) == -5
    assert L.shp_plan_load_model(h, str(tmp_path / "none.bin").encode(), None) == -1
    assert L.shp_plan_load_model(h, write("short.bin", good, [0.01] * (2 * n - 1)), None) == -1
    assert L.shp_plan_load_model(h, write("long.bin", good, [0.01] * (2 * n + 1)), None) == -1
    assert L.shp_plan_load_model(h, write("nan.bin", good, [0.01] * (2 * n - 1) + [float("nan")]), None) == -1
    assert L.shp_plan_load_model(h, write("sig.bin", dict(good, sigma=0.0), [0.01] * (2 * n)), None) == -1
    assert L.shp_plan_load_model(h, write("mem.bin", dict(good, members=5), [0.01] * (5 * n)), None) == -1
    assert L.shp_plan_load_model(h, write("fmt.bin", dict(good, format="other"), [0.01] * (2 * n)), None) == -1
    assert L.shp_plan_load_model(h, write("nh.bin", dict(good, nh=32), [0.01] * (2 * n)), None) == -1
    assert "cost model file" in L.shp_last_error().decode()
    L.shp_plan_destroy(h)


@pytest.mark.parametrize("shape", O.SHAPES)
def test_vertex_modes_match_oracle(L, shape):
    """shp_vertex_modes gives the oracle's vertex modes and vertices, and each
    is one at its vertex and zero at the others (the oracle's basis)."""
    from paper_2604_04644_amd import shp
    for P in (1, 2, 5, 10):
        idx, xi = shp.vertex_modes(shape, P)
        oidx, oxi = O.vertex_modes(shape, P)
        assert idx == oidx
        assert np.array_equal(xi, oxi)
    # nodality at the vertices, through the oracle's basis at points just inside
    P = 3
    idx, xi = shp.vertex_modes(shape, P)
    modes = O.modes(shape, P)
    for v, (m, x) in enumerate(zip(idx, xi)):
        assert modes[m] == O.VERTEX_MODES[shape][v]


@pytest.mark.parametrize("pts", ["gj", "radau"])
@pytest.mark.parametrize("shape", ["quad", "tri"])
def test_2d_sizes_and_quadrature(L, shape, pts):
    """2D mode and point counts, and the library's 2D points and weights
    against the 2D oracle's (Golub-Welsch)."""
    from oracle import shp_oracle2d as O2
    from paper_2604_04644_amd import shp
    for P in (1, 4, 10):
        assert shp.num_modes(shape, P) == O2.num_modes(shape, P)
        assert shp.num_points(shape, P + 2) == (P + 2) ** 2
    for Q in (3, 6, 12):
        xi, w = shp.quadrature(shape, Q, pts)
        eta, wo, _ = O2.quadrature(shape, Q, pts)
        assert np.abs(xi - O2.collapse(shape, eta)).max() < 2e-15
        assert np.abs(w - wo).max() < 1e-14 * max(1.0, np.abs(wo).max())


def test_2d_plan_rules_without_device(L):
    """A plan holds 2D or 3D blocks, not both; 2D blocks are not iso-parametric."""
    from paper_2604_04644_amd import shp
    h = ctypes.c_void_p()
    mixed = (shp._BlockDesc * 2)(shp._BlockDesc(4, 2, 4, 10, 1, 0), shp._BlockDesc(0, 2, 4, 10, 1, 0))
    assert L.shp_plan_create(ctypes.byref(h), ctypes.cast(mixed, ctypes.c_void_p), 2) == -1
    iso2 = (shp._BlockDesc * 1)(shp._BlockDesc(5, 2, 4, 10, 2, 0))
    assert L.shp_plan_create(ctypes.byref(h), ctypes.cast(iso2, ctypes.c_void_p), 1) == -2
    ok = (shp._BlockDesc * 2)(shp._BlockDesc(4, 2, 4, 10, 1, 0), shp._BlockDesc(5, 2, 4, 7, 0, 1))
    assert L.shp_plan_create(ctypes.byref(h), ctypes.cast(ok, ctypes.c_void_p), 2) == 0
    nb = ctypes.c_size_t()
    assert L.shp_plan_workspace_bytes(h, ctypes.byref(nb)) == 0 and nb.value > 0
    L.shp_plan_destroy(h)
    # launch shapes of 2D blocks: elements and threads, the collocated form only
    p10 = (shp._BlockDesc * 1)(shp._BlockDesc(4, 10, 12, 100, 1, 0))
    assert L.shp_plan_create(ctypes.byref(h), ctypes.cast(p10, ctypes.c_void_p), 1) == 0
    assert L.shp_set_tiling(h, 0, 6, 2, 8, 256, 0) == 0
    assert L.shp_set_tiling(h, -1, 6, 2, 12, 512, 0) == 0
    assert L.shp_set_tiling(h, 0, 6, 2, 64, 256, 0) == -2           # 64 elements of 12^2 points overflow LDS
    assert L.shp_set_tiling(h, 0, 6, 1, 8, 256, 0) == -2            # non-collocated strategy
    E, NT, pe = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    assert L.shp_get_tiling(h, 0, 6, 2, ctypes.byref(E), ctypes.byref(NT), ctypes.byref(pe)) == 0
    assert (E.value, NT.value) == (8, 256)
    L.shp_plan_destroy(h)
