"""The seeded input generators: mesh counts, orientation and the two Jacobian
evaluators (numpy and torch) agreeing."""
import numpy as np
import pytest

from paper_2604_04644_amd import workloads as W


def test_quadrant_mesh_counts_and_orientation():
    mesh = W.quadrant_mesh(32)
    assert {s: len(m) for s, m in mesh.items()} == {"hex": 8192, "prism": 16384, "pyr": 49152, "tet": 49152}
    for s, m in mesh.items():
        assert np.all(np.linalg.det(m.A) > 0), s


def test_torch_jacobian_matches_numpy():
    torch = pytest.importorskip("torch")
    maps = W.shape_batch("pyr", 37)
    xi = np.random.default_rng(0).uniform(-1, 1, size=(20, 3))
    for curved in (False, True):
        a = W.jacobian(maps, xi, curved)
        b = W.jacobian_torch(maps, xi, curved, "cpu", chunk=10).numpy()
        assert np.abs(a - b).max() < 1e-14


def test_torch_manufactured_u_matches_numpy():
    torch = pytest.importorskip("torch")
    maps = W.shape_batch("tet", 23)
    xi = np.random.default_rng(1).uniform(-1, 1, size=(17, 3))
    a = W.manufactured_u(W.coords(maps, xi, curved=True))
    b = W.manufactured_u_torch(maps, xi, "cpu", chunk=7).numpy()
    assert np.abs(a - b).max() < 1e-14
