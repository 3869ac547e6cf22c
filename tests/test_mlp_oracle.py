"""Pin of the MLP oracle: its analytic gradient equals central finite
differences of its loss."""
import numpy as np

from oracle import mlp_oracle as M


def test_mlp_oracle_gradient_vs_finite_differences():
    rng = np.random.default_rng(0)
    p = rng.normal(0, 0.3, M.NPARAM)
    X = rng.normal(0, 1, (37, M.NIN))
    t = rng.normal(0, 1, 37)
    _, g = M.loss_grad(p, X, t)
    h = 1e-6
    idx = rng.choice(M.NPARAM, 200, replace=False)
    for i in idx:
        e = np.zeros(M.NPARAM)
        e[i] = h
        fd = (M.loss(p + e, X, t) - M.loss(p - e, X, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_mlp_oracle_shapes():
    assert M.NPARAM == 64 * 11 + 64 + 64 * 64 + 64 + 64 + 1
