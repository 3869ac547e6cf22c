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


def test_adam_oracle_first_step_is_sign_step():
    """From zero moments the bias-corrected moments are g and g^2, so the first
    step moves every parameter by lr * g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    p, g = rng.normal(0, 1, 50), rng.normal(0, 1, 50)
    p1, m1, v1 = M.adam_step(p, g, np.zeros(50), np.zeros(50), 1, lr=1e-2, eps=1e-8)
    assert np.allclose(p1, p - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m1, 0.1 * g, rtol=1e-15) and np.allclose(v1, 0.001 * g * g, rtol=1e-13)


def test_adam_oracle_constant_gradient():
    """A constant gradient keeps mhat = g and vhat = g^2 at every step (the bias
    factors undo the moving averages exactly), so k steps move by
    k lr g / (|g| + eps); the moments are (1 - beta^k) g and (1 - beta^k) g^2."""
    rng = np.random.default_rng(3)
    p0, g = rng.normal(0, 1, 20), rng.normal(0, 1, 20)
    p, m, v = p0.copy(), np.zeros(20), np.zeros(20)
    b1, b2, lr, eps = 0.8, 0.95, 3e-3, 1e-6
    for k in range(1, 8):
        p, m, v = M.adam_step(p, g, m, v, k, lr=lr, beta1=b1, beta2=b2, eps=eps)
        assert np.allclose(m, (1 - b1 ** k) * g, rtol=1e-13, atol=1e-16)
        assert np.allclose(v, (1 - b2 ** k) * g * g, rtol=1e-13, atol=1e-16)
        assert np.allclose(p, p0 - k * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-14)


def test_adam_oracle_zero_gradient_decays_moments_only():
    """With g = 0 the moments decay by beta and the step uses the decayed
    moments' bias-corrected ratio."""
    m0, v0 = np.array([0.5, -0.2]), np.array([0.04, 0.01])
    p1, m1, v1 = M.adam_step(np.zeros(2), np.zeros(2), m0, v0, 3, lr=0.1, beta1=0.5, beta2=0.75, eps=0.0)
    assert np.allclose(m1, 0.5 * m0) and np.allclose(v1, 0.75 * v0)
    mh, vh = m1 / (1 - 0.5 ** 3), v1 / (1 - 0.75 ** 3)
    assert np.allclose(p1, -0.1 * mh / np.sqrt(vh))
