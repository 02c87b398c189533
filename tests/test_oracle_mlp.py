"""Pins for the reference MLP of the learned preconditioner: the manual
backward pass against central finite differences (P17), Adam against its
closed form on a quadratic, and the feature patch layout."""
import numpy as np

from oracle import mlp
from oracle.dgsem import DGSEM, Mesh
from oracle.equations import Euler


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    n_in, H, n_out, B = 7, 6, 5, 4
    theta = mlp.init_params(n_in, H, n_out, rng) + 0.01 * rng.standard_normal(mlp.n_params(n_in, H, n_out))
    X = rng.standard_normal((B, n_in))
    T = rng.standard_normal((B, n_out))
    _, g = mlp.loss_and_grad(theta, X, T, n_in, H, n_out)
    h = 1e-6
    fd = np.zeros_like(theta)
    for i in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd[i] = (mlp.loss_and_grad(tp, X, T, n_in, H, n_out)[0] - mlp.loss_and_grad(tm, X, T, n_in, H, n_out)[0]) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-6 * max(1.0, np.abs(fd).max())


def test_adam_closed_form_first_step():
    """First Adam step moves every coordinate by lr * sign(grad) (bias-corrected)."""
    theta = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    t, m, v = mlp.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, 0.1)
    assert np.allclose(t, theta - 0.1 * np.sign(g) * np.abs(g) / (np.abs(g) + 1e-8))


def test_adam_minimises_quadratic():
    theta = np.array([3.0, -1.0])
    m = v = np.zeros(2)
    for t in range(1, 2001):
        g = 2 * theta
        theta, m, v = mlp.adam_step(theta, g, m, v, t, 0.05)
    assert np.abs(theta).max() < 1e-2


def test_feature_layout():
    """Patch order self, -x, +x, -y, +y with periodic wrap; residual tiles scaled
    by the patch RMS, state tiles raw, then the two coefficients."""
    nelem = [3, 2]
    assert mlp.neighbours(nelem, 0) == [2, 1, 3, 3]
    dg = DGSEM(Mesh(2, nelem, [1.0, 1.0]), 2, Euler(2))
    ne = dg.nvar * dg.nnode
    rt = np.arange(6 * ne, dtype=float).reshape(6, ne)
    w = -rt
    X, s = mlp.features(nelem, rt, w, 0.1, 0.2, [4])
    patch = [4, 3, 5, 1, 1]
    r = np.concatenate([rt[p] for p in patch])
    assert np.isclose(s[0], np.sqrt(np.mean(r ** 2)) + 1e-30)
    assert np.allclose(X[0, :5 * ne], r / s[0])
    assert np.allclose(X[0, 5 * ne:10 * ne], np.concatenate([w[p] for p in patch]))
    assert np.allclose(X[0, -2:], [0.1, 0.2])
