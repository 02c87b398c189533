"""Pins for the reference MLP of the learned preconditioner: the manual
backward pass against central finite differences, Adam against its
closed form on a quadratic, and the feature patch layout."""
import numpy as np

from oracle import mlp
from oracle.dgsem import DGSEM, Mesh
from oracle.equations import Euler


def test_backward_matches_central_differences():
    """All seven parameter blocks, through both the gates and the linear path."""
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
    by the patch RMS, state tiles raw, then the logarithms of the two coefficients."""
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
    assert np.allclose(X[0, -2:], np.log([0.1, 0.2]))


def test_round_bf16_ties_and_library():
    u = 2.0 ** -7   # spacing of bfloat16 values in [1, 2)
    cases = {1.0 + u / 2: 1.0,                      # tie -> even (1.0)
             1.0 + 3 * u / 2: 1.0 + 2 * u,          # tie -> even (1 + 2u)
             1.0 + u / 2 + 2.0 ** -20: 1.0 + u,     # above the tie
             -(1.0 + 3 * u / 2): -(1.0 + 2 * u),
             3.0: 3.0, 0.0: 0.0}
    for x, r in cases.items():
        assert mlp.round_bf16(np.array([x]))[0] == r, x
    torch = __import__("pytest").importorskip("torch")
    x = np.random.default_rng(1).standard_normal(10000) * 10.0 ** np.random.default_rng(2).uniform(-20, 20, 10000)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.round_bf16(x), ref)


def test_rounded_operands_backward_is_consistent():
    """With q = round_bf16 the backward pass is the exact gradient of the loss
    whose products take rounded operands only up to the rounding itself: at
    q = identity it equals the plain gradient, and with rounding it stays
    within the BF16 error of the plain one."""
    rng = np.random.default_rng(4)
    n_in, H, n_out, B = 9, 8, 5, 6
    theta = mlp.init_params(n_in, H, n_out, rng) + 0.05 * rng.standard_normal(mlp.n_params(n_in, H, n_out))
    X = rng.standard_normal((B, n_in))
    T = rng.standard_normal((B, n_out))
    l0, g0 = mlp.loss_and_grad(theta, X, T, n_in, H, n_out)
    l1, g1 = mlp.loss_and_grad(theta, X, T, n_in, H, n_out, q=lambda a: a)
    assert l0 == l1 and np.array_equal(g0, g1)
    l2, g2 = mlp.loss_and_grad(theta, X, T, n_in, H, n_out, q=mlp.round_bf16)
    assert abs(l2 - l0) < 0.05 * l0
    assert np.linalg.norm(g2 - g0) < 0.05 * np.linalg.norm(g0)


def test_network_is_linear_in_the_residual():
    """For fixed state features the output is additive and odd in the residual
    features (so P^-1 is a linear map of the Krylov vector)."""
    rng = np.random.default_rng(8)
    n_in, H, n_out, B = 12, 7, 4, 5
    n_r, n_w = mlp.split(n_in)
    assert (n_r, n_w) == (5, 7)
    theta = mlp.init_params(n_in, H, n_out, rng) + 0.1 * rng.standard_normal(mlp.n_params(n_in, H, n_out))
    Xw = rng.standard_normal((B, n_w))
    R1, R2 = rng.standard_normal((B, n_r)), rng.standard_normal((B, n_r))
    f = lambda R: mlp.forward(theta, np.hstack([R, Xw]), n_in, H, n_out)[0]
    assert np.allclose(f(R1 + R2), f(R1) + f(R2), rtol=1e-12, atol=1e-12)
    assert np.allclose(f(-2.5 * R1), -2.5 * f(R1), rtol=1e-12, atol=1e-12)
    assert np.abs(f(np.zeros((B, n_r)))).max() == 0.0


def test_learned_apply_is_linear():
    nelem = [3, 2]
    dg = DGSEM(Mesh(2, nelem, [10.0, 10.0]), 2, Euler(2))
    ne = dg.nvar * dg.nnode
    n_in = 5 * 2 * ne + 2
    rng = np.random.default_rng(9)
    H = 6
    theta = mlp.init_params(n_in, H, ne, rng) + 0.05 * rng.standard_normal(mlp.n_params(n_in, H, ne))
    X = dg.node_coords()
    from paper_2109_04804_amd import inputs
    w = inputs.isentropic_vortex(X[0], X[1], 4.0, 6.0, 3.0)
    v = [rng.standard_normal(w.shape) for _ in range(4)]
    a = mlp.apply_learned(dg, theta, H, w, v[0], v[1], 0.1, 0.01)
    b = mlp.apply_learned(dg, theta, H, w, v[2], v[3], 0.1, 0.01)
    c = mlp.apply_learned(dg, theta, H, w, v[0] - 3 * v[2], v[1] - 3 * v[3], 0.1, 0.01)
    for k in range(2):
        ref = a[k] - 3 * b[k]
        assert np.linalg.norm(c[k] - ref) <= 1e-12 * np.linalg.norm(ref)


def test_schur_structure_with_exact_element_solve_is_bjext():
    """The learned preconditioner's block structure (r~ = v_w - bcoef K v_s,
    dsigma = v_s + K dw) with the network's element solve replaced by the exact
    S_e^-1 r~ reproduces BJ_ext's apply from the paper's D, E, F, G blocks
    (Sec. 3.2.3) to round-off: a wrong sign in r~ or in the back-substitution
    fails it."""
    import scipy.linalg as sla
    from oracle.solvers import BJExt
    from paper_2109_04804_amd import inputs
    for nelem, N in (([3, 2], 2), ([2, 3], 3)):
        dg = DGSEM(Mesh(2, nelem, [10.0, 10.0]), N, Euler(2), flux="rusanov")
        X = dg.node_coords()
        w = inputs.isentropic_vortex(X[0], X[1], 4.0, 6.0, 3.0)
        a1dt, bcoef = 0.3, 0.02
        pc = BJExt(dg, w, a1dt, bcoef)
        nE, ne = dg.mesh.n_elem, dg.nvar * dg.nnode
        K = dg.local_jacobian(w)
        S = [np.eye(ne) - a1dt * K[i] + bcoef * (K[i] @ K[i]) for i in range(nE)]

        def exact(rt):
            rt = np.asarray(rt).reshape(nE, ne)
            return np.array([sla.solve(S[i], rt[i]) for i in range(nE)])
        rng = np.random.default_rng(11)
        for _ in range(2):
            vw, vs = rng.standard_normal(w.shape), rng.standard_normal(w.shape)
            dw, ds = mlp.schur_apply(dg, w, vw, vs, bcoef, exact)
            ref = pc.apply(np.concatenate([vw.ravel(), vs.ravel()]))
            got = np.concatenate([dw.ravel(), ds.ravel()])
            assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)
