"""Pins for the stage solvers (Secs. 3.2, 4.2) and for whole HBPC steps of the
DGSEM: brute-force dense linear algebra on tiny meshes, exact block-inverse
identities of BJ_ext, linear-problem closed forms, conservation and the exact
solution of periodic advection."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.dgsem import DGSEM, Mesh
from oracle.equations import Advection, Burgers, Euler
from oracle.hbpc import hbpc_step
from oracle.solvers import BJExt, GMRESError, NewtonError, StageSolver, dg_hbpc_step, gmres
from paper_2109_04804_amd import inputs


def tiny_euler(N=2, n=2, beta=2.0):
    """A weak vortex (positive pressure at every trace) on a 2x2 mesh."""
    dg = DGSEM(Mesh(2, [n, n], [10.0, 10.0]), N, Euler(2, 1.4, 1.0), flux="rusanov")
    X = dg.node_coords()
    w = inputs.isentropic_vortex(X[0], X[1], 4.3, 5.6, beta)
    return dg, w


def advection_c1():
    dg = DGSEM(Mesh(1, [16], [1.0]), 3, Advection(1, [1.0]), nodes="lobatto", flux="upwind")
    x = dg.node_coords()[0]
    return dg, inputs.advection_sine(x), x


def test_gmres_matches_direct_solve():
    rng = np.random.default_rng(0)
    n = 60
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n)
    M = lambda v: v / 4.0
    x, its = gmres(lambda v: A @ v, b, M, 1e-12, 10, 1000)
    assert np.linalg.norm(x - np.linalg.solve(A, b)) < 1e-10 * np.linalg.norm(x)
    assert its > 10                              # restarted at least once
    with pytest.raises(GMRESError):
        gmres(lambda v: A @ v, b, M, 1e-12, 10, 3)


def test_jvp_equals_complex_step_jacobian():
    """the extended Jacobian of Eq. nonlinear_eqsys (JVP) equals dG/dX
    obtained column by column with the complex step on a 2x2, N = 2 Euler mesh."""
    dg, w = tiny_euler()
    n = dg.ndof
    rng = np.random.default_rng(1)
    sig = dg.r1(w) + 0.01 * rng.standard_normal(w.shape)
    b = w + 0.01 * rng.standard_normal(w.shape)
    a1dt, bc = 0.25 * 0.1, 0.1 ** 2 / 48
    h = 1e-30
    for col in list(range(0, 2 * n, 17)):
        X = np.zeros(2 * n, dtype=complex)
        X[col] = 1j * h
        wc = w.astype(complex) + X[:n].reshape(w.shape)
        sc = sig.astype(complex) + X[n:].reshape(w.shape)
        R1, R2 = dg.r1_and_r2(wc, sc)
        g1 = wc - a1dt * R1 + bc * R2 - b
        g2 = sc - R1
        cs = np.concatenate([np.imag(g1).ravel(), np.imag(g2).ravel()]) / h
        e = np.zeros(2 * n)
        e[col] = 1.0
        Jw, Js = dg.jvp(w, sig, e[:n].reshape(w.shape), e[n:].reshape(w.shape), a1dt, bc)
        got = np.concatenate([Jw.ravel(), Js.ravel()])
        assert np.abs(got - cs).max() < 1e-12 * (1 + np.abs(cs).max())


def test_block_inverse_identities():
    """P_i = [[A, B], [C, I]] with A = I - a1dt K, B = bcoef K, C = -K;
    A B = B A, and the D, E, F, G blocks invert P exactly (Sec. 3.2.3)."""
    dg, w = tiny_euler()
    a1dt, bc = 0.1, 0.1 ** 2 / 2
    pc = BJExt(dg, w, a1dt, bc)
    K = pc.K
    I = np.eye(K.shape[1])
    for i in range(K.shape[0]):
        A, B = I - a1dt * K[i], bc * K[i]
        assert np.abs(A @ B - B @ A).max() < 1e-12 * np.abs(A @ B).max()
    rng = np.random.default_rng(2)
    n = dg.ndof
    X = rng.standard_normal(2 * n)
    vw, vs = X[:n].reshape(K.shape[0], -1), X[n:].reshape(K.shape[0], -1)
    PXw = np.stack([(I - a1dt * K[i]) @ vw[i] + bc * K[i] @ vs[i] for i in range(K.shape[0])])
    PXs = np.stack([-K[i] @ vw[i] + vs[i] for i in range(K.shape[0])])
    back = pc.apply(np.concatenate([PXw.ravel(), PXs.ravel()]))
    assert np.linalg.norm(back - X) < 1e-11 * np.linalg.norm(X)


def test_bjext_is_exact_for_element_decoupled_linear_problem():
    """With a linear flux and no neighbour coupling BJ_ext is the exact inverse:
    central flux with a = 0 in one direction has no coupling; use advection with
    a = 0 (R1 = 0, K = 0): P = J = identity blocks, GMRES converges in 1 iteration."""
    dg = DGSEM(Mesh(2, [3, 3], [1.0, 1.0]), 2, Advection(2, [0.0, 0.0]), flux="central")
    w = inputs.random_field((dg.mesh.n_elem, 1, dg.nnode), 0)
    sol = StageSolver(dg, newton_rtol=1e-12, gmres_rtol=1e-12)
    sol.solve(w + 1.0, 0.1, 0.01, w)
    assert sol.log[-1]["gmres"][0] == 1


def test_dense_newton_equals_gmres_newton():
    """a stage solve by Newton with dense LU and by Newton-GMRES(BJ_ext)
    agree to the solver tolerance (tiny 2-D Euler mesh)."""
    dg, w = tiny_euler(N=1)
    b = w + 0.05 * dg.r1(w)
    a1dt, bc = 0.25 * 0.2, 0.2 ** 2 / 48
    W1 = StageSolver(dg, newton_rtol=1e-13, linear="dense").solve(b, a1dt, bc, w)
    s2 = StageSolver(dg, newton_rtol=1e-13, gmres_rtol=1e-10, gmres_restart=60)
    W2 = s2.solve(b, a1dt, bc, w)
    assert np.linalg.norm(W1 - W2) < 1e-11 * np.linalg.norm(W1)
    # the converged W solves the stage equation g(W) = b with sigma = R1(W)
    g = W2 - a1dt * dg.r1(W2) + bc * dg.r2(W2) - b
    assert np.linalg.norm(g) < 1e-10 * np.linalg.norm(b)


def test_newton_stops_at_rounding_floor():
    """With an unreachable relative tolerance and no absolute one, Newton still ends, by
    the rounding-floor test (residual stalled, update at the state's rounding level),
    within a few iterations, at the root of a tightly converged dense-LU solve."""
    dg, w = tiny_euler(N=1)
    b = w + 0.05 * dg.r1(w)
    a1dt, bc = 0.25 * 0.2, 0.2 ** 2 / 48
    ref = StageSolver(dg, newton_rtol=1e-13, linear="dense").solve(b, a1dt, bc, w)
    s = StageSolver(dg, newton_rtol=1e-30, newton_atol_dw=0.0, linear="dense")
    W = s.solve(b, a1dt, bc, w)
    assert s.log[-1]["floor_stop"] and 2 <= s.log[-1]["newton"] < 10
    assert np.linalg.norm(W - ref) < 1e-13 * np.linalg.norm(ref)
    # a tolerance that is reached ends the solve before the floor
    s2 = StageSolver(dg, newton_rtol=1e-6, linear="dense")
    s2.solve(b, a1dt, bc, w)
    assert not s2.log[-1]["floor_stop"]


def test_fd_jvp_within_fd_error_bound():
    """Eq. MatrixFree_nonlinear agrees with the exact JVP to O(sqrt(eps_mach))."""
    dg, w = tiny_euler()
    sig = dg.r1(w)
    rng = np.random.default_rng(4)
    dX = rng.standard_normal(2 * dg.ndof)
    a1dt, bc = 0.1, 0.005
    exact = StageSolver(dg).jacobian_op(w, sig, a1dt, bc)(dX)
    fd = StageSolver(dg, jvp="fd").jacobian_op(w, sig, a1dt, bc)(dX)
    assert np.linalg.norm(fd - exact) < 1e-6 * np.linalg.norm(exact)


def test_linear_step_is_matrix_rational_function():
    """for 1-D advection one HBPC(6,3) step with Newton-GMRES(BJ_ext)
    equals the same step taken with exact dense solves of the stage systems."""
    dg, w, x = advection_c1()
    n = dg.ndof
    L = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        L[:, c] = dg.r1(e.reshape(w.shape)).ravel()
    I = np.eye(n)
    ref = hbpc_step(w.ravel(), 0.05, 6, 3, lambda v: L @ v, lambda v: L @ (L @ v),
                    lambda b, a1dt, bc, g: np.linalg.solve(I - a1dt * L + bc * (L @ L), b))
    sol = StageSolver(dg, newton_rtol=1e-12, gmres_rtol=1e-11, gmres_restart=128)
    got = dg_hbpc_step(dg, w, 0.05, 6, 3, sol)
    assert np.linalg.norm(got.ravel() - ref) < 1e-11 * np.linalg.norm(ref)


def test_central_flux_hbpc4_conserves_energy():
    """with the central flux L is skew in the DG mass inner product and the
    HBPC(4,k) step is the (2,2)-Pade map, so sum J omega w^2 is conserved."""
    dg = DGSEM(Mesh(1, [16], [1.0]), 3, Advection(1, [1.0]), nodes="lobatto", flux="central")
    x = dg.node_coords()[0]
    w = inputs.advection_sine(x)
    Wq = dg.quad_weights()
    e0 = np.sum(Wq * w[:, 0] ** 2)
    sol = StageSolver(dg, newton_rtol=1e-13, linear="dense")
    u = w
    for _ in range(3):
        u = dg_hbpc_step(dg, u, 0.05, 4, 2, sol)
    assert abs(np.sum(Wq * u[:, 0] ** 2) - e0) < 1e-13 * e0


def test_constant_state_step_takes_no_newton_iterations():
    """At step level: a constant state is unchanged by an HBPC step."""
    dg = DGSEM(Mesh(2, [3, 3], [10.0, 10.0]), 3, Euler(2), flux="rusanov")
    w = np.zeros((9, 4, 16))
    w[:, 0], w[:, 1], w[:, 2], w[:, 3] = 1.0, 0.3, 0.2, 2.6
    sol = StageSolver(dg)
    u = dg_hbpc_step(dg, w, 0.1, 6, 2, sol)
    assert np.abs(u - w).max() < 1e-13
    assert all(s["newton"] == 0 for s in sol.log)


def test_mass_conservation_dense_and_gmres():
    """sum J omega w per variable is conserved by a step to round-off with
    the dense Newton (1-D viscous Burgers), and to the Newton tolerance with
    Newton-GMRES (2-D Euler)."""
    dg = DGSEM(Mesh(1, [4], [2 * np.pi]), 3, Burgers(1, 0.05), flux="lf", lam=1.0)
    x = dg.node_coords()[0]
    w = (0.5 + 0.3 * np.sin(x))[:, None, :]
    m0 = dg.integral(w)
    u = dg_hbpc_step(dg, w, 0.2, 6, 1, StageSolver(dg, newton_rtol=1e-12, linear="dense"))
    assert np.abs(dg.integral(u) - m0).max() < 1e-13 * np.abs(m0).max()
    assert np.abs(u - w).max() > 1e-3
    dg, w = tiny_euler()
    m0 = dg.integral(w)
    u = dg_hbpc_step(dg, w, 0.2, 6, 1, StageSolver(dg, newton_rtol=1e-10, gmres_rtol=1e-4))
    assert np.abs(dg.integral(u) - m0).max() < 1e-8 * np.abs(m0).max()


def test_advection_step_against_exact_solution():
    """20 HBPC(6,3) steps of dt = 0.05 on the 1-D advection workload stay
    within the spatial error of the N = 3, 16-element discretisation of
    sin(2 pi (x - t)) (error at t = 1 vs. the semi-discrete bound)."""
    dg, w, x = advection_c1()
    sol = StageSolver(dg, newton_rtol=1e-12, gmres_rtol=1e-10, gmres_restart=128)
    u = w
    for _ in range(20):
        u = dg_hbpc_step(dg, u, 0.05, 6, 3, sol)
    err = np.abs(u[:, 0] - np.sin(2 * np.pi * (x - 1.0))).max()
    assert err < 1e-4


def test_newton_failure_is_reported():
    dg, w = tiny_euler()
    b = w + 0.3 * dg.r1(w)
    with pytest.raises(NewtonError):
        StageSolver(dg, newton_rtol=1e-15, newton_atol_dw=0.0, newton_maxit=1, linear="dense").solve(
            b, 0.05, 0.001, w)
