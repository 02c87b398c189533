"""Pins for the DGSEM operators R1_h, R2_h, the Hessian term and the local
Jacobian (Sec. 3.1, Eq. nonlinear_eqsys).  Each check compares the oracle with
something it does not compute itself: exact solutions of the PDE, invariants
(conservation, free stream), closed forms for linear fluxes, complex-step
derivatives, textbook eigenvalues of the Euler flux Jacobian."""
import numpy as np
import pytest

from oracle import jets
from oracle.dgsem import DGSEM, Mesh
from oracle.equations import Advection, Burgers, Euler, numerical_flux
from paper_2109_04804_amd import inputs


def make(kind, n=4, N=3, nodes="gauss", flux=None):
    if kind == "adv1":
        return DGSEM(Mesh(1, [n], [1.0]), N, Advection(1, [1.0]), nodes=nodes, flux=flux or "upwind")
    if kind == "adv2":
        return DGSEM(Mesh(2, [n, n + 1], [2.0, 2.0], [-1, -1]), N, Advection(2, [0.3, -0.7]), nodes=nodes,
                     flux=flux or "upwind")
    if kind == "adv3":
        return DGSEM(Mesh(3, [n, n, n], [1.0, 1.0, 1.0]), N, Advection(3, [0.3, 0.5, -0.2]), nodes=nodes,
                     flux=flux or "upwind")
    if kind == "burgers":
        return DGSEM(Mesh(2, [n, n], [2 * np.pi, 2 * np.pi]), N, Burgers(2, 0.01), nodes=nodes,
                     flux=flux or "lf", lam=1.0)
    if kind == "burgers1":
        return DGSEM(Mesh(1, [n], [2 * np.pi]), N, Burgers(1, 0.05), nodes=nodes, flux=flux or "lf", lam=1.0)
    if kind == "euler2":
        return DGSEM(Mesh(2, [n, n], [10.0, 10.0]), N, Euler(2, 1.4, 1.0), nodes=nodes, flux=flux or "rusanov")
    if kind == "euler2_lfl":   # Eq. Riemann as printed with the Euler set-up's diagonal lambda
        return DGSEM(Mesh(2, [n, n], [10.0, 10.0]), N, Euler(2, 1.4, 0.5), nodes=nodes, flux=flux or "lf_literal")
    if kind == "euler3":
        return DGSEM(Mesh(3, [n, n, n], [2 * np.pi] * 3), N, Euler(3, 1.4, 0.1), nodes=nodes,
                     flux=flux or "rusanov")
    raise ValueError(kind)


def smooth_state(dg, seed=0):
    """A smooth, physically admissible state for each equation."""
    X = dg.node_coords()
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0, 2 * np.pi, size=4)
    if dg.nvar == 1:
        s = sum(np.sin(2 * np.pi * x / dg.mesh.length[m] + ph[m]) for m, x in enumerate(X))
        return (0.5 + 0.2 * s)[:, None, :]
    if dg.d == 2:
        xc, yc, beta = 5.0 + ph[0] / 3, 5.0 - ph[1] / 3, 5.0
        return inputs.isentropic_vortex(X[0], X[1], xc, yc, beta)
    # shifted so that no face sits on a symmetry plane of the Taylor-Green field
    # (there lambda_L = lambda_R to rounding, a tie of the Rusanov max that the
    # complex step cannot resolve); v_z = 0 exactly is a kink of |v_z| for the
    # same reason, so a smooth v_z is added
    w = inputs.taylor_green(X[0] + ph[0], X[1] + ph[2], X[2] + ph[3], eps=dg.eq.eps)
    w[:, 3, :] += 0.05 * np.sin(X[0] + X[2] + ph[1])
    return w


def rel(a, b):
    return np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


ALL = ["adv1", "adv2", "adv3", "burgers", "burgers1", "euler2", "euler2_lfl", "euler3"]


# ------------------------------------------------------------------
@pytest.mark.parametrize("kind", ALL)
@pytest.mark.parametrize("nodes", ["gauss", "lobatto"])
def test_free_stream(kind, nodes):
    """a constant state is a steady solution, R1 = 0 (to round-off)."""
    dg = make(kind, n=3, nodes=nodes)
    w = np.zeros((dg.mesh.n_elem, dg.nvar, dg.nnode))
    const = [1.3, 0.4, -0.3, 0.2, 3.0][: dg.nvar] if dg.nvar > 1 else [0.7]
    if dg.nvar == dg.d + 2:
        const = [1.3] + [0.4, -0.3, 0.2][: dg.d] + [3.0]
    for v in range(dg.nvar):
        w[:, v, :] = const[v]
    assert np.abs(dg.r1(w)).max() < 1e-12


# ------------------------------------------------------------------
@pytest.mark.parametrize("kind", ALL)
def test_conservation(kind):
    """sum_e J sum omega (.) = 0 for R1, R2 and the Hessian term on periodic meshes."""
    dg = make(kind, n=3)
    w = smooth_state(dg)
    rng = np.random.default_rng(1)
    sig = rng.standard_normal(w.shape) * 0.01
    dw = rng.standard_normal(w.shape) * 0.01
    scale = np.abs(dg.r1(w)).max() + 1.0
    for val in (dg.r1(w), dg.r2(w, sig), dg.hessian_term(w, sig, dw)):
        assert np.abs(dg.integral(val)).max() < 1e-12 * scale * np.prod(dg.mesh.length)


# ------------------------------------------------------------------
@pytest.mark.parametrize("nodes", ["gauss", "lobatto"])
def test_advection_spectral_convergence(nodes):
    """R1 of the sine interpolant -> -a u_x; the pointwise error of this
    derivative falls like h^N (N = 3)."""
    errs = []
    for n in (4, 8, 16):
        dg = make("adv1", n=n, N=3, nodes=nodes)
        x = dg.node_coords()[0]
        w = np.sin(2 * np.pi * x)[:, None, :]
        errs.append(np.abs(dg.r1(w)[:, 0] + 2 * np.pi * np.cos(2 * np.pi * x)).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() > 2.5 and rates[-1] > 2.85, (errs, rates)


@pytest.mark.parametrize("flux", ["rusanov", "lf_literal"])
def test_euler_density_wave_first_and_second_time_derivative(flux):
    """Euler: on the density wave rho = 1 + 0.3 sin(pi (x + y - 2 a t)),
    v = (a, a), p = 1 the exact w_t and w_tt are known; R1 -> w_t and
    R2(w, R1(w)) -> w_tt spectrally (the latter checks Eq. DGSEM_wtt), with
    the Rusanov flux and with Eq. Riemann as printed (diagonal lambda)."""
    a = 0.3
    errs1, errs2 = [], []
    for n in (8, 16):
        dg = DGSEM(Mesh(2, [n, n], [2.0, 2.0], [-1.0, -1.0]), 4, Euler(2, 1.4, 1.0), flux=flux)
        X = dg.node_coords()
        w = inputs.density_wave(X, a=a)
        s = np.pi * (X[0] + X[1])
        rho_t = -2 * a * 0.3 * np.pi * np.cos(s)
        rho_tt = -(2 * a) ** 2 * 0.3 * np.pi ** 2 * np.sin(s)
        fac = np.array([1.0, a, a, 0.5 * (2 * a * a)])
        wt = rho_t[:, None, :] * fac[None, :, None]
        wtt = rho_tt[:, None, :] * fac[None, :, None]
        errs1.append(rel(dg.r1(w), wt))
        errs2.append(rel(dg.r2(w), wtt))
    # the printed flux carries twice the textbook dissipation: a larger constant, the same rates
    assert errs1[-1] < 1e-4 and errs2[-1] < (5e-3 if flux == "rusanov" else 1e-2)
    assert errs1[0] / errs1[1] > 12 and errs2[0] / errs2[1] > 6


def test_burgers_viscous_rhs():
    """BR1: u = 0.5 + 0.25 sin(x+y): u_t = -u (u_x + u_y) + nu Laplace u,
    and the viscous part alone, (R1_nu - R1_0)/nu, converges to Laplace u."""
    errs, errs_lap = [], []
    for n in (8, 16):
        dg = make("burgers", n=n, N=4)
        dg0 = DGSEM(dg.mesh, 4, Burgers(2, 0.0), flux="lf", lam=1.0)
        X = dg.node_coords()
        u = 0.5 + 0.25 * np.sin(X[0] + X[1])
        ut = -u * 0.5 * np.cos(X[0] + X[1]) - 0.01 * 0.5 * np.sin(X[0] + X[1])
        r = dg.r1(u[:, None, :])[:, 0]
        errs.append(rel(r, ut))
        lap = (r - dg0.r1(u[:, None, :])[:, 0]) / 0.01
        errs_lap.append(rel(lap, -0.5 * np.sin(X[0] + X[1])))
    assert errs[-1] < 1e-5 and errs[0] / errs[1] > 12
    assert errs_lap[-1] < 1e-4 and errs_lap[0] / errs_lap[1] > 6


def test_vortex_translation():
    """the isentropic vortex translates with the background flow, so R1 of
    the exact solution approaches its time derivative (central difference in
    t) under refinement."""
    errs = []
    for n in (8, 16):
        dg = make("euler2", n=n, N=5)
        X = dg.node_coords()
        xc, yc, beta = 5.0, 5.0, 5.0
        w = inputs.isentropic_vortex(X[0], X[1], xc, yc, beta)
        d = 1e-4
        wt = (inputs.isentropic_vortex(X[0], X[1], xc, yc, beta, t=d)
              - inputs.isentropic_vortex(X[0], X[1], xc, yc, beta, t=-d)) / (2 * d)
        errs.append(rel(dg.r1(w), wt))
    assert errs[-1] < 3e-3 and errs[0] / errs[1] > 8, errs


# ------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["adv1", "adv2", "adv3"])
def test_linear_flux_closed_forms(kind):
    """for a linear flux R2(w, s) = R1(s) and the Hessian term is 0 (Sec. 3.2.1)."""
    dg = make(kind, n=3)
    rng = np.random.default_rng(3)
    w = rng.standard_normal((dg.mesh.n_elem, 1, dg.nnode))
    s = rng.standard_normal(w.shape)
    assert rel(dg.r2(w, s), dg.r1(s)) < 1e-13
    assert np.abs(dg.hessian_term(w, s, rng.standard_normal(w.shape))).max() == 0.0


# ------------------------------------------------------------------
@pytest.mark.parametrize("kind", ALL)
def test_complex_step_r2_and_hessian(kind):
    """Im R1(w + i h v)/h = R2(w, v) and Im R2(w + i h dw, s)/h = Hessian term."""
    dg = make(kind, n=3)
    w = smooth_state(dg, seed=5)
    rng = np.random.default_rng(6)
    v = rng.standard_normal(w.shape) * np.abs(w).mean()
    h = 1e-30
    cs = np.imag(dg.r1_complex(w + 1j * h * v)) / h
    assert rel(dg.r2(w, v), cs) < 1e-12
    s = rng.standard_normal(w.shape) * np.abs(w).mean()
    dw = rng.standard_normal(w.shape) * np.abs(w).mean()
    R = dg._r1_vars(dg._jet(np.asarray(w + 1j * h * dw, dtype=complex), s.astype(complex)))
    cs2 = np.imag(dg.to_flat([jets.part(x, "b") for x in R])) / h
    T3 = dg.hessian_term(w, s, dw)
    if np.abs(cs2).max() == 0:
        assert np.abs(T3).max() == 0
    else:
        assert rel(T3, cs2) < 1e-11


def test_rusanov_tie_rule_matches_complex_step_branch():
    """at lambda_L = lambda_R the derivative takes the L branch, as the
    complex step with real-part branching does."""
    eq = Euler(2)
    wL = [np.array([1.0]), np.array([0.3]), np.array([0.1]), np.array([2.5])]
    wR = [x.copy() for x in wL]
    wR[2] = -wR[2]                                       # same |v_1| and c: a tie
    rng = np.random.default_rng(0)
    dL = [rng.standard_normal(1) for _ in range(4)]
    dR = [rng.standard_normal(1) for _ in range(4)]
    jL = [jets.HD(a, b) for a, b in zip(wL, dL)]
    jR = [jets.HD(a, b) for a, b in zip(wR, dR)]
    f = numerical_flux(eq, "rusanov", 0, jL, jR, 0)
    h = 1e-30
    cL = [a + 1j * h * b for a, b in zip(wL, dL)]
    cR = [a + 1j * h * b for a, b in zip(wR, dR)]
    fc = numerical_flux(eq, "rusanov", 0, cL, cR, 0)
    for v in range(4):
        assert abs(f[v].b[0] - fc[v].imag[0] / h) < 1e-13


# ------------------------------------------------------------------ Euler flux
@pytest.mark.parametrize("d,eps", [(2, 1.0), (3, 0.1), (2, 0.3)])
def test_euler_flux_jacobian_eigenvalues(d, eps):
    """The eps-scaled Euler flux Jacobian A_m has eigenvalues v_m (d-fold) and
    v_m +- c/eps, c = sqrt(gamma p / rho): the wave speed used by Rusanov."""
    eq = Euler(d, 1.4, eps)
    rng = np.random.default_rng(d)
    rho = 1.2
    vel = rng.uniform(-0.5, 0.5, d)
    p = 0.9
    E = p / 0.4 + 0.5 * eps ** 2 * rho * vel @ vel
    w = np.array([rho, *(rho * vel), E])
    for m in range(d):
        A = np.zeros((d + 2, d + 2))
        for u in range(d + 2):
            st = [jets.HD(np.array([w[k]]), np.array([1.0 if k == u else 0.0])) for k in range(d + 2)]
            F = eq.flux(st, m)
            A[:, u] = [F[k].b[0] for k in range(d + 2)]
        ev = np.sort(np.linalg.eigvals(A).real)
        c = np.sqrt(1.4 * p / rho)
        ref = np.sort([vel[m]] * d + [vel[m] - c / eps, vel[m] + c / eps])
        assert np.allclose(ev, ref, atol=1e-10)


@pytest.mark.parametrize("d,eps", [(2, 1.0), (2, 0.3), (3, 0.1), (3, 1.0)])
def test_wave_speed_is_flux_jacobian_spectral_radius(d, eps):
    """Rusanov's lambda on one side, Euler.wave_speed(w, m), equals the
    spectral radius of the flux Jacobian A_m(w) built column by column from
    jets (Eq. Riemann with the eps-scaled system of Eq. Euler).  The states
    include negative velocity components, so a missing |.|, a missing square
    root or c/eps^2 in place of c/eps changes the value."""
    eq = Euler(d, 1.4, eps)
    rng = np.random.default_rng(100 + d)
    for trial in range(4):
        rho = rng.uniform(0.5, 2.0)
        vel = rng.uniform(-0.8, 0.8, d)
        vel[trial % d] = -abs(vel[trial % d]) - 0.1
        p = rng.uniform(0.3, 3.0)
        E = p / 0.4 + 0.5 * eps ** 2 * rho * vel @ vel
        w = np.array([rho, *(rho * vel), E])
        for m in range(d):
            A = np.zeros((d + 2, d + 2))
            for u in range(d + 2):
                st = [jets.HD(np.array([w[k]]), np.array([1.0 if k == u else 0.0])) for k in range(d + 2)]
                F = eq.flux(st, m)
                A[:, u] = [F[k].b[0] for k in range(d + 2)]
            radius = np.abs(np.linalg.eigvals(A)).max()
            lam = eq.wave_speed([np.array([x]) for x in w], m)[0]
            assert abs(lam - radius) <= 1e-10 * radius, (trial, m, lam, radius)


def test_upwind_flux_is_upwind():
    eq = Advection(1, [0.7])
    f = numerical_flux(eq, "upwind", 0, [np.array([2.0])], [np.array([-5.0])], 0)
    assert f[0][0] == pytest.approx(0.7 * 2.0)


# ------------------------------------------------------------------ local Jacobian
@pytest.mark.parametrize("kind", ["adv2", "euler2", "burgers1"])
def test_local_jacobian_is_diagonal_block(kind):
    """K_i (neighbour data constant) equals the diagonal block of the full
    Jacobian, obtained column by column with the complex step, on a mesh with
    3 elements per direction (own and neighbour elements distinct).  For BR1
    the full block also holds the path through the neighbours' liftings, which
    K_i leaves out by definition; there only the inviscid part is compared."""
    if kind == "burgers1":
        dg = DGSEM(Mesh(1, [3], [2 * np.pi]), 3, Burgers(1, 0.0), flux="lf", lam=1.0)
    else:
        dg = make(kind, n=3, N=2)
    w = smooth_state(dg, seed=2)
    K = dg.local_jacobian(w)
    nE, ne = dg.mesh.n_elem, dg.nvar * dg.nnode
    h = 1e-30
    for col in range(ne):
        for e in range(nE):
            pert = np.zeros((nE, ne), dtype=complex)
            pert[e, col] = 1j * h
            R = dg.r1_complex(w + pert.reshape(w.shape)).reshape(nE, ne)
            assert np.abs(np.imag(R[e]) / h - K[e, :, col]).max() < 1e-10 * (1 + np.abs(K).max())
        if col > 3:
            break
