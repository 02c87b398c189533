"""Physical and numerical fluxes (Eqs. hyperbolic, Euler, Riemann).

All functions take the state as a list of per-variable arrays (plain NumPy
arrays, complex arrays for complex-step checks, or jets.HD) so that the same
definition yields values, exact directional derivatives and complex-step
derivatives.

Numerical flux (Eq. Riemann, read with the textbook factor 1/2 on the
dissipation, which makes lambda = |a.n| the exact upwind flux):

    f*(wL, wR; n) = 1/2 (F(wL) + F(wR)).n + 1/2 lambda (wL - wR)

On the Cartesian meshes used here n = +e_m; wL is the trace of the element on
the minus side of the face, wR the one on the plus side.

lambda by flux type:
  central   0
  upwind    |a.n|                                (advection, Sec. 4.1.1)
  lf        a global constant                     (the paper's global LF)
  rusanov   max(|vL.n| + cL/eps, |vR.n| + cR/eps) (state dependent, c = sqrt(gamma p / rho))

The Euler system is the eps-scaled form of Eq. Euler: momentum flux carries
p / eps^2 and p = (gamma - 1)(E - eps^2/2 rho |v|^2); eps = 1 is textbook Euler.
"""
import numpy as np
from . import jets


class Advection:
    """w_t + div(a w) = 0, scalar."""

    def __init__(self, dim, adv):
        self.dim = dim
        self.nvar = 1
        self.a = [float(adv[m]) for m in range(dim)]

    def flux(self, w, m):
        return [w[0] * self.a[m]]

    def is_linear(self):
        return True


class Burgers:
    """u_t + div(u^2/2 * (1,..,1)) = nu Laplace(u); inviscid part only here.

    The viscous flux -nu q (q the BR1-lifted gradient) is added by the DGSEM
    operator, which owns the lifting."""

    def __init__(self, dim, nu):
        self.dim = dim
        self.nvar = 1
        self.nu = float(nu)

    def flux(self, w, m):
        return [0.5 * w[0] * w[0]]

    def is_linear(self):
        return False


class Euler:
    """eps-scaled compressible Euler, w = (rho, rho v_1..rho v_d, E)."""

    def __init__(self, dim, gamma=1.4, eps=1.0):
        self.dim = dim
        self.nvar = dim + 2
        self.gamma = float(gamma)
        self.eps = float(eps)

    def pressure(self, w):
        d = self.dim
        rho, E = w[0], w[d + 1]
        mom2 = w[1] * w[1]
        for k in range(2, d + 1):
            mom2 = mom2 + w[k] * w[k]
        return (self.gamma - 1.0) * (E - 0.5 * self.eps ** 2 * mom2 / rho)

    def flux(self, w, m):
        d = self.dim
        rho, E = w[0], w[d + 1]
        p = self.pressure(w)
        vm = w[1 + m] / rho
        out = [w[1 + m]]
        for k in range(d):
            fk = w[1 + k] * vm
            if k == m:
                fk = fk + p / self.eps ** 2
            out.append(fk)
        out.append((E + p) * vm)
        return out

    def wave_speed(self, w, m):
        """|v_m| + c / eps with c = sqrt(gamma p / rho)."""
        rho = w[0]
        p = self.pressure(w)
        c = jets.sqrt(p * self.gamma / rho)
        return jets.absval(w[1 + m] / rho) + c / self.eps

    def is_linear(self):
        return False


class NavierStokes(Euler):
    """Compressible Navier-Stokes (Sec. 5.1, Eq. NavierStokes) on the eps-scaled Euler
    system: w_t + div(F(w) - F^v(w, grad w)) = 0 with the viscous flux as printed,

        F^v = (0, tau, tau.v + q),
        tau = mu (grad v + grad v^T - 2/3 (div v) I),   q = kappa grad T,
        kappa = c_p mu / Pr,  c_p = R gamma / (gamma - 1),  R = 1 / (gamma eps^2),
        p = rho R T,  Pr = 0.72 by default.

    The viscous flux depends on w and on the gradients d = grad w_grad of
    w_grad = (v_1, .., v_d, T) (Eq. LiftingEq), which the DGSEM operator lifts."""

    def __init__(self, dim, gamma=1.4, eps=1.0, mu=1e-3, Pr=0.72):
        super().__init__(dim, gamma, eps)
        self.mu = float(mu)
        self.Pr = float(Pr)
        self.R = 1.0 / (self.gamma * self.eps ** 2)
        self.cp = self.R * self.gamma / (self.gamma - 1.0)
        self.kappa = self.cp * self.mu / self.Pr
        self.ngrad = dim + 1

    def grad_vars(self, w):
        """w_grad = (v_1, .., v_d, T) with T = p / (rho R)."""
        rho = w[0]
        out = [w[1 + k] / rho for k in range(self.dim)]
        out.append(self.pressure(w) / (rho * self.R))
        return out

    def viscous_flux(self, w, g, m):
        """F^v_m(w, d), g[k][j] = d w_grad_k / d x_j."""
        d = self.dim
        rho = w[0]
        vel = [w[1 + k] / rho for k in range(d)]
        div = g[0][0]
        for k in range(1, d):
            div = div + g[k][k]
        tau = []
        for i in range(d):     # tau_{i m}
            t = (g[i][m] + g[m][i]) * self.mu
            if i == m:
                t = t - div * (2.0 / 3.0 * self.mu)
            tau.append(t)
        energy = g[d][m] * self.kappa
        for i in range(d):
            energy = energy + tau[i] * vel[i]
        return [rho * 0.0] + tau + [energy]


def numerical_flux(eq, kind, lam_const, wL, wR, m):
    """f* in direction +e_m from the two traces (lists of per-variable arrays)."""
    FL = eq.flux(wL, m)
    FR = eq.flux(wR, m)
    if kind == "central":
        lam = 0.0
    elif kind == "upwind":
        lam = abs(eq.a[m])
    elif kind == "lf":
        lam = float(lam_const)
    elif kind == "rusanov":
        lam = jets.maxval(eq.wave_speed(wL, m), eq.wave_speed(wR, m))
    elif kind == "lf_literal":
        # Eq. Riemann as printed, without the 1/2 on the dissipation, with the diagonal
        # lambda of the Euler set-up (Sec. 4.1.2): 1/eps on density and energy, 1 on momenta
        lam_v = [1.0 / eq.eps] + [1.0] * (eq.nvar - 2) + [1.0 / eq.eps]
        return [0.5 * (FL[v] + FR[v]) + lam_v[v] * (wL[v] - wR[v]) for v in range(eq.nvar)]
    else:
        raise ValueError(kind)
    return [0.5 * (FL[v] + FR[v]) + 0.5 * lam * (wL[v] - wR[v]) for v in range(eq.nvar)]
