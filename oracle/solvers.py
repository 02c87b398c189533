"""Stage solvers: Newton on G(X) = 0, restarted right-preconditioned GMRES,
the BJ_ext preconditioner and a dense direct solve (Secs. 3.2.1-3.2.3, 4.2).

Stopping rules (the paper states relative tolerances without a norm; this
reading uses the Euclidean norm over all coefficients of X = (w, sigma)):
  * Newton stops after iteration r when ||G(X^r)|| <= eps_N ||G(X^0)|| or
    ||dw^r||_2 / sqrt(ndof) <= atol_dw, or (r >= 2) when the residual has
    reached the rounding floor of its FP64 evaluation: ||G(X^r)|| >
    0.5 ||G(X^(r-1))|| with ||dw^r||_2 <= 1e-12 ||w^0||_2 (a corrector stage
    started from an accurate prediction can have eps_N ||G(X^0)|| below that
    floor; the step is then at the state's rounding level).  The paper adds the absolute criterion
    ||dw||_2 <= 1e-12 (Sec. 5.2) because corrector solves start so close to the
    solution that round-off stalls the relative one; it is read per
    coefficient here (1e-12 over the paper's 262,144 coefficients gives
    atol_dw = 1.95e-15), so that it keeps its meaning at every size.  It takes
    no iteration when
    ||G(X^0)|| <= 1e-14 sqrt(len(X)); more than newton_maxit iterations is an
    error.
  * GMRES starts from dX = 0 and stops when ||r_j|| <= eps_G ||r_0||, r_0 = -G;
    it restarts every `restart` iterations; more than gmres_maxit iterations
    per Newton step is an error.
  * Newton initial guesses: X^0 = (guess, R1(guess)), so G2(X^0) = 0.

BJ_ext (Sec. 3.2.3): with K_i the element-local dR1/dw (dgsem.local_jacobian),
A_i = I - a1dt K_i, B_i = bcoef K_i, C_i = -K_i and S_i = A_i - B_i C_i =
I - a1dt K_i + bcoef K_i^2, the inverse of the block-diagonal P has blocks
D = S^-1, E = -B S^-1, F = -C S^-1, G = A S^-1, applied as
P^-1 (vw, vs) = (D vw + E vs, F vw + G vs), S^-1 through an LU factorisation.

BJ^H_ext (Sec. 3.2.3): the same P with the element-local Hessian block
H_i = dR2_i/dw_i (dgsem.local_hessian, at the state (w, sigma)) kept in
A^H_i = I - a1dt K_i + bcoef H_i.  S^H_i = A^H_i - B_i C_i =
I - a1dt K_i + bcoef (H_i + K_i^2) no longer commutes with K_i, and the blocks
of P^-1 are D^H = S^-1, E^H = -S^-1 B, F^H = -C S^-1, G^H = I + C S^-1 B.
"""
import numpy as np
import scipy.linalg as sla


class SolverError(Exception):
    pass


class NewtonError(SolverError):
    pass


class GMRESError(SolverError):
    pass


def gmres(Aop, rhs, M, rtol, restart, maxit):
    """Right-preconditioned restarted GMRES with modified Gram-Schmidt and
    Givens rotations; solves A x = rhs from x = 0.  Returns (x, iterations)."""
    n = rhs.shape[0]
    x = np.zeros(n)
    beta0 = np.linalg.norm(rhs)
    if beta0 == 0.0:
        return x, 0
    total = 0
    r = rhs.copy()
    while True:
        beta = np.linalg.norm(r)
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        converged = False
        jlast = -1
        for j in range(restart):
            z = M(V[j])
            Z.append(z)
            wv = Aop(z)
            for i in range(j + 1):
                H[i, j] = np.dot(V[i], wv)
                wv = wv - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(wv)
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            jlast = j
            if abs(g[j + 1]) <= rtol * beta0:
                converged = True
                break
            if total >= maxit:
                break
            hn = np.linalg.norm(wv)
            if hn == 0.0:
                converged = True
                break
            V.append(wv / hn)
        k = jlast + 1
        y = sla.solve_triangular(H[:k, :k], g[:k])
        for i in range(k):
            x = x + y[i] * Z[i]
        if converged:
            return x, total
        if total >= maxit:
            raise GMRESError("GMRES did not reach eps_G within %d iterations" % maxit)
        r = rhs - Aop(x)


class BJExt:
    """Extended block-Jacobi preconditioner BJ_ext, built at linearisation state w."""

    def __init__(self, dg, w, a1dt, bcoef):
        self.dg = dg
        self.a1dt = a1dt
        self.bcoef = bcoef
        K = dg.local_jacobian(w)
        ne = K.shape[1]
        I = np.eye(ne)
        self.K = K
        self.lu = []
        for i in range(K.shape[0]):
            S = I - a1dt * K[i] + bcoef * (K[i] @ K[i])
            self.lu.append(sla.lu_factor(S))

    def apply(self, X):
        dg = self.dg
        n = dg.ndof
        nE = dg.mesh.n_elem
        vw = X[:n].reshape(nE, -1)
        vs = X[n:].reshape(nE, -1)
        out_w = np.empty_like(vw)
        out_s = np.empty_like(vs)
        for i in range(nE):
            K = self.K[i]
            y = sla.lu_solve(self.lu[i], vw[i])            # D vw
            z = sla.lu_solve(self.lu[i], vs[i])            # S^-1 vs
            Dw = y
            Es = -self.bcoef * (K @ z)                     # E vs = -B S^-1 vs
            Fw = K @ y                                     # F vw = -C S^-1 vw
            Gs = z - self.a1dt * (K @ z)                   # G vs = A S^-1 vs
            out_w[i] = Dw + Es
            out_s[i] = Fw + Gs
        return np.concatenate([out_w.reshape(-1), out_s.reshape(-1)])


class BJExtH:
    """Extended block-Jacobi preconditioner with the Hessian block, BJ^H_ext, built at
    the state (w, sigma)."""

    def __init__(self, dg, w, sigma, a1dt, bcoef):
        self.dg = dg
        self.a1dt = a1dt
        self.bcoef = bcoef
        K = dg.local_jacobian(w)
        H = dg.local_hessian(w, sigma)
        ne = K.shape[1]
        I = np.eye(ne)
        self.K = K
        self.H = H
        self.lu = []
        for i in range(K.shape[0]):
            A = I - a1dt * K[i] + bcoef * H[i]
            B = bcoef * K[i]
            C = -K[i]
            self.lu.append(sla.lu_factor(A - B @ C))

    def apply(self, X):
        dg = self.dg
        n = dg.ndof
        nE = dg.mesh.n_elem
        vw = X[:n].reshape(nE, -1)
        vs = X[n:].reshape(nE, -1)
        out_w = np.empty_like(vw)
        out_s = np.empty_like(vs)
        for i in range(nE):
            B = self.bcoef * self.K[i]
            C = -self.K[i]
            Dw = sla.lu_solve(self.lu[i], vw[i])           # D^H vw = S^-1 vw
            Es = -sla.lu_solve(self.lu[i], B @ vs[i])      # E^H vs = -S^-1 B vs
            Fw = -(C @ Dw)                                 # F^H vw = -C S^-1 vw
            Gs = vs[i] + C @ (-Es)                         # G^H vs = vs + C S^-1 B vs
            out_w[i] = Dw + Es
            out_s[i] = Fw + Gs
        return np.concatenate([out_w.reshape(-1), out_s.reshape(-1)])


class StageSolver:
    """Newton on the extended residual of one DGSEM stage equation."""

    def __init__(self, dg, newton_rtol=1e-8, newton_atol_dw=1.95e-15, newton_maxit=30,
                 linear="gmres", gmres_rtol=1e-3, gmres_restart=30, gmres_maxit=7000,
                 precond="bjext", hessian=True, jvp="exact"):
        self.dg = dg
        self.newton_rtol = newton_rtol
        self.newton_atol_dw = newton_atol_dw
        self.newton_maxit = newton_maxit
        self.linear = linear
        self.gmres_rtol = gmres_rtol
        self.gmres_restart = gmres_restart
        self.gmres_maxit = gmres_maxit
        self.precond = precond
        self.hessian = hessian
        self.jvp_mode = jvp
        self.log = []

    def _jvp_fd(self, w, sigma, dX, a1dt, bcoef, r1w, r2ws):
        """Finite-difference JVP (Eq. MatrixFree_nonlinear) with
        eps_FD = sqrt(eps_machine) / (eps ||d||_2), eps the reference Mach number."""
        dg = self.dg
        n = dg.ndof
        dw, ds = dX[:n].reshape(w.shape), dX[n:].reshape(w.shape)
        emach = np.finfo(np.float64).eps
        epsref = getattr(dg.eq, "eps", 1.0)
        nw, ns = np.linalg.norm(dw), np.linalg.norm(ds)
        T1 = np.zeros_like(w)
        T3 = np.zeros_like(w)
        T2 = np.zeros_like(w)
        if nw > 0:
            ew = np.sqrt(emach) / (epsref * nw)
            T1 = (dg.r1(w + ew * dw) - r1w) / ew
            T3 = (dg.r2(w + ew * dw, sigma) - r2ws) / ew
        if ns > 0:
            es = np.sqrt(emach) / (epsref * ns)
            T2 = (dg.r2(w, sigma + es * ds) - r2ws) / es
        Jw = dw - a1dt * T1 + bcoef * (T3 + T2)
        Js = ds - T1
        return np.concatenate([Jw.reshape(-1), Js.reshape(-1)])

    def jacobian_op(self, w, sigma, a1dt, bcoef):
        dg = self.dg
        n = dg.ndof
        if self.jvp_mode == "fd":
            r1w = dg.r1(w)
            r2ws = dg.r2(w, sigma)
            return lambda dX: self._jvp_fd(w, sigma, dX, a1dt, bcoef, r1w, r2ws)

        def op(dX):
            Jw, Js = dg.jvp(w, sigma, dX[:n].reshape(w.shape), dX[n:].reshape(w.shape),
                            a1dt, bcoef, hessian=self.hessian)
            return np.concatenate([Jw.reshape(-1), Js.reshape(-1)])
        return op

    def dense_jacobian(self, w, sigma, a1dt, bcoef):
        op = self.jacobian_op(w, sigma, a1dt, bcoef)
        n2 = 2 * self.dg.ndof
        J = np.zeros((n2, n2))
        for c in range(n2):
            e = np.zeros(n2)
            e[c] = 1.0
            J[:, c] = op(e)
        return J

    def solve(self, b, a1dt, bcoef, guess):
        dg = self.dg
        n = dg.ndof
        shape = guess.shape
        w = guess.copy()
        sigma = dg.r1(w)

        def G(w, s):
            g1, g2 = dg.residual_G(w, s, b, a1dt, bcoef)
            return np.concatenate([g1.reshape(-1), g2.reshape(-1)])

        Gr = G(w, sigma)
        n0 = np.linalg.norm(Gr)
        stats = {"newton": 0, "gmres": []}
        if n0 <= 1e-14 * np.sqrt(2 * n):
            self.log.append(stats)
            return w
        nw0 = np.linalg.norm(w)
        nr_prev = n0
        stats["floor_stop"] = False
        pc = None
        if self.linear == "gmres" and self.precond == "bjext":
            pc = BJExt(dg, w, a1dt, bcoef)                 # once per Newton solve, at X^0
        elif self.linear == "gmres" and self.precond == "bjext_h":
            pc = BJExtH(dg, w, sigma, a1dt, bcoef)
        for it in range(1, self.newton_maxit + 1):
            if self.linear == "dense":
                J = self.dense_jacobian(w, sigma, a1dt, bcoef)
                dX = np.linalg.solve(J, -Gr)
            else:
                op = self.jacobian_op(w, sigma, a1dt, bcoef)
                M = pc.apply if pc is not None else (lambda v: v.copy())
                dX, its = gmres(op, -Gr, M, self.gmres_rtol, self.gmres_restart, self.gmres_maxit)
                stats["gmres"].append(its)
            w = w + dX[:n].reshape(shape)
            sigma = sigma + dX[n:].reshape(shape)
            Gr = G(w, sigma)
            stats["newton"] = it
            nr = np.linalg.norm(Gr)
            ndw = np.linalg.norm(dX[:n])
            if nr <= self.newton_rtol * n0 or ndw / np.sqrt(n) <= self.newton_atol_dw:
                self.log.append(stats)
                return w
            if it >= 2 and nr > 0.5 * nr_prev and ndw <= 1e-12 * nw0:
                stats["floor_stop"] = True
                self.log.append(stats)
                return w
            nr_prev = nr
        raise NewtonError("Newton did not converge in %d iterations" % self.newton_maxit)


def dg_hbpc_step(dg, w, dt, q, kmax, solver):
    """One HBPC(q, k_max) step of the DGSEM semi-discretisation."""
    from .hbpc import hbpc_step
    return hbpc_step(w, dt, q, kmax, dg.r1, lambda x: dg.r2(x), solver.solve)
