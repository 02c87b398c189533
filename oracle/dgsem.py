"""DGSEM spatial operators on uniform periodic Cartesian meshes (Sec. 3.1).

R1_h (Eq. DGSEM_wt, written for d = 1, 2, 3):

    R1_node = - sum_m (2/h_m) [ sum_lam Dhat[i_m, lam] F_m(w at i_m -> lam)
                                + f*_{+m} lhat_{i_m}(+1) - f*_{-m} lhat_{i_m}(-1) ]

  * Cartesian metric terms (the paper defers them to Hindenlang et al.):
    J = prod h_m / 2, contravariant flux (2J/h_m) F_m, surface element 2J/h_m;
    net effect a factor 2/h_m per direction.
  * traces w(+-1) = sum_i l_i(+-1) w_i along each line (Eq. Interpolation).
  * f*_{+m} is the numerical flux (equations.numerical_flux) at the element's
    +e_m face with the element itself on the L side; f*_{-m} is the flux at
    its -e_m face with the element on the R side.

R2_h (Eq. DGSEM_wtt) is the directional derivative of R1_h at w along sigma;
for a globally constant lambda this is exactly the paper's formula (flux
Jacobian times sigma in the volume, f-tilde* on faces).  For the Rusanov flux
it also carries the derivative of lambda (tie rules in jets).  The Hessian
term dR2/dw dw of the extended Jacobian (Eq. nonlinear_eqsys) is the mixed
second derivative R1''(w)[sigma, dw].

BR1 for viscous Burgers: q_m = (2/h_m)[Dhat u + u*_+ lhat(+1) - u*_- lhat(-1)]
with u* = (uL + uR)/2; viscous flux -nu q_m in the volume, -nu (qL + qR)/2 on
faces.

BR2 for Navier-Stokes (Sec. 5.1, Eqs. NS_System, Lifting, Riemann_visc), with
g = w_grad(w) = (v, T) at the nodes, g^+- = w_grad(w^+-) at a face from the
traces of w, and g* = (g^L + g^R)/2:
  * volume gradients (global lifting, strong form):
        d_{k,j} = (2/h_j)[D g_k + lhat(+1)(g*_{k,+j} - g^+_k) - lhat(-1)(g*_{k,-j} - g^-_k)]
    with D_{i lam} = l_lam'(xi_i);
  * face gradients (BR2 local lifting of the face's own jump): on the +e_m
    face d^L_{k,j} = [(2/h_j) D_j g_k](+1 along m) + eta delta_jm (2/h_m) c_+ (g*_k - g^+_k),
    on the -e_m face the same with l(-1), c_- and a minus sign;
    c_+- = sum_i l_i(+-1)^2 / omega_i (the local lifting evaluated on its face);
  * volume flux F - F^v(w, d); face flux f*(wL, wR) - (F^v(wL, d^L) + F^v(wR, d^R))/2.
eta (eta_br2) is the BR2 stabilisation parameter, 2 by default.  R2 is again
the exact directional derivative, so that the linearised lifting (the eta
auxiliary variable of Eq. Lifting_eta) is carried by the jets.

Layout of flat arrays: w[e][v][node], node = i + (N+1)(j + (N+1)k), elements
lexicographic with x fastest.  Internally each variable is an array of shape
(n_{d-1}, .., n_0, N+1, .., N+1) whose last axis is the x node index.
"""
import numpy as np
from . import jets
from .basis import Basis1D
from .equations import numerical_flux, Burgers, NavierStokes


class Mesh:
    """Uniform periodic Cartesian mesh: nelem[m] elements of size h_m in direction m."""

    def __init__(self, dim, nelem, length, origin=None):
        self.dim = dim
        self.nelem = tuple(int(n) for n in nelem[:dim])
        self.length = tuple(float(x) for x in length[:dim])
        self.origin = tuple(float(x) for x in (origin or [0.0] * 3)[:dim])
        self.h = tuple(self.length[m] / self.nelem[m] for m in range(dim))
        self.n_elem = int(np.prod(self.nelem))


def _lin(fn, x):
    """Apply a linear map to a value or to every component of a jet."""
    if isinstance(x, jets.HD):
        return jets.HD(fn(x.a), fn(x.b), fn(x.c), fn(x.d))
    return fn(x)


def _const(x):
    """Drop all derivative parts (used for neighbour data in the local Jacobian)."""
    return x.a if isinstance(x, jets.HD) else x


def _const_but_b(x):
    """Keep the value and the b part, drop the others (neighbour data in the local
    Hessian block: sigma of the neighbours stays, their dependence on w does not)."""
    if isinstance(x, jets.HD):
        z = np.zeros_like(x.a)
        return jets.HD(x.a, x.b, z, z)
    return x


class DGSEM:
    def __init__(self, mesh, N, eq, nodes="gauss", flux="rusanov", lam=0.0, eta_br2=2.0):
        self.mesh = mesh
        self.d = mesh.dim
        self.N = N
        self.np = N + 1
        self.eq = eq
        self.basis = Basis1D(N, nodes)
        self.flux_kind = flux
        self.lam = lam
        self.nvar = eq.nvar
        self.nnode = self.np ** self.d
        self.ndof = mesh.n_elem * self.nvar * self.nnode
        self.viscous = isinstance(eq, Burgers) and eq.nu != 0.0
        self.is_burgers = isinstance(eq, Burgers)
        self.ns = isinstance(eq, NavierStokes)
        self.eta_br2 = float(eta_br2)

    # ---------------------------------------------------------------- layout
    def _egrid(self):
        return tuple(reversed(self.mesh.nelem))

    def to_vars(self, flat):
        """flat (nE, nvar, nnode) or (ndof,) -> list of nvar arrays (egrid + ngrid)."""
        d = self.d
        a = np.asarray(flat).reshape(self._egrid() + (self.nvar,) + (self.np,) * d)
        a = np.moveaxis(a, d, 0)
        return [a[v] for v in range(self.nvar)]

    def to_flat(self, vars_):
        d = self.d
        a = np.stack(vars_, axis=d)
        return a.reshape(self.mesh.n_elem, self.nvar, self.nnode)

    def _nax(self, m):          # node axis of direction m
        return self.d + (self.d - 1 - m)

    def _eax(self, m):          # element axis of direction m
        return self.d - 1 - m

    # ------------------------------------------------------------ primitives
    def _contract(self, M, x, m):
        """result[.., i, ..] = sum_lam M[i, lam] x[.., lam, ..] along direction m's node axis."""
        ax = self._nax(m)

        def f(a):
            r = np.tensordot(a, M, axes=([ax], [1]))    # new axis last
            return np.moveaxis(r, -1, ax)
        return _lin(f, x)

    def _trace(self, x, lvec, m):
        ax = self._nax(m)
        return _lin(lambda a: np.tensordot(a, lvec, axes=([ax], [0])), x)

    def _spread(self, f, lvec, m):
        """Broadcast face data f back along direction m's node axis, times lvec."""
        ax = self._nax(m)
        shape = [1] * (2 * self.d)
        shape[ax] = self.np
        lv = lvec.reshape(shape)
        return _lin(lambda a: np.expand_dims(a, ax) * lv, f)

    def _roll(self, x, shift, m):
        ax = self._eax(m)
        return _lin(lambda a: np.roll(a, shift, axis=ax), x)

    # ------------------------------------------------------------- operators
    def _neighbour_traces(self, u, m, local):
        """Own traces at -/+ faces and neighbour traces across them."""
        b = self.basis
        up = [self._trace(u[v], b.l_plus, m) for v in range(len(u))]
        um = [self._trace(u[v], b.l_minus, m) for v in range(len(u))]
        nb_right = [self._roll(um[v], -1, m) for v in range(len(u))]   # minus-trace of element e+1
        nb_left = [self._roll(up[v], +1, m) for v in range(len(u))]    # plus-trace of element e-1
        if local:
            keep = _const_but_b if local == "b" else _const
            nb_right = [keep(x) for x in nb_right]
            nb_left = [keep(x) for x in nb_left]
        return up, um, nb_left, nb_right

    def lift(self, u, local=False):
        """BR1 lifted gradient q_m of the scalar u (list of d arrays)."""
        b = self.basis
        q = []
        for m in range(self.d):
            up, um, nl, nr = self._neighbour_traces([u], m, local)
            ustar_p = 0.5 * (up[0] + nr[0])
            ustar_m = 0.5 * (nl[0] + um[0])
            vol = self._contract(b.Dhat, u, m)
            s = vol + self._spread(ustar_p, b.lhat_plus, m) - self._spread(ustar_m, b.lhat_minus, m)
            q.append(s * (2.0 / self.mesh.h[m]))
        return q

    def _r1_ns(self, u, local=False):
        """R1_h of the Navier-Stokes equations with BR2 lifting (module docstring)."""
        b = self.basis
        eq = self.eq
        d = self.d
        nv = self.nvar
        ng = eq.ngrad
        h = self.mesh.h
        keep = (_const_but_b if local == "b" else _const) if local else (lambda x: x)
        g = eq.grad_vars(u)
        # strong (broken) gradient at the nodes: dvol[k][j] = (2/h_j) D_j g_k
        dvol = [[self._contract(b.Dstd, g[k], j) * (2.0 / h[j]) for j in range(d)] for k in range(ng)]
        faces = []
        for m in range(d):
            up, um, nl, nr = self._neighbour_traces(u, m, local)
            gp, gm = eq.grad_vars(up), eq.grad_vars(um)
            gnl, gnr = eq.grad_vars(nl), eq.grad_vars(nr)
            jp = [0.5 * (gp[k] + gnr[k]) - gp[k] for k in range(ng)]   # g* - g^+ on the +e_m face
            jm = [0.5 * (gnl[k] + gm[k]) - gm[k] for k in range(ng)]   # g* - g^- on the -e_m face
            faces.append((up, um, nl, nr, jp, jm))
        # global lifting: the volume gradients
        dglob = [[None] * d for _ in range(ng)]
        for j in range(d):
            jp, jm = faces[j][4], faces[j][5]
            for k in range(ng):
                s = self._spread(jp[k], b.lhat_plus, j) - self._spread(jm[k], b.lhat_minus, j)
                dglob[k][j] = dvol[k][j] + s * (2.0 / h[j])
        c_p = float(np.sum(b.l_plus ** 2 / b.w))
        c_m = float(np.sum(b.l_minus ** 2 / b.w))
        R = [None] * nv
        for m in range(d):
            up, um, nl, nr, jp, jm = faces[m]
            # own BR2 face gradients on the +-e_m faces
            dfp = [[self._trace(dvol[k][j], b.l_plus, m) for j in range(d)] for k in range(ng)]
            dfm = [[self._trace(dvol[k][j], b.l_minus, m) for j in range(d)] for k in range(ng)]
            for k in range(ng):
                dfp[k][m] = dfp[k][m] + jp[k] * (self.eta_br2 * 2.0 / h[m] * c_p)
                dfm[k][m] = dfm[k][m] - jm[k] * (self.eta_br2 * 2.0 / h[m] * c_m)
            # the neighbours' face gradients on the shared faces (computed by the neighbours)
            dfnr = [[keep(self._roll(dfm[k][j], -1, m)) for j in range(d)] for k in range(ng)]
            dfnl = [[keep(self._roll(dfp[k][j], +1, m)) for j in range(d)] for k in range(ng)]
            F = eq.flux(u, m)
            Fv = eq.viscous_flux(u, dglob, m)
            F = [F[v] - Fv[v] for v in range(nv)]
            fp = numerical_flux(eq, self.flux_kind, self.lam, up, nr, m)    # element on L side
            fm = numerical_flux(eq, self.flux_kind, self.lam, nl, um, m)    # element on R side
            vp_own, vp_nb = eq.viscous_flux(up, dfp, m), eq.viscous_flux(nr, dfnr, m)
            vm_nb, vm_own = eq.viscous_flux(nl, dfnl, m), eq.viscous_flux(um, dfm, m)
            fp = [fp[v] - 0.5 * (vp_own[v] + vp_nb[v]) for v in range(nv)]
            fm = [fm[v] - 0.5 * (vm_nb[v] + vm_own[v]) for v in range(nv)]
            for v in range(nv):
                vol = self._contract(b.Dhat, F[v], m)
                s = vol + self._spread(fp[v], b.lhat_plus, m) - self._spread(fm[v], b.lhat_minus, m)
                s = s * (2.0 / h[m])
                R[v] = s if R[v] is None else R[v] + s
        return [-x for x in R]

    def _r1_vars(self, u, local=False):
        """R1_h on a list of per-variable arrays (values, complex or jets)."""
        if self.ns:
            return self._r1_ns(u, local)
        b = self.basis
        eq = self.eq
        nv = self.nvar
        q = self.lift(u[0], local) if self.viscous else None
        R = [None] * nv
        for m in range(self.d):
            F = eq.flux(u, m)
            if self.viscous:
                F = [F[0] - q[m] * eq.nu]
            up, um, nl, nr = self._neighbour_traces(u, m, local)
            fp = numerical_flux(eq, self.flux_kind, self.lam, up, nr, m)    # element on L side
            fm = numerical_flux(eq, self.flux_kind, self.lam, nl, um, m)    # element on R side
            if self.viscous:
                qp, qm, qnl, qnr = self._neighbour_traces([q[m]], m, local)
                fp = [fp[0] - 0.5 * eq.nu * (qp[0] + qnr[0])]
                fm = [fm[0] - 0.5 * eq.nu * (qnl[0] + qm[0])]
            for v in range(nv):
                vol = self._contract(b.Dhat, F[v], m)
                s = vol + self._spread(fp[v], b.lhat_plus, m) - self._spread(fm[v], b.lhat_minus, m)
                s = s * (2.0 / self.mesh.h[m])
                R[v] = s if R[v] is None else R[v] + s
        return [-x for x in R]

    # public flat-array API -------------------------------------------------
    def r1(self, w):
        """R1_h(w) (Eq. DGSEM_wt)."""
        return self.to_flat(self._r1_vars(self.to_vars(w)))

    def r1_complex(self, w):
        """R1_h on complex input (for complex-step derivative checks)."""
        return self.to_flat(self._r1_vars(self.to_vars(np.asarray(w, dtype=np.complex128))))

    def _jet(self, w, b=None, c=None):
        wv = self.to_vars(w)
        bv = self.to_vars(b) if b is not None else [np.zeros_like(x) for x in wv]
        cv = self.to_vars(c) if c is not None else [np.zeros_like(x) for x in wv]
        return [jets.HD(wv[v], bv[v], cv[v], np.zeros_like(wv[v])) for v in range(self.nvar)]

    def r2(self, w, sigma=None, local=False):
        """R2_h(w, sigma) = R1_h'(w) sigma (Eq. DGSEM_wtt); sigma defaults to R1_h(w)."""
        if sigma is None:
            sigma = self.r1(w)
        R = self._r1_vars(self._jet(w, sigma), local)
        return self.to_flat([jets.part(x, "b") for x in R])

    def r1_and_r2(self, w, sigma):
        R = self._r1_vars(self._jet(w, sigma))
        return (self.to_flat([jets.part(x, "a") for x in R]),
                self.to_flat([jets.part(x, "b") for x in R]))

    def hessian_term(self, w, sigma, dw):
        """T3 = R1''(w)[sigma, dw] = (dR2_h/dw)(w, sigma) dw."""
        R = self._r1_vars(self._jet(w, sigma, dw))
        return self.to_flat([jets.part(x, "d") for x in R])

    def residual_G(self, w, sigma, b, a1dt, bcoef):
        """Extended residual G(X) (Sec. 3.2.1) with X = (w, sigma):
        G1 = w - a1dt R1(w) + bcoef R2(w, sigma) - b,  G2 = sigma - R1(w);
        a1dt = alpha1 dt, bcoef = alpha2 dt^2 / 2 (Eq. Newton_Residual)."""
        R1, R2 = self.r1_and_r2(w, sigma)
        return w - a1dt * R1 + bcoef * R2 - b, sigma - R1

    def jvp(self, w, sigma, dw, dsig, a1dt, bcoef, hessian=True):
        """Extended Jacobian times (dw, dsigma) (Eq. nonlinear_eqsys):
        ( dw - a1dt T1 + bcoef (T2 + T3),  dsigma - T1 ),
        T1 = R1'(w) dw, T2 = R1'(w) dsigma (= dR2/dsigma dsigma), T3 = dR2/dw dw."""
        T1 = self.r2(w, dw)
        T2 = self.r2(w, dsig)
        T3 = self.hessian_term(w, sigma, dw) if hessian else np.zeros_like(T1)
        return dw - a1dt * T1 + bcoef * (T2 + T3), dsig - T1

    # ------------------------------------------------- element-local Jacobian
    def local_jacobian(self, w):
        """K_i = dR1_i/dw_i for every element (neighbour data held constant).

        Every quantity read from a neighbouring element (its traces, and for
        BR1 its lifted gradient) is a constant; the own-side dependence of the
        face fluxes and of the own lifting is kept.  Returns (nE, ne, ne) with
        ne = nvar (N+1)^d and row/column index v*(N+1)^d + node."""
        nE = self.mesh.n_elem
        ne = self.nvar * self.nnode
        K = np.zeros((nE, ne, ne))
        for col in range(ne):
            e = np.zeros((nE, ne))
            e[:, col] = 1.0
            R = self._r1_vars(self._jet(w, e.reshape(nE, self.nvar, self.nnode)), local=True)
            K[:, :, col] = self.to_flat([jets.part(x, "b") for x in R]).reshape(nE, ne)
        return K

    def local_hessian(self, w, sigma):
        """H_i = dR2_i/dw_i at (w, sigma) for every element: the element-local block of
        R1''(w)[sigma, .], which BJ^H_ext adds to S_i (Sec. 3.2.3).

        sigma is the global field, so the neighbour traces keep their value and sigma
        parts; only the dependence on the neighbours' w is held constant.  Same shape
        and index convention as local_jacobian."""
        nE = self.mesh.n_elem
        ne = self.nvar * self.nnode
        H = np.zeros((nE, ne, ne))
        for col in range(ne):
            e = np.zeros((nE, ne))
            e[:, col] = 1.0
            R = self._r1_vars(self._jet(w, sigma, e.reshape(nE, self.nvar, self.nnode)), local="b")
            H[:, :, col] = self.to_flat([jets.part(x, "d") for x in R]).reshape(nE, ne)
        return H

    # ------------------------------------------------------------- utilities
    def node_coords(self):
        """Physical node coordinates, list of d flat arrays shaped (nE, nnode)."""
        d = self.d
        xi = self.basis.xi
        out = []
        for m in range(d):
            n = self.mesh.nelem[m]
            h = self.mesh.h[m]
            xc = self.mesh.origin[m] + h * (np.arange(n) + 0.5)
            # element axis m, node axis m
            eshape = [1] * d
            eshape[self._eax(m)] = n
            nshape = [1] * d
            nshape[d - 1 - m] = self.np
            x = xc.reshape(eshape + [1] * d) + 0.5 * h * xi.reshape([1] * d + nshape)
            x = np.broadcast_to(x, self._egrid() + (self.np,) * d)
            out.append(np.ascontiguousarray(x).reshape(self.mesh.n_elem, self.nnode))
        return out

    def quad_weights(self):
        """J * prod omega at each node, shape (nE, nnode): the DG mass diagonal."""
        d = self.d
        w1 = self.basis.w
        W = np.ones(())
        for m in range(d):
            W = np.multiply.outer(w1, W) if W.ndim else w1.copy()
        J = np.prod([h / 2.0 for h in self.mesh.h])
        return np.broadcast_to(J * W.reshape(-1), (self.mesh.n_elem, self.nnode))

    def integral(self, w):
        """sum_e J sum_nodes omega w, per variable (discrete mass)."""
        W = self.quad_weights()
        return np.einsum("en,evn->v", W, np.asarray(w).reshape(self.mesh.n_elem, self.nvar, self.nnode))
