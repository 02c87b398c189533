"""1-D reference operators of the DGSEM (Sec. 3.1.1, Eqs. Interpolation, DGSEM_wt).

Nodes xi_i and weights omega_i, i = 0..N, on [-1, 1]:
  * Gauss-Legendre (the paper's choice for interpolation and quadrature);
  * Gauss-Lobatto (used by the 1-D advection workload).

Lagrange basis l_i of degree N through the nodes, its derivative at the
nodes, the boundary values l_i(+-1) and l-hat_i(+-1) = l_i(+-1) / omega_i.

D-hat.  The paper prints D-hat_{ij} = -(omega_i/omega_j) l_i'(xi_j).  Deriving
the collocated weak form (Eq. weakform) for one element,

    (h/2) omega_i d/dt w_i - sum_lam omega_lam F_lam l_i'(xi_lam)
        + f*_+ l_i(1) - f*_- l_i(-1) = 0,

gives  d/dt w_i = -(2/h) [ sum_lam Dhat[i, lam] F_lam + f*_+ lhat_i(1) - f*_- lhat_i(-1) ]
with   Dhat[i, lam] = -(omega_lam / omega_i) l_i'(xi_lam).
The printed weight ratio is the inverse of this; the derived form is the one
that is consistent (free-stream and polynomial exactness hold, tests pin it).
"""
import numpy as np
from numpy.polynomial import legendre as _leg


def gauss_legendre(N):
    """N+1 Gauss-Legendre nodes and weights (library routine)."""
    x, w = _leg.leggauss(N + 1)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def gauss_lobatto(N):
    """N+1 Gauss-Lobatto nodes: +-1 and the roots of P_N'; weights 2/(N(N+1) P_N(x)^2)."""
    if N < 1:
        raise ValueError("Gauss-Lobatto needs N >= 1")
    cN = np.zeros(N + 1)
    cN[N] = 1.0                                  # Legendre series of P_N
    inner = _leg.legroots(_leg.legder(cN)) if N >= 2 else np.zeros(0)
    x = np.concatenate([[-1.0], np.sort(np.real(inner)), [1.0]])
    PN = _leg.legval(x, cN)
    w = 2.0 / (N * (N + 1) * PN ** 2)
    return x, w


def nodes(N, kind):
    if kind == "gauss":
        return gauss_legendre(N)
    if kind == "lobatto":
        return gauss_lobatto(N)
    raise ValueError(kind)


def lagrange_eval(xi, x):
    """Matrix L[k, i] = l_i(x_k) by the product formula."""
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(xi)
    L = np.ones((len(x), n))
    for i in range(n):
        for j in range(n):
            if j != i:
                L[:, i] *= (x - xi[j]) / (xi[i] - xi[j])
    return L


def lagrange_derivative_at_nodes(xi):
    """Matrix Dstd[k, i] = l_i'(xi_k) (derivative of basis i at node k).

    l_i'(x) = sum_{m != i} 1/(xi_i - xi_m) prod_{j != i, m} (x - xi_j)/(xi_i - xi_j).
    """
    n = len(xi)
    D = np.zeros((n, n))
    for k in range(n):
        for i in range(n):
            s = 0.0
            for m in range(n):
                if m == i:
                    continue
                p = 1.0 / (xi[i] - xi[m])
                for j in range(n):
                    if j != i and j != m:
                        p *= (xi[k] - xi[j]) / (xi[i] - xi[j])
                s += p
            D[k, i] = s
    return D


class Basis1D:
    """All 1-D operators for degree N on the chosen node set."""

    def __init__(self, N, kind="gauss"):
        self.N = N
        self.np = N + 1
        self.kind = kind
        self.xi, self.w = nodes(N, kind)
        Dstd = lagrange_derivative_at_nodes(self.xi)          # Dstd[lam, i] = l_i'(xi_lam)
        # Dhat[i, lam] = -(w_lam / w_i) l_i'(xi_lam)   (weak form, see module doc)
        self.Dhat = -(self.w[None, :] / self.w[:, None]) * Dstd.T
        self.Dstd = Dstd
        self.l_minus = lagrange_eval(self.xi, -1.0)[0]         # l_i(-1)
        self.l_plus = lagrange_eval(self.xi, 1.0)[0]           # l_i(+1)
        self.lhat_minus = self.l_minus / self.w
        self.lhat_plus = self.l_plus / self.w
