"""Pins for the HBPC(q, k_max) driver (Algorithm 1, appendix tableaux).

* each tableau row is an exact Hermite-Birkhoff quadrature of order q;
* on y' = z y the step is a rational function of z whose Taylor series
      matches e^z to order min(4 + k_max, q) (remark after Algorithm 1);
* the predictor substep is the (2,2)-Pade approximant, |R(iy)| = 1;
* for q = 4 the corrector leaves the predictor result unchanged;
* temporal EOC on the 1-D advection DGSEM semi-discretisation against the
      matrix exponential.
The power series are exact rationals, so these checks do not depend on
floating point.
"""
from fractions import Fraction as Fr
from math import factorial

import numpy as np
import pytest
import scipy.linalg as sla

from oracle.hbpc import hbpc_step
from oracle.tableaux import tableau

ORDER = 12      # power series truncation


class PS:
    """Truncated power series in z with exact rational coefficients."""

    def __init__(self, c):
        c = list(c)[:ORDER + 1]
        self.c = [Fr(x) for x in c] + [Fr(0)] * (ORDER + 1 - len(c))

    def __add__(self, o):
        return PS([a + b for a, b in zip(self.c, o.c)])

    def __sub__(self, o):
        return PS([a - b for a, b in zip(self.c, o.c)])

    def __mul__(self, o):
        if isinstance(o, PS):
            out = [Fr(0)] * (ORDER + 1)
            for i, a in enumerate(self.c):
                if a:
                    for j in range(ORDER + 1 - i):
                        out[i + j] += a * o.c[j]
            return PS(out)
        return PS([a * o for a in self.c])

    def div(self, o):
        q = [Fr(0)] * (ORDER + 1)
        r = list(self.c)
        for k in range(ORDER + 1):
            q[k] = r[k] / o.c[0]
            for j in range(k, ORDER + 1):
                r[j] -= q[k] * o.c[j - k]
        return PS(q)


Z = PS([0, 1])


def dahlquist_step(q, kmax):
    """Amplification factor R(z) of one HBPC step on y' = z y (dt = 1)."""
    one = PS([1])
    return hbpc_step(one, Fr(1), q, kmax,
                     lambda W: W * Z, lambda W: W * Z * Z,
                     lambda b, a1dt, bc, g: b.div(one - Z * a1dt + Z * Z * bc))


def order_of(R):
    for k in range(ORDER + 1):
        if R.c[k] != Fr(1, factorial(k)):
            return k - 1
    return ORDER


@pytest.mark.parametrize("q", [4, 6, 8])
def test_tableau_rows_are_exact_quadratures(q):
    """int_0^{c_l} t^p dt = sum_j B1 c_j^p + sum_j B2 p c_j^(p-1) for p <= q-1."""
    tab = tableau(q)
    for l in range(1, tab.s):
        for p in range(q):
            exact = tab.c[l] ** (p + 1) / (p + 1)
            quad = sum(tab.B1[l][j] * tab.c[j] ** p for j in range(tab.s))
            quad += sum(tab.B2[l][j] * (p * tab.c[j] ** (p - 1) if p > 0 else 0) for j in range(tab.s))
            assert quad == exact, (q, l, p)
    # and the last row is not exact one degree higher (order is exactly q)
    l = tab.s - 1
    p = q
    exact = tab.c[l] ** (p + 1) / (p + 1)
    quad = sum(tab.B1[l][j] * tab.c[j] ** p for j in range(tab.s))
    quad += sum(tab.B2[l][j] * p * tab.c[j] ** (p - 1) for j in range(tab.s))
    assert quad != exact


@pytest.mark.parametrize("q,orders", [(4, [4, 4, 4, 4]),
                                      (6, [4, 5, 6, 6, 6]),
                                      (8, [4, 5, 6, 7, 8, 8, 8])])
def test_dahlquist_order(q, orders):
    """order min(4 + k_max, q)."""
    got = [order_of(dahlquist_step(q, k)) for k in range(len(orders))]
    assert got == orders


def test_predictor_is_pade22():
    """one predictor substep of length c dt is (1 + x/2 + x^2/12)/(1 - x/2 + x^2/12), x = c z."""
    R = dahlquist_step(4, 0)
    pade = (PS([1]) + Z * Fr(1, 2) + Z * Z * Fr(1, 12)).div(PS([1]) - Z * Fr(1, 2) + Z * Z * Fr(1, 12))
    assert R.c == pade.c
    # |R(iy)| = 1 on the imaginary axis (evaluated in complex floating point)
    for y in [0.1, 1.0, 7.0, 50.0]:
        z = 1j * y
        val = (1 + z / 2 + z * z / 12) / (1 - z / 2 + z * z / 12)
        assert abs(abs(val) - 1.0) < 1e-14


def test_q4_corrector_is_noop():
    """for q = 4 the corrector sweeps reproduce the predictor exactly."""
    R0 = dahlquist_step(4, 0)
    for k in (1, 2, 3):
        assert dahlquist_step(4, k).c == R0.c


def test_corrector_without_quadrature_term_breaks_order():
    """The corrector right-hand side needs the quadrature I_l: without it the
    q = 6 scheme does not gain order (pins the reading of Eq. nonlinear_corrector)."""
    one = PS([1])
    tab = tableau(6)

    def step_without_I():
        W = [one, None, None]
        r1 = lambda v: v * Z
        r2 = lambda v: v * Z * Z
        for l in (1, 2):
            dc = tab.c[l] - tab.c[l - 1]
            a1, bc = dc / 2, dc * dc / 12
            b = W[l - 1] + r1(W[l - 1]) * a1 + r2(W[l - 1]) * bc
            W[l] = b.div(one - Z * a1 + Z * Z * bc)
        Wn = list(W)
        for l in (1, 2):
            b = W[0] - r1(W[l]) + r2(W[l]) * Fr(1, 2)
            Wn[l] = b.div(one - Z + Z * Z * Fr(1, 2))
        return Wn[2]
    assert order_of(step_without_I()) < 5


def _advection_matrix():
    from oracle.dgsem import DGSEM, Mesh
    from oracle.equations import Advection
    dg = DGSEM(Mesh(1, [16], [1.0]), 3, Advection(1, [1.0]), nodes="lobatto", flux="upwind")
    n = dg.ndof
    Lm = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        Lm[:, c] = dg.r1(e.reshape(16, 1, 4)).reshape(-1)
    x = dg.node_coords()[0]
    return Lm, np.sin(2 * np.pi * x).reshape(-1)


@pytest.mark.parametrize("q,k,expected", [(6, 0, 4), (6, 1, 5), (6, 2, 6), (6, 3, 6), (8, 4, 8)])
def test_temporal_eoc_advection(q, k, expected):
    """error against expm(T L) u0 decays with order min(4 + k, q) (Fig. 7's claim)."""
    Lm, u0 = _advection_matrix()
    I = np.eye(len(u0))
    T = 1.0
    exact = sla.expm(T * Lm) @ u0

    def solve(b, a1dt, bc, g):
        return np.linalg.solve(I - a1dt * Lm + bc * (Lm @ Lm), b)
    errs = []
    for dt in (0.05, 0.025, 0.0125):
        u = u0.copy()
        for _ in range(int(round(T / dt))):
            u = hbpc_step(u, dt, q, k, lambda v: Lm @ v, lambda v: Lm @ (Lm @ v), solve)
        errs.append(np.linalg.norm(u - exact) / np.linalg.norm(exact))
    rate = np.log2(errs[1] / errs[2])
    assert abs(rate - expected) < 0.35, (errs, rate)
