"""Pins for the 1-D reference operators (Sec. 3.1.1): closed forms and
polynomial exactness, independent of the oracle's own formulas."""
import numpy as np
import pytest
from numpy.polynomial import legendre as L

from oracle.basis import Basis1D, gauss_lobatto


@pytest.mark.parametrize("kind", ["gauss", "lobatto"])
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7])
def test_quadrature_exactness(kind, N):
    """Gauss is exact to degree 2N+1, Lobatto to 2N-1 (textbook)."""
    b = Basis1D(N, kind)
    top = 2 * N + 1 if kind == "gauss" else 2 * N - 1
    for p in range(top + 1):
        exact = (1.0 - (-1.0) ** (p + 1)) / (p + 1)
        assert abs(np.dot(b.w, b.xi ** p) - exact) < 1e-13


def test_lobatto_known_nodes():
    """N = 2 Lobatto: nodes -1, 0, 1 with weights 1/3, 4/3, 1/3; N = 3 interior nodes +-1/sqrt(5)."""
    x, w = gauss_lobatto(2)
    assert np.allclose(x, [-1, 0, 1]) and np.allclose(w, [1 / 3, 4 / 3, 1 / 3])
    x, w = gauss_lobatto(3)
    assert np.allclose(x, [-1, -1 / np.sqrt(5), 1 / np.sqrt(5), 1])
    assert np.allclose(w, [1 / 6, 5 / 6, 5 / 6, 1 / 6])


@pytest.mark.parametrize("kind", ["gauss", "lobatto"])
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7])
def test_free_stream_identity(kind, N):
    """sum_lam Dhat[i,lam] + lhat_i(1) - lhat_i(-1) = 0: a constant flux gives R = 0."""
    b = Basis1D(N, kind)
    assert np.abs(b.Dhat.sum(axis=1) + b.lhat_plus - b.lhat_minus).max() < 1e-12


@pytest.mark.parametrize("kind", ["gauss", "lobatto"])
@pytest.mark.parametrize("N", [2, 3, 5, 7])
def test_weak_derivative_exact_for_polynomials(kind, N):
    """For F in P_N: Dhat F + F(1) lhat(1) - F(-1) lhat(-1) = F'(xi) exactly.

    F is a random Legendre series; F' from numpy's Legendre derivative."""
    b = Basis1D(N, kind)
    rng = np.random.default_rng(N + 10 * (kind == "gauss"))
    c = rng.standard_normal(N + 1)
    F = L.legval(b.xi, c)
    dF = L.legval(b.xi, L.legder(c))
    got = b.Dhat @ F + L.legval(1.0, c) * b.lhat_plus - L.legval(-1.0, c) * b.lhat_minus
    assert np.abs(got - dF).max() < 1e-11 * max(1.0, np.abs(dF).max())


def test_printed_weight_ratio_is_not_consistent():
    """The D-hat printed with omega_i/omega_j (weights inverted) breaks the
    free-stream identity; this documents why the derived form is used."""
    b = Basis1D(3, "gauss")
    printed = -(b.w[:, None] / b.w[None, :]) * b.Dstd.T
    err = np.abs(printed.sum(axis=1) + b.lhat_plus - b.lhat_minus).max()
    assert err > 1e-2


@pytest.mark.parametrize("N", [2, 3, 5])
def test_lagrange_boundary_values(N):
    """l_i(+-1) reproduces polynomials: sum_i l_i(1) p(xi_i) = p(1)."""
    b = Basis1D(N, "gauss")
    for p in range(N + 1):
        assert abs(np.dot(b.l_plus, b.xi ** p) - 1.0) < 1e-12
        assert abs(np.dot(b.l_minus, b.xi ** p) - (-1.0) ** p) < 1e-12
