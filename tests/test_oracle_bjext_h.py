"""Pins for the BJ^H_ext preconditioner of Sec. 3.2.3: the element-local Hessian
block against complex-step derivatives of R2, the four blocks of P against the
element-diagonal blocks of the dense extended Jacobian, the inverse blocks
D^H, E^H, F^H, G^H against P itself, and the reduction to BJ_ext for a linear
flux (the Hessian contribution vanishes there)."""
import numpy as np
import pytest

from oracle.solvers import BJExt, BJExtH, StageSolver
from tests.test_oracle_dgsem import make, rel, smooth_state


def _sigma(dg, w, seed):
    """sigma near R1(w) but not equal to it (a Newton iterate)."""
    rng = np.random.default_rng(seed)
    r1 = dg.r1(w)
    return r1 + 0.05 * np.abs(r1).max() * rng.standard_normal(w.shape)


@pytest.mark.parametrize("kind", ["adv2", "euler2", "burgers", "euler3"])
def test_local_hessian_is_diagonal_block_of_dR2_dw(kind):
    """H_i equals d R2_i / d w_i at fixed sigma, column by column with the complex
    step on a mesh with 3 elements per direction; zero for the linear flux."""
    dg = make(kind, n=3, N=2 if kind != "euler3" else 1)
    w = smooth_state(dg, seed=3)
    sig = _sigma(dg, w, 4)
    H = dg.local_hessian(w, sig)
    nE, ne = dg.mesh.n_elem, dg.nvar * dg.nnode
    if kind == "adv2":
        assert np.abs(H).max() == 0.0
        return
    assert np.abs(H).max() > 1e-3
    h = 1e-30
    cols = range(0, ne, max(1, ne // 6))
    for col in cols:
        for e in (0, nE // 2, nE - 1):
            pert = np.zeros((nE, ne), dtype=complex)
            pert[e, col] = 1j * h
            _, R2 = dg.r1_and_r2(w.astype(complex) + pert.reshape(w.shape), sig.astype(complex))
            col_cs = np.imag(R2.reshape(nE, ne)[e]) / h
            assert np.abs(col_cs - H[e, :, col]).max() < 1e-10 * (1 + np.abs(H).max())


def _blocks(pc, i, a1dt, bc):
    K = pc.K[i]
    ne = K.shape[0]
    I = np.eye(ne)
    H = pc.H[i] if hasattr(pc, "H") else np.zeros_like(K)
    return np.block([[I - a1dt * K + bc * H, bc * K], [-K, I]])


def test_bjext_h_blocks_are_the_diagonal_blocks_of_the_jacobian():
    """The element blocks A^H_i, B_i, C_i, I of P are the element-diagonal blocks of
    the dense extended Jacobian (columns from the exact JVP with the Hessian term)."""
    dg = make("euler2", n=3, N=2)
    w = smooth_state(dg, seed=5)
    sig = _sigma(dg, w, 6)
    a1dt, bc = 0.04, 0.02 ** 2 / 2
    J = StageSolver(dg).dense_jacobian(w, sig, a1dt, bc)
    pc = BJExtH(dg, w, sig, a1dt, bc)
    n = dg.ndof
    nE, ne = dg.mesh.n_elem, dg.nvar * dg.nnode
    for i in range(nE):
        rows = np.r_[i * ne:(i + 1) * ne, n + i * ne:n + (i + 1) * ne]
        Jii = J[np.ix_(rows, rows)]
        assert np.abs(Jii - _blocks(pc, i, a1dt, bc)).max() < 1e-11 * np.abs(Jii).max()


@pytest.mark.parametrize("kind", ["euler2", "burgers"])
def test_bjext_h_inverts_its_block_matrix(kind):
    """P^-1 (P v) = v element by element, P assembled from A^H, B, C, I."""
    dg = make(kind, n=3, N=2)
    w = smooth_state(dg, seed=7)
    sig = _sigma(dg, w, 8)
    a1dt, bc = 0.3, 0.3 ** 2 / 2
    pc = BJExtH(dg, w, sig, a1dt, bc)
    n = dg.ndof
    nE, ne = dg.mesh.n_elem, dg.nvar * dg.nnode
    v = np.random.default_rng(9).standard_normal(2 * n)
    vw, vs = v[:n].reshape(nE, ne), v[n:].reshape(nE, ne)
    Pw = np.empty_like(vw)
    Ps = np.empty_like(vs)
    for i in range(nE):
        y = _blocks(pc, i, a1dt, bc) @ np.concatenate([vw[i], vs[i]])
        Pw[i], Ps[i] = y[:ne], y[ne:]
    back = pc.apply(np.concatenate([Pw.reshape(-1), Ps.reshape(-1)]))
    assert rel(back, v) < 1e-11


def test_bjext_h_reduces_to_bjext_for_linear_flux():
    dg = make("adv2", n=3, N=3)
    w = smooth_state(dg, seed=1)
    sig = _sigma(dg, w, 2)
    a1dt, bc = 0.2, 0.2 ** 2 / 2
    v = np.random.default_rng(3).standard_normal(2 * dg.ndof)
    a = BJExtH(dg, w, sig, a1dt, bc).apply(v)
    b = BJExt(dg, w, a1dt, bc).apply(v)
    assert rel(a, b) < 1e-13


def test_stage_solve_with_bjext_h():
    """A stage solve preconditioned with BJ^H_ext reaches the same solution as with
    BJ_ext (the preconditioner changes the path, not the root)."""
    dg = make("euler2", n=3, N=3)
    w0 = smooth_state(dg, seed=11)
    dt = 0.5
    b = w0 + 0.5 * dt * dg.r1(w0)
    sols, its = {}, {}
    for pc in ("bjext", "bjext_h"):
        s = StageSolver(dg, newton_rtol=1e-10, gmres_rtol=1e-6, precond=pc)
        sols[pc] = s.solve(b, 0.5 * dt, dt ** 2 / 12, w0)
        its[pc] = sum(s.log[-1]["gmres"])
    assert rel(sols["bjext_h"], sols["bjext"]) < 1e-9
    assert its["bjext_h"] > 0 and its["bjext"] > 0
