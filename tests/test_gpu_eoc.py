"""Temporal order of HBPC(q, k_max) on the GPU for q = 4, 6, 8 (the order
min(4 + k_max, q) the paper states for its convergence studies, Sec. 4.3 and
Fig. 7): 1-D linear advection, 16 elements, N = 3 on Lobatto nodes, upwind
flux, u0 = sin(2 pi x), T = 1.  The error is taken against exp(T L) u0 for
the operator L of the same semi-discretisation (assembled column by column
from the oracle's R1), so it is the time error alone; both rates over the
halvings dt = 0.1 -> 0.05 -> 0.025 must be within 0.35 of the stated order
(the oracle's own rates on this set-up: 3.97/3.99, 5.09/5.03, 6.20/6.07,
7.83/8.01).  Stage solves: eps_N = 1e-14 (ended by the rounding-floor
test), eps_G = 1e-12, GMRES(64)."""
import numpy as np
import pytest
import scipy.linalg as sla

from gpu_cases import CASES, lib_kwargs, oracle_for, rel
from paper_2109_04804_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def operator_matrix(dg):
    n = dg.ndof
    L = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        L[:, c] = dg.r1(e.reshape(dg.mesh.n_elem, dg.nvar, dg.nnode)).reshape(-1)
    return L


@pytest.mark.parametrize("q,k,expected", [(4, 0, 4), (6, 1, 5), (6, 2, 6), (8, 4, 8)])
def test_temporal_order(q, k, expected):
    from paper_2109_04804_amd.hbpc import Context
    case = CASES["adv1_upwind"]
    dg = oracle_for(case)
    x = dg.node_coords()[0]
    u0 = inputs.advection_sine(x)
    exact = sla.expm(1.0 * operator_matrix(dg)) @ u0.reshape(-1)
    errs = []
    for dt in (0.1, 0.05, 0.025):
        kw = lib_kwargs(case)
        kw.update(q=q, kmax=k, newton_rtol=1e-14, gmres_rtol=1e-12, gmres_restart=64)
        ctx = Context(case["dim"], case["nelem"], case["length"], case["N"], case["equation"], **kw)
        w = torch.tensor(np.ascontiguousarray(u0).reshape(-1), dtype=torch.float64, device="cuda")
        for _ in range(int(round(1.0 / dt))):
            ctx.step(w, dt)
        torch.cuda.synchronize()
        errs.append(rel(w.cpu().numpy(), exact))
        ctx.close()
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    print("HBPC(%d,%d)" % (q, k), "errors", errs, "rates", rates, flush=True)
    assert all(abs(r - expected) < 0.35 for r in rates), (errs, rates)
