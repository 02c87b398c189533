"""Parity at the full benchmark sizes, on sampled elements.

The GPU evaluates the operators on the whole mesh (the launch configuration
the benchmark times); the oracle evaluates each sampled element on the 3^d
patch of elements around it (a periodic 3^d mesh with the same element size,
so the centre element sees exactly its true neighbours; 5^d for viscous
Burgers, whose BR1 lifted gradients of the neighbours read their own
neighbours), which is all the operators depend on.  Samples: seeded random
elements plus the first and last element (periodic wrap in every direction).

Workloads: the 2-D Euler vortex, 128 x 128 elements, N = 5 (2,359,296 DOF),
the 3-D eps-scaled Euler Taylor-Green vortex, 48^3 elements, N = 3
(35,389,440 DOF), and 2-D viscous Burgers with BR1, 64 x 64 elements, N = 4
(102,400 DOF).  Tolerances as in test_gpu_parity.
"""
import time

import numpy as np
import pytest

from gpu_cases import (check, flux_scale, half_storage_bound, half_storage_rss, oracle_for, patch_indices,
                       patch_oracle, rel)
from oracle.solvers import BJExt
from paper_2109_04804_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

VORTEX = dict(dim=2, nelem=[128, 128], length=[10.0, 10.0], N=5, equation="euler", nodes="gauss", flux="rusanov")
TGV = dict(dim=3, nelem=[48, 48, 48], length=[2 * np.pi] * 3, N=3, equation="euler", nodes="gauss",
           flux="rusanov", eps_ref=0.1)
BURGERS = dict(dim=2, nelem=[64, 64], length=[2 * np.pi] * 2, N=4, equation="burgers", nodes="gauss", flux="lf",
               nu=0.01, **{"lambda": 1.0})


def ctx_for(case, **over):
    from paper_2109_04804_amd.hbpc import Context
    kw = {k: v for k, v in case.items() if k not in ("dim", "nelem", "length", "N", "equation")}
    kw.update(over)
    return Context(case["dim"], case["nelem"], case["length"], case["N"], case["equation"], **kw)


def full_state(case, ctx):
    xi, _ = ctx.nodes()
    X = inputs.node_coords(case["dim"], case["nelem"], case["length"], [0, 0, 0], xi)
    if case["equation"] == "burgers":
        return inputs.burgers(X[0], X[1])
    if case["dim"] == 2:
        xc, yc, beta = inputs.vortex_params(inputs.DEFAULT_SEED, beta=5.0)
        return inputs.isentropic_vortex(X[0], X[1], xc, yc, beta)
    # shifted off the mesh faces: on a symmetry plane of the Taylor-Green field
    # lambda_L = lambda_R holds to rounding, and which side the tie rule of the
    # Rusanov max picks (and hence R2 there) is decided by rounding noise
    return inputs.taylor_green(X[0] + 0.1234, X[1] + 0.2345, X[2] + 0.3456, eps=case["eps_ref"])


def samples(nE, k=6, seed=7):
    rng = np.random.default_rng(seed)
    return sorted(set([0, nE - 1] + list(rng.integers(0, nE, size=k))))


def gather(arr, idx, ne):
    return arr.reshape(-1, ne)[idx].reshape(len(idx), -1)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("case", [VORTEX, TGV, BURGERS], ids=["vortex128", "tgv48", "burgers64"])
def test_fullsize_residuals_and_jvp(case):
    ctx = ctx_for(case, gmres_restart=1, precond="none")
    print("full-size case", case["nelem"], "ndof", ctx.ndof, flush=True)
    ne = ctx.block
    nE = int(np.prod(case["nelem"]))
    w = full_state(case, ctx)
    rng = np.random.default_rng(11)
    # sigma smooth, as the Newton iterate sigma ~ R1(w) is: the Hessian term carries
    # (d lambda . dw)(sigma_L - sigma_R) from the side the Rusanov max picks, and
    # where lambda_L = lambda_R to rounding (the nearly uniform far field) that side
    # is decided by rounding noise; a smooth sigma makes the jump, and with it the
    # ambiguity, vanish (a rough sigma does not: at faces where the two Rusanov speeds tie to
    # rounding, the side the tie rule picks differs between the two implementations)
    xi, _ = ctx.nodes()
    X = inputs.node_coords(case["dim"], case["nelem"], case["length"], [0, 0, 0], xi)
    ph = sum(np.sin(2 * np.pi * X[m] / case["length"][m] + m) for m in range(case["dim"]))
    s = 0.1 * np.stack([ph * (1 + 0.3 * v) for v in range(w.shape[1])], axis=1)
    dw = 0.1 * rng.standard_normal(w.shape)
    ds = 0.1 * rng.standard_normal(w.shape)
    dev = lambda x: torch.tensor(np.ascontiguousarray(x).reshape(-1), dtype=torch.float64, device="cuda")
    wd, sd = dev(w), dev(s)
    r1 = torch.empty_like(wd)
    r2 = torch.empty_like(wd)
    ctx.residual1(wd, r1)
    ctx.residual2(wd, sd, r2)
    J = torch.empty(2 * ctx.ndof, dtype=torch.float64, device="cuda")
    a1dt, bc = 0.1, 0.1 ** 2 / 2
    ctx.jvp(wd, sd, a1dt, bc, dev(np.concatenate([dw.ravel(), ds.ravel()])), J)
    J32 = torch.empty(2 * ctx.ndof, dtype=torch.float32, device="cuda")
    f32 = lambda x: np.asarray(x, dtype=np.float32).astype(np.float64)
    w32, s32, dw32, ds32 = f32(w), f32(s), f32(dw), f32(ds)
    ctx.jvp_f32(wd.float(), sd.float(), a1dt, bc,
                torch.cat([dev(dw).float(), dev(ds).float()]), J32)
    R1, R2, JJ, JJ32 = host(r1), host(r2), host(J), host(J32)
    n = ctx.ndof
    radius = 2 if case["equation"] == "burgers" else 1   # BR1: neighbours' lifted gradients
    for e in samples(nE):
        idx = patch_indices(case["nelem"], e, radius)
        dgp, c = patch_oracle(case, None, radius)
        wp, sp, dwp, dsp = (gather(x, idx, ne).reshape(len(idx), dgp.nvar, dgp.nnode) for x in (w, s, dw, ds))
        ref1 = dgp.r1(wp)[c]
        check(R1.reshape(nE, ne)[e], ref1, flux_scale(dgp, wp) , label="R1 e=%d" % e)
        ref2 = dgp.r2(wp, sp)[c]
        check(R2.reshape(nE, ne)[e], ref2, flux_scale(dgp, wp, sp) , label="R2 e=%d" % e)
        Jw, Js = dgp.jvp(wp, sp, dwp, dsp, a1dt, bc)
        got = np.concatenate([JJ[:n].reshape(nE, ne)[e], JJ[n:].reshape(nE, ne)[e]])
        assert rel(got, np.concatenate([Jw[c].ravel(), Js[c].ravel()])) < 1e-12
        p32 = [gather(x, idx, ne).reshape(len(idx), dgp.nvar, dgp.nnode) for x in (w32, s32, dw32, ds32)]
        Jw, Js = dgp.jvp(*p32, a1dt, bc)
        got = np.concatenate([JJ32[:n].reshape(nE, ne)[e], JJ32[n:].reshape(nE, ne)[e]])
        assert rel(got, np.concatenate([Jw[c].ravel(), Js[c].ravel()])) < 5e-5


def test_fullsize_bjext_apply_vortex():
    """BJ_ext build + apply at 128 x 128, N = 5 (element blocks of 144 unknowns)."""
    case = VORTEX
    ctx = ctx_for(case, gmres_restart=1, precond="none")
    ne = ctx.block
    nE = int(np.prod(case["nelem"]))
    w = full_state(case, ctx)
    rng = np.random.default_rng(12)
    X = rng.standard_normal(2 * ctx.ndof)
    a1dt, bc = 0.1, 0.1 ** 2 / 2
    dev = lambda x: torch.tensor(np.ascontiguousarray(x).reshape(-1), dtype=torch.float64, device="cuda")
    ctx.pc_build(dev(w), a1dt, bc, "fp64")
    Y = torch.empty(2 * ctx.ndof, dtype=torch.float64, device="cuda")
    ctx.pc_apply(dev(X), Y)
    Yh = host(Y)
    n = ctx.ndof
    for e in samples(nE, k=4):
        idx = patch_indices(case["nelem"], e)
        dgp, c = patch_oracle(case, None)
        wp = gather(w, idx, ne).reshape(len(idx), dgp.nvar, dgp.nnode)
        pc = BJExt(dgp, wp, a1dt, bc)
        Xp = np.concatenate([gather(X[:n], idx, ne).ravel(), gather(X[n:], idx, ne).ravel()])
        ref = pc.apply(Xp)
        m = len(idx) * ne
        refc = np.concatenate([ref[:m].reshape(len(idx), ne)[c], ref[m:].reshape(len(idx), ne)[c]])
        got = np.concatenate([Yh[:n].reshape(nE, ne)[e], Yh[n:].reshape(nE, ne)[e]])
        assert rel(got, refc) < 1e-10


def test_fullsize_bjext_h_apply_vortex():
    """BJ^H_ext build + apply at 128 x 128, N = 5: sigma a smooth synthetic field (a Newton
    iterate's sigma need not equal R1(w), but is smooth like it: where the two Rusanov speeds of
    a face tie to rounding, in the nearly uniform far field, the Hessian block carries
    (d lambda . e)(sigma_L - sigma_R) from the side the tie rule picks, which rounding noise
    decides, and a rough sigma turns that into an O(1) difference between two correct
    readings).  The Hessian block of an element reads the sigma traces of its neighbours,
    which the 3^2 patch holds.  FP64 within 1e-10; FP32 blocks and vectors within
    max(1e-4, u32 kappa_2(S_e)), u32 = 2^-24."""
    from oracle.solvers import BJExtH
    case = VORTEX
    ctx = ctx_for(case, gmres_restart=1, precond="none")
    ne = ctx.block
    nE = int(np.prod(case["nelem"]))
    n = ctx.ndof
    w = full_state(case, ctx)
    rng = np.random.default_rng(13)
    xi, _ = ctx.nodes()
    Xn = inputs.node_coords(case["dim"], case["nelem"], case["length"], [0, 0, 0], xi)
    ph = sum(np.sin(2 * np.pi * Xn[m] / case["length"][m] + m) for m in range(case["dim"]))
    sig = 0.1 * np.stack([ph * (1 + 0.3 * v) for v in range(w.shape[1])], axis=1)
    X = rng.standard_normal(2 * n)
    a1dt, bc = 0.1, 0.1 ** 2 / 2
    dev = lambda x, dt=torch.float64: torch.tensor(np.ascontiguousarray(x).reshape(-1), dtype=dt, device="cuda")
    ctx.pc_build_hess(dev(w), dev(sig), a1dt, bc, "fp64")
    Y = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    ctx.pc_apply(dev(X), Y)
    Yh = host(Y)
    ctx.pc_build_hess(dev(w), dev(sig), a1dt, bc, "mixed")
    Y32 = torch.empty(2 * n, dtype=torch.float32, device="cuda")
    ctx.pc_apply_f32(dev(X, torch.float32), Y32)
    Y32h = host(Y32)
    for e in samples(nE, k=4):
        idx = patch_indices(case["nelem"], e)
        dgp, c = patch_oracle(case, None)
        wp = gather(w, idx, ne).reshape(len(idx), dgp.nvar, dgp.nnode)
        sp = gather(sig, idx, ne).reshape(len(idx), dgp.nvar, dgp.nnode)
        pc = BJExtH(dgp, wp, sp, a1dt, bc)
        Xp = np.concatenate([gather(X[:n], idx, ne).ravel(), gather(X[n:], idx, ne).ravel()])
        ref = pc.apply(Xp)
        m = len(idx) * ne
        refc = np.concatenate([ref[:m].reshape(len(idx), ne)[c], ref[m:].reshape(len(idx), ne)[c]])
        got = np.concatenate([Yh[:n].reshape(nE, ne)[e], Yh[n:].reshape(nE, ne)[e]])
        got32 = np.concatenate([Y32h[:n].reshape(nE, ne)[e], Y32h[n:].reshape(nE, ne)[e]])
        S = np.eye(ne) - a1dt * pc.K[c] + bc * (pc.K[c] @ pc.K[c] + pc.H[c])
        bound32 = max(1e-4, 2.0 ** -24 * np.linalg.cond(S))
        err, err32 = rel(got, refc), rel(got32, refc)
        print("element", e, "FP64", err, "FP32", err32, "bound", bound32, flush=True)
        assert err < 1e-10
        assert err32 < bound32


def test_fullsize_bjext_h_apply_tgv():
    """BJ^H_ext build + apply at 48^3, N = 3: blocks of 320 unknowns (blocked inversion with the
    Hessian term), built in 22 chunks of K and H.  Smooth sigma as in the 2-D case; FP64 within
    1e-10, FP32 within max(1e-4, u32 kappa_2(S_e))."""
    from oracle.solvers import BJExtH
    case = TGV
    ctx = ctx_for(case, gmres_restart=1, precond="none")
    ne = ctx.block
    nE = int(np.prod(case["nelem"]))
    n = ctx.ndof
    w = full_state(case, ctx)
    rng = np.random.default_rng(14)
    xi, _ = ctx.nodes()
    Xn = inputs.node_coords(case["dim"], case["nelem"], case["length"], [0, 0, 0], xi)
    ph = sum(np.sin(2 * np.pi * Xn[m] / case["length"][m] + m) for m in range(case["dim"]))
    sig = 0.1 * np.stack([ph * (1 + 0.3 * v) for v in range(w.shape[1])], axis=1)
    X = rng.standard_normal(2 * n)
    a1dt, bc = 0.1, 0.1 ** 2 / 2
    dev = lambda x, dt=torch.float64: torch.tensor(np.ascontiguousarray(x).reshape(-1), dtype=dt, device="cuda")
    refs, bounds = {}, {}
    for e in samples(nE, k=1):
        idx = patch_indices(case["nelem"], e)
        dgp, c = patch_oracle(case, None)
        wp = gather(w, idx, ne).reshape(len(idx), dgp.nvar, dgp.nnode)
        sp = gather(sig, idx, ne).reshape(len(idx), dgp.nvar, dgp.nnode)
        pc = BJExtH(dgp, wp, sp, a1dt, bc)
        Xp = np.concatenate([gather(X[:n], idx, ne).ravel(), gather(X[n:], idx, ne).ravel()])
        ref = pc.apply(Xp)
        m = len(idx) * ne
        refs[e] = np.concatenate([ref[:m].reshape(len(idx), ne)[c], ref[m:].reshape(len(idx), ne)[c]])
        S = np.eye(ne) - a1dt * pc.K[c] + bc * (pc.K[c] @ pc.K[c] + pc.H[c])
        bounds[e] = max(1e-4, 2.0 ** -24 * np.linalg.cond(S))
    wd, sd = dev(w), dev(sig)
    for prec, vdt in (("fp64", torch.float64), ("mixed", torch.float32)):
        t0 = time.perf_counter()
        ctx.pc_build_hess(wd, sd, a1dt, bc, prec)
        Y = torch.empty(2 * n, dtype=vdt, device="cuda")
        (ctx.pc_apply if prec == "fp64" else ctx.pc_apply_f32)(dev(X, vdt), Y)
        Yh = host(Y)
        print(prec, "build + apply %.1f s" % (time.perf_counter() - t0), flush=True)
        for e in refs:
            got = np.concatenate([Yh[:n].reshape(nE, ne)[e], Yh[n:].reshape(nE, ne)[e]])
            err = rel(got, refs[e])
            tol = 1e-10 if prec == "fp64" else bounds[e]
            print(prec, "element", e, "rel err", err, "tol", tol, flush=True)
            assert err < tol


def test_fullsize_bjext_apply_tgv():
    """BJ_ext build + apply at 48^3, N = 3 (element blocks of 320 unknowns, the blocked
    inversion; S^-1 of the whole mesh: 90.6 GB in FP64, 45.3 GB in FP32).

    Tolerance: 1e-10 in FP64; in FP32, u_32 kappa_2(S_e) (at least 1e-4), the first-order
    error of forming and applying an inverse in unit roundoff u_32 = 2^-24 (with eps = 0.1
    and a1dt = 0.1 these blocks have kappa_2(S_e) about 1e5); with the blocks stored in FP16,
    four times the root-sum-square scale of rounding S^-1 to FP16 (gpu_cases.half_storage_rss), and
    within twice the componentwise rounding bound gpu_cases.half_storage_bound."""
    case = TGV
    ctx = ctx_for(case, gmres_restart=1, precond="none")
    ne = ctx.block
    nE = int(np.prod(case["nelem"]))
    w = full_state(case, ctx)
    rng = np.random.default_rng(13)
    X = rng.standard_normal(2 * ctx.ndof)
    a1dt, bc = 0.1, 0.1 ** 2 / 2
    dev = lambda x, dt=torch.float64: torch.tensor(np.ascontiguousarray(x).reshape(-1), dtype=dt, device="cuda")
    n = ctx.ndof
    picks = samples(nE, k=1)
    refs, kappa, hb, hr = {}, {}, {}, {}
    for e in picks:
        idx = patch_indices(case["nelem"], e)
        dgp, c = patch_oracle(case, None)
        wp = gather(w, idx, ne).reshape(len(idx), dgp.nvar, dgp.nnode)
        pc = BJExt(dgp, wp, a1dt, bc)
        Xp = np.concatenate([gather(X[:n], idx, ne).ravel(), gather(X[n:], idx, ne).ravel()])
        ref = pc.apply(Xp)
        m = len(idx) * ne
        refs[e] = np.concatenate([ref[:m].reshape(len(idx), ne)[c], ref[m:].reshape(len(idx), ne)[c]])
        Ke = pc.K[c]
        kappa[e] = np.linalg.cond(np.eye(ne) - a1dt * Ke + bc * (Ke @ Ke))
        hb[e] = half_storage_bound(pc.K[c:c + 1], X[:n].reshape(nE, ne)[e:e + 1], X[n:].reshape(nE, ne)[e:e + 1],
                                   a1dt, bc, refs[e])
        hr[e] = half_storage_rss(pc.K[c:c + 1], X[:n].reshape(nE, ne)[e:e + 1], X[n:].reshape(nE, ne)[e:e + 1],
                                 a1dt, bc, refs[e])
    wd = dev(w)
    half = ctx_for(case, gmres_restart=1, precond="none", pc_half=1)
    for prec, vdt, tol in (("fp64", torch.float64, 1e-10), ("mixed", torch.float32, 1e-4),
                           ("mixed16", torch.float32, 1e-3)):
        if prec == "mixed16":   # FP16 blocks: a second context (its own blocks), the FP32 ones freed first
            ctx.close()
            ctx, prec = half, "mixed"
        u = 2.0 ** -24
        print("build", prec, "half" if ctx is half else "", flush=True)
        t0 = time.perf_counter()
        ctx.pc_build(wd, a1dt, bc, prec)
        torch.cuda.synchronize()
        print("build", prec, "%.1f ms" % (1e3 * (time.perf_counter() - t0)), flush=True)
        Y = torch.empty(2 * n, dtype=vdt, device="cuda")
        if prec == "fp64":
            ctx.pc_apply(dev(X), Y)
        else:
            ctx.pc_apply_f32(dev(X, torch.float32), Y)
        Yh = host(Y)
        del Y
        for e in picks:
            got = np.concatenate([Yh[:n].reshape(nE, ne)[e], Yh[n:].reshape(nE, ne)[e]])
            err = rel(got, refs[e])
            if ctx is half:
                # the statistical scale of the rounding (4x) and the rigorous componentwise bound
                print("FP16 element", e, "rss scale", hr[e], "componentwise bound", hb[e], flush=True)
                assert err < 2 * hb[e] + 1e-5
                bound = 4 * hr[e] + 1e-5
            else:
                bound = tol if prec == "fp64" else max(tol, u * kappa[e])
            print(prec, "element", e, "rel err", err, "kappa", kappa[e], "bound", bound, flush=True)
            assert err < bound
    ctx.close()


def _integral(case, ctx, w):
    """Per-variable integral of the DG solution: sum over elements of
    (prod_m h_m / 2) sum_nodes (prod_m omega) w."""
    _, om = ctx.nodes()
    d = case["dim"]
    wt = om
    for _ in range(d - 1):
        wt = np.multiply.outer(om, wt)   # node index i fastest: weight omega_i omega_j ...
    wt = wt.reshape(-1)
    jac = np.prod([case["length"][m] / case["nelem"][m] / 2 for m in range(d)])
    nE = int(np.prod(case["nelem"]))
    return jac * np.einsum("evn,n->v", w.reshape(nE, -1, wt.size), wt)


@pytest.mark.parametrize("case,dt,precision", [(VORTEX, 0.1, "mixed"), (TGV, 0.027, "mixed"),
                                              (BURGERS, 0.1, "fp64")], ids=["vortex128", "tgv48", "burgers64"])
def test_fullsize_step_conserves(case, dt, precision):
    """One mixed-precision HBPC(6,4) step at the benchmark's sizes and settings (eps_N 1e-8,
    FGMRES(30) at eps_G 1e-3, BJ_ext): the integral of every conserved variable is kept to the
    Newton tolerance (the stage equations conserve it exactly; the inexact solves leave
    |G| <= 1e-8 |G0|), the state moves and stays finite."""
    ctx = ctx_for(case, q=6, kmax=4, newton_rtol=1e-8, gmres_rtol=1e-3, gmres_restart=30, precision=precision,
                  precond="bjext")
    w0 = full_state(case, ctx)
    wd = torch.tensor(np.ascontiguousarray(w0).reshape(-1), dtype=torch.float64, device="cuda")
    print("full-size step", case["nelem"], "dt", dt, flush=True)
    st = ctx.step(wd, dt)
    print({k: st[k] for k in ("n_solves", "newton_its", "gmres_its", "t_step_ms")}, flush=True)
    w1 = host(wd)
    assert np.isfinite(w1).all()
    m0, m1 = _integral(case, ctx, w0), _integral(case, ctx, w1)
    scale = _integral(case, ctx, np.abs(w0))
    print("integrals", m0, "change", m1 - m0, flush=True)
    # one scale for all variables: the Taylor-Green field has no z momentum at all
    assert np.all(np.abs(m1 - m0) <= 1e-8 * scale.max())
    assert np.abs(w1 - w0.reshape(-1)).max() > 1e-6
    ctx.close()
