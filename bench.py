#!/usr/bin/env python
"""Benchmark of the HBPC hot path on one MI355X.

Workload (default): 2-D compressible Euler isentropic vortex on the periodic
[0,10]^2, gamma 1.4, background Mach 0.5, strength 5, seeded centre
(seed 2109), DGSEM N = 5 on Gauss nodes, 128 x 128 elements (2,359,296 DOF),
Rusanov flux, HBPC(6,4) (3 nodes c = 0, 1/2, 1; 4 corrector sweeps), dt = 0.1,
Newton tolerance 1e-8, FGMRES(30) with eps_G = 1e-3, BJ_ext blocks built once
per predictor stage; the two corrector stages of each sweep solved side by
side on one set of blocks built at the first stage's state in the first sweep
(--pc-rebuild paired; the BJ^H_ext forms and the learned_first / learned_guess
variants keep one set per corrector stage, per_stage).  Three forms are timed:
  fp64     all-FP64, BJ_ext;
  mixed    FP64 Newton, FP32 Krylov vectors, JVP and BJ_ext;
  learned  as mixed with the learned preconditioner (BF16 network, BJ_ext as
           fallback after a 5-iteration probe cycle of the network in each
           solve, --pc-probe-its), trained before timing on Newton pairs of
           FP64 solves of seeded vortices on the same mesh.
On request (--forms) also fp64_h / mixed_h (as fp64 / mixed with BJ^H_ext, the
element-local Hessian block kept in the preconditioner), mixed16 (S^-1 stored
in FP16) and the learned_first / learned_guess variants.
A step is one full HBPC step (all stage solves) on the state resident in HBM;
inputs are synthetic.  Other workloads (--workload): a 32 x 32 vortex, 2-D
viscous Burgers 64 x 64 N = 4, and the 3-D eps-scaled Euler Taylor-Green
vortex (eps = 0.1) with N = 3 on 48^3 (acoustic CFL about 9) or 16^3 (CFL
about 20) elements; there the learned form is trained on translated
Taylor-Green fields.

Prints ONE JSON line: value = DOF-steps/s of the headline form (learned, as
the metric names it), the other forms beside it, the roofline of the dominant
kernel (HIP events around that kernel's launches on the library's stream
during the timed steps, algorithmic bytes per launch, measured HBM traffic
from the committed counter summary), a per-kernel breakdown of the last
warm-up step, and the FP64 NumPy oracle timed on the host on a bounded sample
of the workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "HBPC DOF-steps/s at 1e-8 Newton tol, learned+FP32 vs plain FP64; HBM GB/s"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3

WORKLOADS = {
    "euler_vortex_128x128_N5": dict(dim=2, nelem=[128, 128], length=[10.0, 10.0], N=5, dt=0.1),
    # small variant for quick checks
    "euler_vortex_32x32_N5": dict(dim=2, nelem=[32, 32], length=[10.0, 10.0], N=5, dt=0.1),
    # viscous Burgers with BR1: u0 = 0.5 + 0.25 sin(x+y) + seeded noise, nu = 0.01, LF lambda = 1
    "burgers_64x64_N4": dict(dim=2, nelem=[64, 64], length=[2 * 3.141592653589793] * 2, N=4, dt=0.1,
                             equation="burgers"),
    # 3-D eps-scaled Euler (eps = 0.1, Mach 0.1) Taylor-Green vortex, N = 3 (blocks of 320 unknowns),
    # dt at an acoustic CFL of about 9: dt (|v| + c/eps) (N+1) / h with c/eps ~ 10, |v| <= 1 (at CFL 20
    # corrector stages need more than 7000 FGMRES(30) iterations per Newton step with BJ_ext on 48^3)
    "euler_tgv_48x48x48_N3": dict(dim=3, nelem=[48, 48, 48], length=[2 * 3.141592653589793] * 3, N=3,
                                  dt=0.027, equation="euler", field="tgv", eps_ref=0.1),
    # the same workload at its configured acoustic CFL of about 20 (dt = 0.06), with the longer restart
    # that the paper's Euler runs use (Sec. 4.1.2 restarts after 700): FGMRES(200) in FP32, FGMRES(100) in
    # FP64 (101 + 100 basis vectors of 70.8M FP64 values = 114 GB beside 91 GB of FP64 S^-1 blocks); one
    # stage solve at a time (`rebuild`), since a second system's basis would not fit beside them
    "euler_tgv_48x48x48_N3_cfl20": dict(dim=3, nelem=[48, 48, 48], length=[2 * 3.141592653589793] * 3, N=3,
                                        dt=0.06, equation="euler", field="tgv", eps_ref=0.1,
                                        restart={"fp64": 100, "mixed": 200}, rebuild="per_stage"),
    # the paper's viscous Taylor-Green vortex (Sec. 5.3.3): Navier-Stokes with BR2 lifting, mu = 1.25e-3
    # (Re = 800), eps = 0.1, N = 3 on 32^3 elements of [0, 2 pi]^3, HBPC(4,0) at dt = 0.25 (acoustic CFL
    # about 56), FGMRES(200) in FP32 / FGMRES(100) in FP64
    "ns_tgv_32x32x32_N3": dict(dim=3, nelem=[32, 32, 32], length=[2 * 3.141592653589793] * 3, N=3, dt=0.25,
                               equation="navier_stokes", field="tgv", eps_ref=0.1, mu=1.25e-3, q=4, kmax=0,
                               restart={"fp64": 100, "mixed": 200}, rebuild="per_stage"),
    # the same at a tenth of the step (acoustic CFL about 5.6) with the bench's HBPC(6,4)
    "ns_tgv_32x32x32_N3_dt0025": dict(dim=3, nelem=[32, 32, 32], length=[2 * 3.141592653589793] * 3, N=3,
                                      dt=0.025, equation="navier_stokes", field="tgv", eps_ref=0.1, mu=1.25e-3),
    # the same CFL on a 16^3 mesh
    "euler_tgv_16x16x16_N3": dict(dim=3, nelem=[16, 16, 16], length=[2 * 3.141592653589793] * 3, N=3,
                                  dt=0.18, equation="euler", field="tgv", eps_ref=0.1),
}


def initial_state(ctx, wl):
    import numpy as np
    from paper_2109_04804_amd import inputs
    xi, _ = ctx.nodes()
    X = inputs.node_coords(wl["dim"], wl["nelem"], wl["length"], [0.0] * wl["dim"], xi)
    if wl.get("field") == "tgv":
        return inputs.taylor_green(X[0], X[1], X[2], gamma=1.4, eps=wl["eps_ref"])
    if wl.get("equation") == "burgers":
        return inputs.burgers(X[0], X[1], seed=inputs.DEFAULT_SEED)
    xc, yc, beta = inputs.vortex_params(inputs.DEFAULT_SEED, beta=5.0)
    return inputs.isentropic_vortex(X[0], X[1], xc, yc, beta, mach=0.5, gamma=1.4, box=wl["length"][0])


def _eqkw(wl):
    if wl.get("equation") == "burgers":
        return dict(flux="lf", nu=0.01, **{"lambda": 1.0})
    kw = dict(flux="rusanov", gamma=1.4, eps_ref=wl.get("eps_ref", 1.0))
    if wl.get("equation") == "navier_stokes":
        kw["mu"] = wl["mu"]
    return kw


def scheme_of(wl):
    """(q, k_max) of a workload: HBPC(6,4) unless it names another."""
    return wl.get("q", 6), wl.get("kmax", 4)


def training_state(wl, X, seed):
    """Seeded training state: a vortex with centre in [3,7]^2 and strength in [3,7]
    (2-D workloads), or the Taylor-Green field translated by an offset drawn
    uniformly from [0, 2 pi)^3 (3-D workload)."""
    import numpy as np
    from paper_2109_04804_amd import inputs
    if wl.get("field") == "tgv":
        off = np.random.default_rng(seed).uniform(0.0, 2 * np.pi, size=3)
        return inputs.taylor_green(X[0] + off[0], X[1] + off[1], X[2] + off[2], gamma=1.4, eps=wl["eps_ref"])
    xc, yc, beta = inputs.vortex_params(seed)
    return inputs.isentropic_vortex(X[0], X[1], xc, yc, beta, mach=0.5, gamma=1.4, box=wl["length"][0])


def train_learned(wl, samples=20480, per_correction=512, seeds=(1, 2), epochs=20):
    """Training of the learned preconditioner on the workload's mesh: Newton pairs
    from FP64 BJ_ext solves at eps_G 1e-6 of seeded states (training_state; one
    HBPC(6,4) step per seed until `samples` pairs are in), then BF16 Adam.
    Returns (parameters, report)."""
    import numpy as np
    import torch
    from paper_2109_04804_amd import inputs
    from paper_2109_04804_amd.hbpc import Context
    t0 = time.perf_counter()
    q, kmax = scheme_of(wl)
    col = Context(wl["dim"], wl["nelem"], wl["length"], wl["N"], wl.get("equation", "euler"), q=q, kmax=kmax,
                  newton_rtol=1e-8,
                  gmres_rtol=1e-6, gmres_restart=restart_of(wl, "fp64"), gmres_maxit=7000, precond="bjext",
                  precision="fp64",
                  **_eqkw(wl))
    n_in, H, n_out, n_p = col.mlp_shape()
    X = torch.zeros(samples * n_in, dtype=torch.float32, device="cuda")
    T = torch.zeros(samples * n_out, dtype=torch.float32, device="cuda")
    col.mlp_collect(X, T, samples, per_correction, 2109, source="newton")
    xi, _ = col.nodes()
    Xc = inputs.node_coords(wl["dim"], wl["nelem"], wl["length"], [0.0] * wl["dim"], xi)
    for seed in seeds:
        w0 = training_state(wl, Xc, seed)
        w = torch.tensor(np.ascontiguousarray(w0).reshape(-1), dtype=torch.float64, device="cuda")
        st = col.step(w, wl["dt"])
        print("[bench] learned: collected %d pairs (seed %d, %d Krylov iterations)" % (col.mlp_collected(), seed,
              st["gmres_its"]), file=sys.stderr, flush=True)
        if col.mlp_collected() >= samples:
            break
    count = col.mlp_collected()
    col.close()
    t_collect = time.perf_counter() - t0
    tr = Context(wl["dim"], wl["nelem"], wl["length"], wl["N"], wl.get("equation", "euler"), precond="learned",
                 precision="mixed",
                 **_eqkw(wl))
    tr.mlp_init(7)
    log = tr.train_mlp(X, T, count, epochs=epochs, batch=256, lr=1e-3, seed=5, precision="bf16")
    out = torch.zeros(n_p, dtype=torch.float32, device="cuda")
    tr.mlp_get_params(out)
    tr.close()
    del X, T
    print("[bench] learned: trained on %d pairs, loss %.4g -> %.4g, %.1f s" % (count, log["loss_first"],
          log["loss_last"], log["ms"] * 1e-3), file=sys.stderr, flush=True)
    return out, {"pairs": count, "source": "Newton corrections of FP64 BJ_ext solves, eps_G 1e-6",
                 "per_correction": per_correction,
                 "seeds": list(seeds), "collect_s": round(t_collect, 2), "train_ms": round(log["ms"], 1),
                 "adam_steps": log["steps"], "loss_first_epoch": log["loss_first"],
                 "loss_last_epoch": log["loss_last"]}


FORMS = ("fp64", "mixed", "learned", "learned_first", "learned_guess", "mixed16", "fp64_h", "mixed_h")


def form_settings(form):
    """(precision, preconditioner, FP16 blocks) of a benchmark form."""
    if form not in FORMS:
        raise ValueError("unknown form %r (one of %s)" % (form, ", ".join(FORMS)))
    precision = "fp64" if form in ("fp64", "fp64_h") else "mixed"
    if form.startswith("learned"):
        pc = form
    else:
        pc = "bjext_h" if form.endswith("_h") else "bjext"
    return precision, pc, 1 if form == "mixed16" else 0


def restart_of(wl, precision):
    """FGMRES restart length of a workload in a precision (30 unless the workload names one)."""
    r = wl.get("restart", 30)
    return r[precision] if isinstance(r, dict) else r


def run_form(wl, form, steps, warmup, theta=None, pc_rebuild="per_solve", pc_reuse_steps=4, pc_probe_its=0):
    import numpy as np
    import torch
    from paper_2109_04804_amd.hbpc import Context
    precision, pc, half = form_settings(form)
    if pc_rebuild == "paired" and pc not in ("bjext", "learned"):
        pc_rebuild = "per_stage"   # the paired corrector solves run BJ_ext or the learned preconditioner
    q, kmax = scheme_of(wl)
    ctx = Context(wl["dim"], wl["nelem"], wl["length"], wl["N"], wl.get("equation", "euler"), q=q, kmax=kmax,
                  newton_rtol=1e-8, gmres_rtol=1e-3, gmres_restart=restart_of(wl, precision), gmres_maxit=7000,
                  precond=pc,
                  precision=precision, pc_fallback=0.5, pc_rebuild=pc_rebuild, pc_half=half,
                  pc_reuse_steps=pc_reuse_steps, pc_probe_its=pc_probe_its, **_eqkw(wl))
    if pc.startswith("learned"):
        ctx.mlp_set_params(theta)
    w0 = initial_state(ctx, wl)
    w = torch.tensor(np.ascontiguousarray(w0).reshape(-1), dtype=torch.float64, device="cuda")
    # the last warm-up step records every launch (kernel breakdown, choice of the dominant kernel);
    # the timed steps record only the dominant kernel's launches, so that events around every other
    # launch do not slow the timed region
    breakdown = None
    for i in range(warmup):
        if i == warmup - 1:
            ctx.profile_read(reset=True)
            ctx.profile_enable(True)
        st = ctx.step(w, wl["dt"])
        print("[bench] %s warmup %d: newton %d gmres %d fallbacks %d  %.1f ms" % (form, i, st["newton_its"],
              st["gmres_its"], st["pc_fallbacks"], st["t_step_ms"]), file=sys.stderr, flush=True)
    if warmup > 0:
        breakdown = ctx.profile_read(reset=True)
        ctx.profile_enable(True)
        ctx.profile_only(dominant_class(breakdown))
    else:
        ctx.profile_enable(True)
    stats = []
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    t_start.record()
    for i in range(steps):
        st = ctx.step(w, wl["dt"])
        stats.append(st)
        print("[bench] %s step %d: newton %d gmres %d fallbacks %d  %.1f ms" % (form, i, st["newton_its"],
              st["gmres_its"], st["pc_fallbacks"], st["t_step_ms"]), file=sys.stderr, flush=True)
    t_end.record()
    torch.cuda.synchronize()
    ms = t_start.elapsed_time(t_end)
    prof = ctx.profile_read(reset=True)
    ctx.profile_enable(False)
    if breakdown is None:
        breakdown = prof
    finite = bool(torch.isfinite(w).all().item())
    ctx.close()
    return {"ms_total": ms, "ms_per_step": ms / steps, "dof": ctx.ndof,
            "newton_its": [s["newton_its"] for s in stats], "gmres_its": [s["gmres_its"] for s in stats],
            "pc_builds": [s["pc_builds"] for s in stats], "pc_fallbacks": [s["pc_fallbacks"] for s in stats],
            "n_solves": [s["n_solves"] for s in stats], "kernels": breakdown, "timed_kernels": prof,
            "finite": finite}


SINGLE_KERNEL_CLASSES = ("bj_apply", "bj_apply4", "bj_invert", "jvp", "pcpre", "kcol", "trace", "res", "r1", "r2",
                         "gs_update")


def dominant_class(prof):
    """Largest total time among the classes that are one kernel each."""
    cand = {k: v for k, v in prof.items() if k in SINGLE_KERNEL_CLASSES}
    return max(cand.items(), key=lambda kv: kv[1]["total_ms"])[0]


def roofline_of(prof, workload, form):
    """The dominant kernel's launches in the timed steps (prof: per class);
    HBM-bound kernels against 8 TB/s, the BJ_ext inversion against the vector
    peak of its arithmetic (FP64 in the fp64 form, FP32 otherwise)."""
    name = dominant_class(prof)
    k = prof[name]
    per_launch_ms = k["total_ms"] / k["launches"]
    if name == "bj_invert":
        peak = FP64_PEAK_TFLOPS if form in ("fp64", "fp64_h") else FP32_PEAK_TFLOPS
        ach = k["flops"] / k["launches"] / (per_launch_ms * 1e-3) / 1e12
        return {"kernel": name, "bound": "alu", "achieved": ach, "peak": peak, "unit": "TFLOP/s",
                "frac": ach / peak, "traffic": None,
                "avg_launch_ms": per_launch_ms, "launches": k["launches"]}
    ach = k["bytes"] / k["launches"] / (per_launch_ms * 1e-3) / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": measured_traffic(name, workload),
            "bytes_per_launch": k["bytes"] / k["launches"], "avg_launch_ms": per_launch_ms,
            "launches": k["launches"]}


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a reference copy), or None when
    there is none for this workload or the kernel's source changed since."""
    import glob
    import hashlib
    import re
    for path in glob.glob(os.path.join(ROOT, "profiles", "%s_*_traffic.md" % kernel)):
        m = re.search(r"<!-- traffic (\{.*\}) -->", open(path).read())
        if not m:
            continue
        rec = json.loads(m.group(1))
        if rec.get("kernel") != kernel or rec.get("workload") != workload:
            continue
        src = os.path.join(ROOT, rec["source"])
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["sha256"]:
            return None
        return float(rec["bytes_per_launch"])
    return None


PARITY_N = 8   # elements per direction of the parity and CPU-baseline sample


def parity_sample():
    """The vortex workload on a reduced 8 x 8-element mesh of the same domain (N = 5):
    (oracle DGSEM, initial state)."""
    from oracle.dgsem import DGSEM, Mesh
    from oracle.equations import Euler
    from paper_2109_04804_amd import inputs
    dg = DGSEM(Mesh(2, [PARITY_N, PARITY_N], [10.0, 10.0]), 5, Euler(2), flux="rusanov")
    X = dg.node_coords()
    xc, yc, beta = inputs.vortex_params(inputs.DEFAULT_SEED, beta=5.0)
    return dg, inputs.isentropic_vortex(X[0], X[1], xc, yc, beta)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline():
    """FP64 NumPy oracle: one HBPC(6,4) step of the parity sample (dt = 0.1, eps_N 1e-8,
    GMRES(30) + BJ_ext), timed on one thread and on all the host threads the process may
    use (OMP_NUM_THREADS, else the CPU count).  Returns (report, the oracle's new state)."""
    from threadpoolctl import threadpool_limits
    from oracle.solvers import StageSolver, dg_hbpc_step
    dg, w = parity_sample()
    runs = {}
    out = None
    threads_all = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    for threads in sorted({1, threads_all}):
        sol = StageSolver(dg, newton_rtol=1e-8, gmres_rtol=1e-3, gmres_restart=30)
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            out = dg_hbpc_step(dg, w, 0.1, 6, 4, sol)
            runs[threads] = time.perf_counter() - t0
        print("[bench] oracle step on %d thread(s): %.1f s" % (threads, runs[threads]), file=sys.stderr, flush=True)
    rep = {"value": dg.ndof / runs[1], "unit": "DOF-steps/s", "cores": 1, "kind": "oracle",
           "sample": "one HBPC(6,4) step, vortex on %dx%d elements of [0,10]^2 (%d DOF), N=5, dt=0.1, "
                     "eps_N 1e-8, GMRES(30)+BJ_ext, NumPy FP64, 1 thread, %.1f s"
                     % (PARITY_N, PARITY_N, dg.ndof, runs[1]),
           "all_cores": {"value": dg.ndof / runs[threads_all], "cores": threads_all, "seconds": runs[threads_all]},
           "cpu_model": cpu_model()}
    return rep, out


def form_parity(wl, forms, ref, theta, pc_rebuild, pc_reuse_steps, pc_probe_its):
    """Relative L2 difference between one GPU step of each form on the parity sample and the
    oracle's step (both at eps_N 1e-8): the error against the FP64 oracle of every timed form."""
    import numpy as np
    import torch
    from paper_2109_04804_amd.hbpc import Context
    _, w0 = parity_sample()
    out = {}
    for f in forms:
        precision, pc, half = form_settings(f)
        rebuild = "per_stage" if (pc_rebuild == "paired" and pc not in ("bjext", "learned")) else pc_rebuild
        ctx = Context(2, [PARITY_N, PARITY_N], [10.0, 10.0], 5, "euler", q=6, kmax=4, newton_rtol=1e-8,
                      gmres_rtol=1e-3, gmres_restart=30, gmres_maxit=7000, precond=pc, precision=precision,
                      pc_fallback=0.5, pc_rebuild=rebuild, pc_half=half, pc_reuse_steps=pc_reuse_steps,
                      pc_probe_its=pc_probe_its, flux="rusanov", gamma=1.4, eps_ref=1.0)
        if pc.startswith("learned"):
            ctx.mlp_set_params(theta)
        w = torch.tensor(np.ascontiguousarray(w0).reshape(-1), dtype=torch.float64, device="cuda")
        st = ctx.step(w, 0.1)
        got = w.cpu().numpy()
        ctx.close()
        out[f] = float(np.linalg.norm(got - ref.ravel()) / np.linalg.norm(ref.ravel()))
        print("[bench] parity %s: rel L2 %.3e (fallbacks %d)" % (f, out[f], st["pc_fallbacks"]), file=sys.stderr,
              flush=True)
    return out


# Preconditioner study of Sec. 4.1.2 (Figs. 4 and 5): the eps-scaled density wave of
# Eq. euler_convtest on [-1,1]^2, 16^2 elements, N = 5, Eq. Riemann as printed with the Euler
# set-up's lambda = diag(1/eps, 1, 1, 1/eps) (lf_literal; the Rusanov flux on request), eps_G 1e-3,
# eps_N 1e-8, FGMRES restarted after 700 iterations and at most 7000 Krylov iterations per Newton
# step, preconditioners rebuilt at every Newton iterate; one time step of the HBPC(4,0) predictor
# per point.  Time steps within the ranges the paper plots for each eps.
STUDY_DT = {1.0: [0.0125, 0.05, 0.2, 0.8], 0.1: [0.003125, 0.0125, 0.05, 0.2],
            0.01: [0.00078125, 0.003125, 0.0125, 0.025]}
STUDY_PC = ("none", "bjext", "bjext_h")


def precond_study(precision, flux="lf_literal", restart=700):
    """Rows (eps, dt, preconditioner, Krylov and Newton iterations, ms per step); a point
    without convergence within the iteration cap is reported with its error code."""
    import numpy as np
    import torch
    from paper_2109_04804_amd import inputs
    from paper_2109_04804_amd.hbpc import Context, HbpcError
    rows = []
    for eps, dts in STUDY_DT.items():
        for dt in dts:
            for pc in STUDY_PC:
                ctx = Context(2, [16, 16], [2.0, 2.0], 5, "euler", origin=(-1.0, -1.0, 0.0), q=4, kmax=0,
                              newton_rtol=1e-8, gmres_rtol=1e-3, gmres_restart=restart, gmres_maxit=7000,
                              precision=precision, precond=pc, pc_rebuild="per_newton_it", flux=flux,
                              gamma=1.4, eps_ref=eps)
                xi, _ = ctx.nodes()
                X = inputs.node_coords(2, [16, 16], [2.0, 2.0], [-1.0, -1.0], xi)
                w0 = torch.tensor(inputs.density_wave(X, a=0.3, eps=eps).reshape(-1), dtype=torch.float64,
                                  device="cuda")
                row = {"eps": eps, "dt": dt, "precond": pc}
                try:
                    for rep_ in range(2):   # the first step warms up, the second is timed
                        w = w0.clone()
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        st = ctx.step(w, dt)
                        torch.cuda.synchronize()
                        ms = (time.perf_counter() - t0) * 1e3
                    row.update(gmres_its=st["gmres_its"], newton_its=st["newton_its"], ms=ms,
                               pc_builds=st.get("pc_builds"))
                except HbpcError as e:
                    row.update(error=e.code)
                ctx.close()
                print("[study] %s" % json.dumps(row), file=sys.stderr, flush=True)
                rows.append(row)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="euler_vortex_128x128_N5", choices=sorted(WORKLOADS))
    ap.add_argument("--forms", default="fp64,mixed,learned",
                    help="comma list of fp64 (BJ_ext FP64), mixed (BJ_ext, FP32 Krylov), learned "
                         "(learned preconditioner with BJ_ext fallback, FP32 Krylov, BF16 network), "
                         "learned_first (network for the first FGMRES direction, then BJ_ext), "
                         "learned_guess (network correction as FGMRES initial guess, then BJ_ext), mixed16 "
                         "(as mixed with the BJ_ext blocks stored in FP16), fp64_h / mixed_h (as fp64 / mixed "
                         "with BJ^H_ext)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pc-rebuild", default=None,
                    choices=["per_solve", "per_stage", "across_steps", "paired"],
                    help="BJ_ext builds: the two corrector stages of a sweep solved side by side on one set of "
                         "blocks built in the first sweep (paired, the default except on the workloads with "
                         "FGMRES(100/200), whose basis leaves no room for a second system; the BJ^H_ext forms and the "
                         "learned_first / learned_guess variants run per_stage), kept per corrector stage "
                         "across sweeps (per_stage), "
                         "once per stage solve, or every stage's blocks kept across --pc-reuse-steps time steps")
    ap.add_argument("--pc-reuse-steps", type=int, default=4)
    ap.add_argument("--pc-probe-its", type=int, default=5,
                    help="learned form: length of the network's first restart cycle per solve, judged at the "
                         "fallback's mean rate per iteration (0: the full restart cycle)")
    ap.add_argument("--study", choices=["precond_eps"], default=None,
                    help="instead of the benchmark: the preconditioner study over eps and dt (none, BJ_ext, "
                         "BJ^H_ext; one JSON line)")
    ap.add_argument("--study-precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--study-flux", choices=["lf_literal", "rusanov"], default="lf_literal")
    ap.add_argument("--study-restart", type=int, default=700)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run a plain device copy of this many bytes three times (reference dispatch "
                         "for scaling hardware byte counters)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py: libhbpc runs on one GPU; --gpus %d is not supported (the path would shard by "
              "elements with a face-trace halo exchange per operator and one all-reduce per "
              "Gram-Schmidt pass)" % a.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(int(os.environ.get("LOCAL_RANK", "0")))
    if a.study == "precond_eps":
        rows = precond_study(a.study_precision, a.study_flux, a.study_restart)
        print(json.dumps({"study": "precond_eps", "precision": a.study_precision, "flux": a.study_flux,
                          "setup": "density wave, [-1,1]^2, 16^2 elements, N = 5, HBPC(4,0) predictor, "
                                   "eps_G 1e-3, eps_N 1e-8, FGMRES(%d), cap 7000 per Newton step, "
                                   "preconditioner rebuilt at every Newton iterate" % a.study_restart,
                          "rows": rows}))
        return
    if a.copy_bytes > 0:
        src = torch.ones(a.copy_bytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print("[bench] reference copy of %d bytes done" % a.copy_bytes, file=sys.stderr, flush=True)
    wl = WORKLOADS[a.workload]
    if a.pc_rebuild is None:   # paired unless the workload's Krylov basis leaves no room for a second system
        a.pc_rebuild = wl.get("rebuild", "paired")
    forms = [f for f in a.forms.split(",") if f]
    for f in forms:
        form_settings(f)   # an unknown form fails before any form runs
    if wl.get("equation") == "burgers":
        forms = [f for f in forms if not f.startswith("learned")]   # the network is trained on Euler states
    res = {}
    theta, train_report = None, None
    if any(f.startswith("learned") for f in forms):
        # 3-D: more pairs per Newton correction, so that one FP64 collection step suffices
        theta, train_report = train_learned(wl, per_correction=1024 if wl["dim"] == 3 else 512)
    for f in forms:
        res[f] = run_form(wl, f, a.steps, a.warmup, theta, a.pc_rebuild, a.pc_reuse_steps, a.pc_probe_its)
    head = "learned" if "learned" in res else ("mixed" if "mixed" in res else forms[0])
    h = res[head]
    dof = h["dof"]
    value = dof * a.steps / (h["ms_total"] * 1e-3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"learned": "f64+f32+bf16", "learned_first": "f64+f32+bf16", "learned_guess": "f64+f32+bf16",
                  "mixed": "f64+f32",
                  "mixed16": "f64+f32+f16", "fp64": "f64", "fp64_h": "f64", "mixed_h": "f64+f32"}[head],
        "data": "synthetic",
        "config": {"workload": a.workload, "dof": dof, "scheme": "HBPC(%d,%d)" % scheme_of(wl), "dt": wl["dt"],
                   "newton_rtol": 1e-8,
                   "krylov": "FGMRES(%d), eps_G 1e-3" % restart_of(wl, form_settings(head)[0]),
                   "pc_rebuild": a.pc_rebuild,
                   "pc_reuse_steps": a.pc_reuse_steps if a.pc_rebuild == "across_steps" else None,
                   "pc_probe_its": a.pc_probe_its,
                   "precond": {"learned": "learned (BJ_ext fallback 0.5)",
                               "learned_first": "learned first direction, then BJ_ext",
                               "learned_guess": "learned initial guess, then BJ_ext", "mixed": "BJ_ext",
                               "mixed16": "BJ_ext, FP16 blocks", "fp64": "BJ_ext", "fp64_h": "BJ^H_ext",
                               "mixed_h": "BJ^H_ext"}[head], "form": head},
        "forms": {f: {"dof_steps_per_s": dof * a.steps / (r["ms_total"] * 1e-3), "ms_per_step": r["ms_per_step"],
                      "newton_its": r["newton_its"], "gmres_its": r["gmres_its"], "pc_fallbacks": r["pc_fallbacks"],
                      "n_solves": r["n_solves"], "finite": r["finite"]}
                  for f, r in res.items()},
        "roofline": roofline_of(h["timed_kernels"], a.workload, head),
        "kernels_from": "last warm-up step, events around every launch",
        "kernels": {f: {k: {"launches": v["launches"], "total_ms": round(v["total_ms"], 3),
                            "GBps": (v["bytes"] / (v["total_ms"] * 1e-3) / 1e9) if v["total_ms"] > 0 else None}
                        for k, v in r["kernels"].items()} for f, r in res.items()},
    }
    if "fp64" in res and head != "fp64":
        out["speedup_vs_fp64"] = res["fp64"]["ms_per_step"] / h["ms_per_step"]
    if train_report:
        out["learned_training"] = train_report
    if not a.no_cpu_baseline:
        cb, ref = cpu_baseline()
        out["cpu_baseline"] = cb
        if wl["dim"] == 2 and wl.get("equation", "euler") == "euler":
            out["parity"] = {"sample": "vortex %dx%d elements, N=5, one HBPC(6,4) step at dt=0.1 in each timed "
                                       "form's composition" % (PARITY_N, PARITY_N),
                             "reference": "FP64 oracle step, eps_N 1e-8, GMRES(30)+BJ_ext",
                             "bound": 1e-8,
                             "rel_l2": form_parity(wl, forms, ref, theta, a.pc_rebuild, a.pc_reuse_steps,
                                                   a.pc_probe_its)}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
