"""Operator micro-benchmark: each hot-path entry point of libhbpc, called repeatedly on one
workload's state, with the library's per-kernel timing (HIP events around every launch on its
stream) and the algorithmic bytes of each kernel.  Used to measure the operator kernels
against the HBM roofline and as the program that rocprofv3 profiles.

    python paper_2109_04804_amd/opbench.py --workload tgv48 --reps 20 [--ops r1,res,jvp32,jvp64,pc32]

Workloads: tgv48 (3-D eps-scaled Euler Taylor-Green field, eps 0.1, N = 3, 48^3 elements),
vortex128 (2-D Euler vortex, N = 5, 128^2 elements), nstgv32 (Navier-Stokes Taylor-Green,
mu = 1.25e-3, eps 0.1, N = 3, 32^3 elements).  Prints one JSON line.
"""
import argparse
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

TWO_PI = 6.283185307179586
WORKLOADS = {
    "tgv48": dict(dim=3, nelem=[48, 48, 48], length=[TWO_PI] * 3, N=3, equation="euler", eps_ref=0.1),
    "vortex128": dict(dim=2, nelem=[128, 128], length=[10.0, 10.0], N=5, equation="euler", eps_ref=1.0),
    "nstgv32": dict(dim=3, nelem=[32, 32, 32], length=[TWO_PI] * 3, N=3, equation="navier_stokes", eps_ref=0.1,
                    mu=1.25e-3),
}
HBM_PEAK_GBS = 8000.0


def state(ctx, wl):
    import numpy as np
    from paper_2109_04804_amd import inputs
    xi, _ = ctx.nodes()
    X = inputs.node_coords(wl["dim"], wl["nelem"], wl["length"], [0.0] * wl["dim"], xi)
    if wl["dim"] == 3:
        return inputs.taylor_green(X[0], X[1], X[2], gamma=1.4, eps=wl["eps_ref"])
    xc, yc, beta = inputs.vortex_params(inputs.DEFAULT_SEED, beta=5.0)
    return inputs.isentropic_vortex(X[0], X[1], xc, yc, beta, box=wl["length"][0])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="tgv48", choices=sorted(WORKLOADS))
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--ops", default="r1,res,jvp32,jvp64,pc32")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first a plain device copy of this many bytes, three times (reference dispatch for "
                         "scaling hardware byte counters)")
    a = ap.parse_args()
    import numpy as np
    import torch
    if a.copy_bytes > 0:
        src = torch.ones(a.copy_bytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    from paper_2109_04804_amd.hbpc import Context
    wl = WORKLOADS[a.workload]
    kw = dict(flux="rusanov", gamma=1.4, eps_ref=wl["eps_ref"])
    if "mu" in wl:
        kw["mu"] = wl["mu"]
    ctx = Context(wl["dim"], wl["nelem"], wl["length"], wl["N"], wl["equation"], gmres_restart=1, precond="bjext",
                  precision="mixed", **kw)
    n = ctx.ndof
    w = torch.tensor(np.ascontiguousarray(state(ctx, wl)).reshape(-1), dtype=torch.float64, device="cuda")
    s = torch.empty_like(w)
    ctx.residual1(w, s)
    rng = np.random.default_rng(7)
    dX = torch.tensor(rng.standard_normal(2 * n) * 1e-3, dtype=torch.float64, device="cuda")
    w32, s32, dX32 = w.float(), s.float(), dX.float()
    out1 = torch.empty(n, dtype=torch.float64, device="cuda")
    G = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    Y64 = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    Y32 = torch.empty(2 * n, dtype=torch.float32, device="cuda")
    a1dt, bc = 0.03, 0.03 ** 2 / 3
    ops = {
        "r1": lambda: ctx.residual1(w, out1),
        "res": lambda: ctx.newton_residual(w, s, w, a1dt, bc, G),
        "jvp32": lambda: ctx.jvp_f32(w32, s32, a1dt, bc, dX32, Y32),
        "jvp64": lambda: ctx.jvp(w, s, a1dt, bc, dX, Y64),
        "pc32": lambda: ctx.pc_apply_f32(dX32, Y32),
    }
    chosen = [o for o in a.ops.split(",") if o]
    if "pc32" in chosen:
        ctx.pc_build(w, a1dt, bc, "mixed")
    report = {"workload": a.workload, "dof": n, "reps": a.reps, "ops": {}}
    for op in chosen:
        ops[op]()   # warm-up
        torch.cuda.synchronize()
        ctx.profile_read(reset=True)
        ctx.profile_enable(True)
        for _ in range(a.reps):
            ops[op]()
        torch.cuda.synchronize()
        prof = ctx.profile_read(reset=True)
        ctx.profile_enable(False)
        rep = {}
        for k, v in prof.items():
            if v["launches"] == 0:
                continue
            ms = v["total_ms"] / v["launches"]
            gbs = v["bytes"] / v["launches"] / (ms * 1e-3) / 1e9 if ms > 0 else None
            rep[k] = {"launches": v["launches"], "avg_ms": round(ms, 5), "bytes_per_launch": v["bytes"] / v["launches"],
                      "GBps": round(gbs, 1) if gbs else None, "frac_hbm": round(gbs / HBM_PEAK_GBS, 4) if gbs else None}
        report["ops"][op] = rep
        print("[opbench] %s %s" % (op, json.dumps(rep)), file=sys.stderr, flush=True)
    ctx.close()
    print(json.dumps(report))


if __name__ == "__main__":
    main()
