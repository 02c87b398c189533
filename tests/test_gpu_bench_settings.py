"""HBPC steps in the benchmark's own composition against the oracle.

The vortex benchmark runs N = 5 (element blocks of 144 unknowns), HBPC(6,4)
(Alg. 1 with three Lobatto nodes and four corrector sweeps), dt = 0.1,
FGMRES(30) at eps_G = 1e-3, the two corrector stages of each sweep solved side
by side, and in its learned form a 5-iteration probe of the network in each
solve.  Here the same composition (the two corrector stages of a sweep solved side by side on one set of
BJ_ext blocks, or one stage at a time with blocks kept per corrector stage) steps an 8 x
8-element vortex of the same domain (element size
1.25) and is compared with one oracle step run at eps_N = 1e-12 (GMRES(30) +
BJ_ext, eps_G 1e-5), i.e. with the stage equations solved to round-off.  The
oracle steps take minutes, so they are stored (tests/golden/step_*.npz,
written by tests/golden/make_step_references.py from the oracle alone):

  fp64     eps_N = 1e-12               relative L2 <= 1e-10
  mixed    eps_N = 1e-8 (the bench's)  relative L2 <= 1e-8
  learned  eps_N = 1e-8, probe 5       relative L2 <= 1e-8

The Taylor-Green case runs the 3-D benchmark's composition (N = 3, blocks of
320, HBPC(6,4), per-stage blocks) on 3^3 elements of the 48^3 mesh's element
size h = 2 pi / 48 (the field's wavelength shrunk to three elements so that
it stays periodic) at dt = 0.06, the acoustic Courant number of about 20
that the 48^3 workload is configured for.  The determinism and split-run tests
check that a step is reproducible bitwise, and that stopping after two steps
and continuing from the saved state in a fresh context changes nothing.
"""
import os
import sys

import numpy as np
import pytest

from gpu_cases import rel
from paper_2109_04804_amd import inputs

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_step_references as golden   # noqa: E402

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

VORTEX_DT = 0.1


def dev(x, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda").reshape(-1)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def bench_context(dim, nelem, length, N, precision, precond, newton_rtol, eps_ref=1.0, probe=0, restart=30,
                  rebuild="paired", half=False):
    from paper_2109_04804_amd.hbpc import Context
    return Context(dim, nelem, length, N, "euler", flux="rusanov", gamma=1.4, eps_ref=eps_ref, q=6, kmax=4,
                   newton_rtol=newton_rtol, gmres_rtol=1e-3, gmres_restart=restart, gmres_maxit=7000,
                   precision=precision, precond=precond, pc_rebuild=rebuild, pc_fallback=0.5,
                   pc_probe_its=probe, pc_half=1 if half else 0)


_THETA = {}


def trained_params(n):
    """Network trained as the benchmark trains it (Newton pairs of FP64 BJ_ext solves at
    eps_G 1e-6 on seeded vortices of the same mesh, BF16 Adam), on a smaller sample."""
    if n in _THETA:
        return _THETA[n]
    from paper_2109_04804_amd.hbpc import Context
    col = Context(2, [n, n], [10.0, 10.0], 5, "euler", flux="rusanov", q=6, kmax=4, newton_rtol=1e-8,
                  gmres_rtol=1e-6, gmres_restart=30, precond="bjext", precision="fp64")
    n_in, H, n_out, n_p = col.mlp_shape()
    cap = 2048
    X = torch.zeros(cap * n_in, dtype=torch.float32, device="cuda")
    T = torch.zeros(cap * n_out, dtype=torch.float32, device="cuda")
    col.mlp_collect(X, T, cap, 64, 2109, source="newton")
    xi, _ = col.nodes()
    Xc = inputs.node_coords(2, [n, n], [10.0, 10.0], [0.0, 0.0], xi)
    for seed in (1, 2):
        xc, yc, beta = inputs.vortex_params(seed)
        col.step(dev(inputs.isentropic_vortex(Xc[0], Xc[1], xc, yc, beta)), VORTEX_DT)
        if col.mlp_collected() >= cap:
            break
    count = col.mlp_collected()
    col.close()
    tr = Context(2, [n, n], [10.0, 10.0], 5, "euler", flux="rusanov", precond="learned", precision="mixed")
    tr.mlp_init(7)
    log = tr.train_mlp(X, T, count, epochs=10, batch=128, lr=1e-3, seed=5, precision="bf16")
    print("trained on", count, "pairs", log, flush=True)
    theta = torch.zeros(n_p, dtype=torch.float32, device="cuda")
    tr.mlp_get_params(theta)
    tr.close()
    _THETA[n] = theta
    return theta


@pytest.mark.parametrize("rebuild", ["paired", "per_stage"])
@pytest.mark.parametrize("form", ["fp64", "mixed", "learned", "mixed16"])
def test_vortex_step_bench_composition(form, rebuild):
    """paired (the benchmark's default, HBPC_PC_PAIRED): lock-step Newton and FGMRES iterations
    of the two corrector stages of a sweep, one S^-1 set built at the first stage's state and
    applied to both stages' four right-hand sides per iteration, the next Arnoldi iteration of
    both in flight ahead of the host; in the learned form each stage solve starts on the network
    and falls back to the shared blocks on its own.  per_stage: one stage solve at a time, blocks
    kept per corrector stage over the sweeps.  mixed16: the mixed form with the S^-1 blocks
    stored in FP16 (the paired apply reads each FP16 block once for four right-hand sides)."""
    w0, ref, meta = golden.load("vortex8")
    n = meta["nelem"][0]
    precision = "fp64" if form == "fp64" else "mixed"
    rtol = 1e-12 if form == "fp64" else 1e-8
    ctx = bench_context(2, [n, n], [10.0, 10.0], 5, precision, "learned" if form == "learned" else "bjext", rtol,
                        probe=5 if form == "learned" else 0, rebuild=rebuild, half=form == "mixed16")
    if form == "learned":
        ctx.mlp_set_params(trained_params(n))
    w = dev(w0)
    st = ctx.step(w, meta["dt"])
    ctx.close()
    err = rel(host(w), ref)
    print(form, rebuild, n, "newton", st["newton_its"], "gmres", st["gmres_its"], "per solve",
          st["gmres_per_solve"], "builds", st["pc_builds"], "fallbacks", st["pc_fallbacks"], "rel err %.3e" % err,
          flush=True)
    assert st["n_solves"] == 10
    if rebuild == "paired":
        assert st["pc_builds"] <= 3   # one per predictor solve, one set for the pair (kept over sweeps)
    else:
        assert st["pc_builds"] <= 4   # one per predictor solve, one per corrector stage (kept over sweeps)
    assert err < (1e-10 if form == "fp64" else 1e-8)


@pytest.mark.parametrize("form", ["fp64", "mixed"])
def test_tgv_step_bench_composition(form):
    """FGMRES(200), as the 48^3 workload at this Courant number runs (FGMRES(30) stalls there)."""
    if not os.path.exists(golden.path_of("tgv3")):
        pytest.skip("the stored oracle step is written by tests/golden/make_step_references.py tgv3")
    w0, ref, meta = golden.load("tgv3")
    precision = "fp64" if form == "fp64" else "mixed"
    rtol = 1e-12 if form == "fp64" else 1e-8
    ctx = bench_context(3, meta["nelem"], meta["length"], 3, precision, "bjext", rtol, eps_ref=0.1,
                        restart=meta["gmres_restart"])
    w = dev(w0)
    st = ctx.step(w, meta["dt"])
    ctx.close()
    err = rel(host(w), ref)
    print(form, "newton", st["newton_its"], "gmres", st["gmres_its"], "per solve", st["gmres_per_solve"],
          "rel err %.3e" % err, flush=True)
    assert err < (1e-10 if form == "fp64" else 1e-8)


def test_step_is_deterministic():
    """Two runs of the same mixed step from the same state give bitwise equal results
    (fixed reduction order in every kernel, no atomics in the sums)."""
    w0 = golden.vortex_case()[1]
    out = []
    for _ in range(2):
        ctx = bench_context(2, [8, 8], [10.0, 10.0], 5, "mixed", "bjext", 1e-8)
        w = dev(w0)
        ctx.step(w, VORTEX_DT)
        ctx.step(w, VORTEX_DT)
        out.append(host(w))
        ctx.close()
    assert np.array_equal(out[0], out[1])


def test_split_run_equals_unbroken_run():
    """A run of four steps equals two runs of two steps, the second started from the state
    the first left (a fresh context, as after a restart from a saved state), bitwise."""
    w0 = golden.vortex_case()[1]
    ctx = bench_context(2, [8, 8], [10.0, 10.0], 5, "mixed", "bjext", 1e-8)
    w = dev(w0)
    for _ in range(4):
        ctx.step(w, VORTEX_DT)
    full = host(w)
    ctx.close()
    half = None
    w = dev(w0)
    for part in range(2):
        ctx = bench_context(2, [8, 8], [10.0, 10.0], 5, "mixed", "bjext", 1e-8)
        if part == 1:
            w = dev(half)   # through host memory, as a checkpoint would be
        for _ in range(2):
            ctx.step(w, VORTEX_DT)
        half = host(w)
        ctx.close()
    assert np.array_equal(half, full)
