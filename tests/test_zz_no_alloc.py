"""hbpc_residual1_noalloc (the entry point for callers that cannot allocate device memory)
against hbpc_residual1 of a context: the same kernels on the same data, so bitwise equal.
Two calls in a row share the one scratch array, the second on a smaller mesh; a mesh whose
traces do not fit the scratch is refused before any device work."""
import numpy as np
import pytest

from gpu_cases import CASES, lib_kwargs, oracle_for, state

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _pair(case):
    from paper_2109_04804_amd.hbpc import Context, residual1_noalloc
    kw = lib_kwargs(case)
    dg = oracle_for(case)
    w = torch.tensor(np.ascontiguousarray(state(dg, seed=3)).reshape(-1), dtype=torch.float64, device="cuda")
    ctx = Context(case["dim"], case["nelem"], case["length"], case["N"], case["equation"], **kw)
    ref = torch.empty_like(w)
    ctx.residual1(w, ref)
    torch.cuda.synchronize()
    ctx.close()
    out = torch.full_like(w, float("nan"))
    residual1_noalloc(case["dim"], case["nelem"], case["length"], case["N"], case["equation"], w, out, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ref.cpu().numpy()


@pytest.mark.parametrize("first,second", [("euler2_n5", "euler2_single"), ("burgers2", "burgers1_lobatto"),
                                          ("euler3_n3", "adv2_ragged")])
def test_noalloc_matches_context_twice(first, second):
    big = dict(CASES[first])
    if first == "euler2_n5":
        big["nelem"] = [40, 30]   # larger than the second call's mesh
    for case in (big, CASES[second]):
        got, ref = _pair(case)
        print(case["equation"], case["nelem"], "max |diff|", float(np.abs(got - ref).max()), flush=True)
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref)


def test_noalloc_refuses_meshes_beyond_the_scratch():
    from paper_2109_04804_amd.hbpc import HbpcError, residual1_noalloc
    # 48^3 elements, N = 3, 5 variables: 425 MB of traces > 64 MiB
    w = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(HbpcError) as ei:
        residual1_noalloc(3, [48, 48, 48], [6.28] * 3, 3, "euler", w, w, flux="rusanov", eps_ref=0.1)
    assert ei.value.code == -1
