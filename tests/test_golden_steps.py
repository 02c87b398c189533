"""The stored oracle steps (tests/golden/step_*.npz) belong to the inputs the
generators produce today: the stored initial state is the generator's, the
settings are the ones the GPU tests run, and the oracle's step conserves the
integrals of the conserved variables (mass, momentum, energy: a property of
the DGSEM on a periodic mesh that the stored result must keep)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
import make_step_references as golden   # noqa: E402


@pytest.mark.parametrize("name", sorted(golden.CASES))
def test_stored_step_matches_its_inputs(name):
    if not os.path.exists(golden.path_of(name)):
        pytest.skip("not generated")
    w0, w1, meta = golden.load(name)
    dg, w0_now, meta_now = golden.CASES[name]()
    assert np.array_equal(w0, w0_now)
    for k, v in meta_now.items():
        assert meta[k] == v, k
    assert np.all(np.isfinite(w1)) and w1.shape == w0.shape
    m0, m1 = dg.integral(w0), dg.integral(w1)
    assert np.allclose(m1, m0, rtol=0, atol=1e-9 * np.abs(m0).max()), (m0, m1)
    # the step moved the state (dt is not negligible)
    assert np.linalg.norm(w1 - w0) > 1e-4 * np.linalg.norm(w0)
