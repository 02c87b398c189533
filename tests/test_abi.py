"""The C-ABI library loads and exports every function include/hbpc.h declares
(no compute call: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hbpc.h")
LIB = os.path.join(ROOT, "paper_2109_04804_amd", "libhbpc.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(hbpc_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["hbpc_create", "hbpc_destroy", "hbpc_ndof", "hbpc_residual1", "hbpc_residual2",
                     "hbpc_newton_residual", "hbpc_jvp", "hbpc_jvp_f32", "hbpc_pc_build", "hbpc_pc_apply",
                     "hbpc_step", "hbpc_strerror", "hbpc_last_error"]:
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhbpc.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhbpc.so not built")
def test_binding_covers_header():
    from paper_2109_04804_amd import hbpc
    assert set(hbpc.SIGNATURES) == set(declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhbpc.so not built")
def test_host_only_calls():
    """Calls that touch no device memory: defaults, error strings, argument checks."""
    from paper_2109_04804_amd import hbpc
    lib = hbpc.load_library()
    p = hbpc.default_params()
    assert p.q == 6 and p.kmax == 4 and p.gmres_restart == 30 and abs(p.newton_rtol - 1e-8) < 1e-20
    assert p.pc_reuse_steps == 4 and p.pc_rebuild == 0 and p.pc_probe_its == 0
    assert lib.hbpc_strerror(-5) == b"Newton did not converge"
    h = ctypes.c_void_p()
    assert lib.hbpc_create(None, 3, 3, ctypes.byref(p), ctypes.byref(h)) == -1
    assert lib.hbpc_destroy(None) == -1
    assert lib.hbpc_ndof(None) == 0
    # degrees outside the instantiated range are rejected before any device work
    for dim, N in ((2, 8), (1, 1), (3, 6)):
        m = hbpc.make_mesh(dim, [2] * dim, [1.0] * dim)
        pa = hbpc.make_params(flux="upwind", adv=[1.0, 0.5, 0.25])
        assert lib.hbpc_create(ctypes.byref(m), N, 1, ctypes.byref(pa), ctypes.byref(h)) == -7, (dim, N)
    m = hbpc.make_mesh(2, [2, 2], [1.0, 1.0])
    for bad in (dict(gmres_restart=1025), dict(pc_rebuild="paired", precond="none"),
                dict(pc_rebuild="paired", jvp_mode="fd"), dict(pc_rebuild="paired", precond="bjext_h"),
                dict(pc_rebuild="paired", precond="learned_first")):
        pa = hbpc.make_params(flux="upwind", adv=[1.0, 0.5], **bad)
        assert lib.hbpc_create(ctypes.byref(m), 3, 1, ctypes.byref(pa), ctypes.byref(h)) == -1, bad
    pa = hbpc.make_params(flux="upwind", adv=[1.0, 0.5], gmres_restart=1025)
    assert lib.hbpc_create(ctypes.byref(m), 3, 1, ctypes.byref(pa), ctypes.byref(h)) == -1


def test_struct_layouts_match_header():
    """ctypes mirrors of the header structs: field order and names."""
    src = open(HEADER).read()
    body = src[src.index("typedef struct {\n    int nodes;"):]
    body = body[:body.index("} hbpc_params;")]
    fields = re.findall(r"^\s+[a-z_ *]+?\b([a-z_0-9]+)(?:\[\d+\])?;", body, flags=re.M)
    from paper_2109_04804_amd.hbpc import HbpcParams
    got = [f[0].rstrip("_") for f in HbpcParams._fields_]
    assert got == fields
