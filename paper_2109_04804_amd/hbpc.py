"""Thin ctypes binding of libhbpc (include/hbpc.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  Buffers are torch tensors on the GPU (contiguous, float64 unless
the call ends in _f32); the library never allocates or frees them.  The
library is loaded from this package directory and must have been built with
`python -m paper_2109_04804_amd.build`; importing this module without it
raises, there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhbpc.so")

HBPC_OK = 0
ERRORS = {-1: "HBPC_ERR_ARG", -2: "HBPC_ERR_OOM", -3: "HBPC_ERR_HIP", -4: "HBPC_ERR_NONFINITE",
          -5: "HBPC_ERR_NEWTON", -6: "HBPC_ERR_GMRES", -7: "HBPC_ERR_UNSUPPORTED"}
EQ = {"advection": 1, "burgers": 2, "euler": 3, "navier_stokes": 4}
NODES = {"gauss": 0, "lobatto": 1}
FLUX = {"central": 0, "upwind": 1, "lf": 2, "rusanov": 3, "lf_literal": 4}
PRECISION = {"fp64": 0, "mixed": 1}
PRECOND = {"none": 0, "bjext": 1, "learned": 2, "learned_first": 3, "learned_guess": 4, "bjext_h": 5}
MLP_PRECISION = {"bf16": 0, "fp32": 1}
PAIRS = {"newton": 0, "krylov": 1, "random": 2}
PC_REBUILD = {"per_solve": 0, "per_newton_it": 1, "per_stage": 2, "across_steps": 3, "paired": 4}
JVP = {"linearised": 0, "fd": 1}
MAX_SOLVES = 64


class HbpcMesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nelem", ctypes.c_int * 3),
                ("length", ctypes.c_double * 3), ("origin", ctypes.c_double * 3)]


class HbpcParams(ctypes.Structure):
    _fields_ = [("nodes", ctypes.c_int), ("flux", ctypes.c_int), ("lambda_", ctypes.c_double),
                ("adv", ctypes.c_double * 3), ("nu", ctypes.c_double), ("gamma", ctypes.c_double),
                ("eps_ref", ctypes.c_double), ("mu", ctypes.c_double), ("prandtl", ctypes.c_double),
                ("eta_br2", ctypes.c_double), ("q", ctypes.c_int), ("kmax", ctypes.c_int),
                ("newton_rtol", ctypes.c_double), ("newton_atol_dw", ctypes.c_double),
                ("newton_maxit", ctypes.c_int), ("gmres_rtol", ctypes.c_double),
                ("gmres_restart", ctypes.c_int), ("gmres_maxit", ctypes.c_int),
                ("precision", ctypes.c_int), ("precond", ctypes.c_int), ("pc_rebuild", ctypes.c_int),
                ("jvp_mode", ctypes.c_int), ("hessian", ctypes.c_int), ("mlp_precision", ctypes.c_int),
                ("pc_fallback", ctypes.c_double), ("pc_half", ctypes.c_int),
                ("pc_reuse_steps", ctypes.c_int), ("pc_probe_its", ctypes.c_int), ("stream", ctypes.c_void_p)]


class HbpcStats(ctypes.Structure):
    _fields_ = [("n_solves", ctypes.c_int), ("newton_its", ctypes.c_int), ("gmres_its", ctypes.c_int),
                ("pc_builds", ctypes.c_int), ("newton_per_solve", ctypes.c_int * MAX_SOLVES),
                ("gmres_per_solve", ctypes.c_int * MAX_SOLVES), ("t_step_ms", ctypes.c_double),
                ("t_pc_build_ms", ctypes.c_double), ("t_gmres_ms", ctypes.c_double),
                ("t_residual_ms", ctypes.c_double), ("pc_fallbacks", ctypes.c_int), ("mlp_samples", ctypes.c_int),
                ("newton_floor_stops", ctypes.c_int)]

    def as_dict(self):
        n = min(self.n_solves, MAX_SOLVES)
        return {"n_solves": self.n_solves, "newton_its": self.newton_its, "gmres_its": self.gmres_its,
                "pc_builds": self.pc_builds, "newton_per_solve": list(self.newton_per_solve[:n]),
                "gmres_per_solve": list(self.gmres_per_solve[:n]), "t_step_ms": self.t_step_ms,
                "t_pc_build_ms": self.t_pc_build_ms, "t_gmres_ms": self.t_gmres_ms,
                "pc_fallbacks": self.pc_fallbacks, "mlp_samples": self.mlp_samples,
                "newton_floor_stops": self.newton_floor_stops}


class HbpcKernelProf(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 16), ("launches", ctypes.c_int), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("flops", ctypes.c_double)]


class HbpcTrainCfg(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("seed", ctypes.c_ulonglong), ("precision", ctypes.c_int)]


class HbpcTrainLog(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("ms", ctypes.c_double)]


# every symbol include/hbpc.h declares, with its ctypes signature
_P = ctypes.c_void_p
_D = ctypes.c_double
_I = ctypes.c_int
SIGNATURES = {
    "hbpc_default_params": (None, [ctypes.POINTER(HbpcParams)]),
    "hbpc_create": (_I, [ctypes.POINTER(HbpcMesh), _I, _I, ctypes.POINTER(HbpcParams), ctypes.POINTER(_P)]),
    "hbpc_destroy": (_I, [_P]),
    "hbpc_set_stream": (_I, [_P, _P]),
    "hbpc_ndof": (ctypes.c_size_t, [_P]),
    "hbpc_block_size": (_I, [_P]),
    "hbpc_nodes": (_I, [_P, _P, _P]),
    "hbpc_residual1": (_I, [_P, _P, _P]),
    "hbpc_residual1_noalloc": (_I, [ctypes.POINTER(HbpcMesh), _I, _I, ctypes.POINTER(HbpcParams), _P, _P]),
    "hbpc_residual2": (_I, [_P, _P, _P, _P]),
    "hbpc_newton_residual": (_I, [_P, _P, _P, _P, _D, _D, _P]),
    "hbpc_jvp": (_I, [_P, _P, _P, _D, _D, _P, _P, _I]),
    "hbpc_jvp_f32": (_I, [_P, _P, _P, _D, _D, _P, _P]),
    "hbpc_pc_build": (_I, [_P, _P, _D, _D, _I]),
    "hbpc_pc_build_hess": (_I, [_P, _P, _P, _D, _D, _I]),
    "hbpc_pc_apply": (_I, [_P, _P, _P]),
    "hbpc_pc_apply_f32": (_I, [_P, _P, _P]),
    "hbpc_step": (_I, [_P, _P, _D, ctypes.POINTER(HbpcStats)]),
    "hbpc_mlp_shape": (_I, [_P, _P, _P, _P, _P]),
    "hbpc_mlp_set_params": (_I, [_P, _P]),
    "hbpc_mlp_get_params": (_I, [_P, _P]),
    "hbpc_mlp_init": (_I, [_P, ctypes.c_ulonglong]),
    "hbpc_mlp_features": (_I, [_P, _P, _P, _P, _P, _I, _D, _D, _P, _P, _P]),
    "hbpc_mlp_forward": (_I, [_P, _P, _I, _P, _I]),
    "hbpc_mlp_loss_grad": (_I, [_P, _P, _P, _I, _P, ctypes.POINTER(_D), _I]),
    "hbpc_mlp_adam": (_I, [_P, _P, _D, _D, _D, _D]),
    "hbpc_mlp_collect": (_I, [_P, _P, _P, ctypes.c_size_t, _I, ctypes.c_ulonglong, _I, _I]),
    "hbpc_mlp_collected": (ctypes.c_size_t, [_P]),
    "hbpc_default_train_cfg": (None, [ctypes.POINTER(HbpcTrainCfg)]),
    "hbpc_train_mlp": (_I, [_P, _P, _P, ctypes.c_size_t, ctypes.POINTER(HbpcTrainCfg),
                            ctypes.POINTER(HbpcTrainLog)]),
    "hbpc_profile_enable": (_I, [_P, _I]),
    "hbpc_profile_only": (_I, [_P, ctypes.c_char_p]),
    "hbpc_profile_read": (_I, [_P, ctypes.POINTER(HbpcKernelProf), _I, _I]),
    "hbpc_strerror": (ctypes.c_char_p, [_I]),
    "hbpc_last_error": (ctypes.c_char_p, [_P]),
}

_lib = None


def load_library(path=LIB_PATH):
    """Load libhbpc.so and set the signatures; raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libhbpc.so is not built (%s); run python -m paper_2109_04804_amd.build" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class HbpcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


def default_params():
    lib = load_library()
    p = HbpcParams()
    lib.hbpc_default_params(ctypes.byref(p))
    return p


def make_params(**kw):
    """HbpcParams from the defaults plus keyword overrides (string enums accepted)."""
    p = default_params()
    maps = {"nodes": NODES, "flux": FLUX, "precision": PRECISION, "precond": PRECOND, "jvp_mode": JVP,
            "mlp_precision": MLP_PRECISION, "pc_rebuild": PC_REBUILD}
    for k, v in kw.items():
        if k in maps and isinstance(v, str):
            v = maps[k][v]
        if k == "lambda":
            k = "lambda_"
        if k == "adv":
            for i, a in enumerate(v):
                p.adv[i] = float(a)
            continue
        setattr(p, k, v)
    return p


def make_mesh(dim, nelem, length, origin=(0.0, 0.0, 0.0)):
    m = HbpcMesh()
    m.dim = dim
    for i in range(3):
        m.nelem[i] = int(nelem[i]) if i < len(nelem) else 1
        m.length[i] = float(length[i]) if i < len(length) else 1.0
        m.origin[i] = float(origin[i]) if i < len(origin) else 0.0
    return m


def _ptr(t, n, dtype):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if t.dtype != dtype:
        raise TypeError("expected %s, got %s" % (dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if t.numel() != n:
        raise ValueError("expected %d values, got %d" % (n, t.numel()))
    return ctypes.c_void_p(t.data_ptr())


def residual1_noalloc(dim, nelem, length, N, equation, w, out, origin=(0.0, 0.0, 0.0), stream=None, **params):
    """hbpc_residual1_noalloc: R1(w) -> out without a context or any device allocation
    (w, out: float64 GPU tensors of the mesh's ndof values)."""
    import torch
    lib = load_library()
    p = make_params(**params)
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    p.stream = ctypes.c_void_p(stream)
    m = make_mesh(dim, nelem, length, origin)
    eq = EQ[equation] if isinstance(equation, str) else int(equation)
    n = w.numel()
    rc = lib.hbpc_residual1_noalloc(ctypes.byref(m), int(N), eq, ctypes.byref(p), _ptr(w, n, torch.float64),
                                    _ptr(out, n, torch.float64))
    if rc != HBPC_OK:
        raise HbpcError(rc, "hbpc_residual1_noalloc failed (%s)" % lib.hbpc_strerror(rc).decode())
    return out


class Context:
    """One libhbpc context (mesh, degree, equation, parameters)."""

    def __init__(self, dim, nelem, length, N, equation, origin=(0.0, 0.0, 0.0), stream=None, **params):
        import torch
        self.lib = load_library()
        self.params = make_params(**params)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.params.stream = ctypes.c_void_p(stream)
        self.mesh = make_mesh(dim, nelem, length, origin)
        h = ctypes.c_void_p()
        eq = EQ[equation] if isinstance(equation, str) else int(equation)
        rc = self.lib.hbpc_create(ctypes.byref(self.mesh), int(N), eq, ctypes.byref(self.params), ctypes.byref(h))
        if rc != HBPC_OK:
            raise HbpcError(rc, "hbpc_create failed (%s)" % self.lib.hbpc_strerror(rc).decode())
        self.h = h
        self.ndof = int(self.lib.hbpc_ndof(h))
        self.block = int(self.lib.hbpc_block_size(h))
        self.dim = dim
        self.N = N

    def close(self):
        if getattr(self, "h", None):
            self.lib.hbpc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != HBPC_OK:
            raise HbpcError(rc, self.lib.hbpc_last_error(self.h).decode())

    def nodes(self):
        import numpy as np
        xi = (ctypes.c_double * (self.N + 1))()
        w = (ctypes.c_double * (self.N + 1))()
        self._check(self.lib.hbpc_nodes(self.h, ctypes.cast(xi, ctypes.c_void_p), ctypes.cast(w, ctypes.c_void_p)))
        return np.array(xi[:]), np.array(w[:])

    def residual1(self, w, out):
        import torch
        n = self.ndof
        self._check(self.lib.hbpc_residual1(self.h, _ptr(w, n, torch.float64), _ptr(out, n, torch.float64)))
        return out

    def residual2(self, w, sigma, out):
        import torch
        n = self.ndof
        self._check(self.lib.hbpc_residual2(self.h, _ptr(w, n, torch.float64), _ptr(sigma, n, torch.float64),
                                            _ptr(out, n, torch.float64)))
        return out

    def newton_residual(self, w, sigma, b, a1dt, bcoef, G):
        import torch
        n = self.ndof
        self._check(self.lib.hbpc_newton_residual(self.h, _ptr(w, n, torch.float64), _ptr(sigma, n, torch.float64),
                                                  _ptr(b, n, torch.float64), float(a1dt), float(bcoef),
                                                  _ptr(G, 2 * n, torch.float64)))
        return G

    def jvp(self, w, sigma, a1dt, bcoef, dX, out, mode="linearised"):
        import torch
        n = self.ndof
        self._check(self.lib.hbpc_jvp(self.h, _ptr(w, n, torch.float64), _ptr(sigma, n, torch.float64),
                                      float(a1dt), float(bcoef), _ptr(dX, 2 * n, torch.float64),
                                      _ptr(out, 2 * n, torch.float64), JVP[mode]))
        return out

    def jvp_f32(self, w, sigma, a1dt, bcoef, dX, out):
        import torch
        n = self.ndof
        self._check(self.lib.hbpc_jvp_f32(self.h, _ptr(w, n, torch.float32), _ptr(sigma, n, torch.float32),
                                          float(a1dt), float(bcoef), _ptr(dX, 2 * n, torch.float32),
                                          _ptr(out, 2 * n, torch.float32)))
        return out

    def pc_build(self, w, a1dt, bcoef, precision="fp64"):
        import torch
        self._check(self.lib.hbpc_pc_build(self.h, _ptr(w, self.ndof, torch.float64), float(a1dt), float(bcoef),
                                           PRECISION[precision]))

    def pc_build_hess(self, w, sigma, a1dt, bcoef, precision="fp64"):
        import torch
        n = self.ndof
        self._check(self.lib.hbpc_pc_build_hess(self.h, _ptr(w, n, torch.float64), _ptr(sigma, n, torch.float64),
                                                float(a1dt), float(bcoef), PRECISION[precision]))

    def pc_apply(self, X, out):
        import torch
        n2 = 2 * self.ndof
        self._check(self.lib.hbpc_pc_apply(self.h, _ptr(X, n2, torch.float64), _ptr(out, n2, torch.float64)))
        return out

    def pc_apply_f32(self, X, out):
        import torch
        n2 = 2 * self.ndof
        self._check(self.lib.hbpc_pc_apply_f32(self.h, _ptr(X, n2, torch.float32), _ptr(out, n2, torch.float32)))
        return out

    def profile_enable(self, on=True):
        self._check(self.lib.hbpc_profile_enable(self.h, 1 if on else 0))

    def profile_only(self, name):
        """Record only launches of kernel class `name` (None: all)."""
        self._check(self.lib.hbpc_profile_only(self.h, None if name is None else name.encode()))

    def profile_read(self, reset=True):
        """Per kernel class: launches, total ms, algorithmic bytes and flops."""
        arr = (HbpcKernelProf * 32)()
        k = self.lib.hbpc_profile_read(self.h, arr, 32, 1 if reset else 0)
        if k < 0:
            self._check(k)
        return {arr[i].name.decode(): {"launches": arr[i].launches, "total_ms": arr[i].total_ms,
                                       "bytes": arr[i].bytes, "flops": arr[i].flops} for i in range(k)}

    def step(self, w, dt):
        """One HBPC step in place; returns the solver statistics."""
        import torch
        st = HbpcStats()
        self._check(self.lib.hbpc_step(self.h, _ptr(w, self.ndof, torch.float64), float(dt), ctypes.byref(st)))
        return st.as_dict()

    # ---- learned preconditioner network
    def mlp_shape(self):
        """(n_in, hidden, n_out, n_params) of the per-element network."""
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        n = ctypes.c_size_t()
        self._check(self.lib.hbpc_mlp_shape(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                            ctypes.byref(n)))
        return a.value, b.value, c.value, n.value

    def mlp_set_params(self, theta):
        import torch
        self._check(self.lib.hbpc_mlp_set_params(self.h, _ptr(theta, self.mlp_shape()[3], torch.float32)))

    def mlp_init(self, seed):
        """Seeded initial parameters (library generator)."""
        self._check(self.lib.hbpc_mlp_init(self.h, int(seed)))

    def mlp_get_params(self, out):
        import torch
        self._check(self.lib.hbpc_mlp_get_params(self.h, _ptr(out, self.mlp_shape()[3], torch.float32)))
        return out

    def mlp_features(self, rt, w, a1dt, bcoef, X, scale=None, dw=None, T=None, elems=None, count=None):
        import torch
        n_in, _, n_out, _ = self.mlp_shape()
        if count is None:
            count = elems.numel() if elems is not None else self.ndof // self.block
        self._check(self.lib.hbpc_mlp_features(
            self.h, _ptr(rt, self.ndof, torch.float64), _ptr(w, self.ndof, torch.float64),
            _ptr(dw, self.ndof, torch.float64), _ptr(elems, count, torch.int32), int(count), float(a1dt),
            float(bcoef), _ptr(X, count * n_in, torch.float32), _ptr(T, count * n_out, torch.float32),
            _ptr(scale, count, torch.float32)))
        return X

    def mlp_forward(self, X, rows, Y, precision="bf16"):
        import torch
        n_in, _, n_out, _ = self.mlp_shape()
        self._check(self.lib.hbpc_mlp_forward(self.h, _ptr(X, rows * n_in, torch.float32), int(rows),
                                              _ptr(Y, rows * n_out, torch.float32), MLP_PRECISION[precision]))
        return Y

    def mlp_loss_grad(self, X, T, rows, grad, precision="bf16"):
        """Mean squared error (host float) and its gradient (into grad)."""
        import torch
        n_in, _, n_out, n_p = self.mlp_shape()
        loss = ctypes.c_double()
        self._check(self.lib.hbpc_mlp_loss_grad(self.h, _ptr(X, rows * n_in, torch.float32),
                                                _ptr(T, rows * n_out, torch.float32), int(rows),
                                                _ptr(grad, n_p, torch.float32), ctypes.byref(loss),
                                                MLP_PRECISION[precision]))
        return loss.value

    def mlp_adam(self, grad, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        import torch
        self._check(self.lib.hbpc_mlp_adam(self.h, _ptr(grad, self.mlp_shape()[3], torch.float32), float(lr),
                                           float(beta1), float(beta2), float(eps)))

    def mlp_collect(self, X, T, capacity, per_event, seed, source="newton", every=1):
        """Collect (features, target) pairs during subsequent steps into X, T (device
        float32 views of at least capacity rows); source "newton" or "krylov"."""
        import torch
        n_in, _, n_out, _ = self.mlp_shape()
        if capacity == 0:
            self._check(self.lib.hbpc_mlp_collect(self.h, None, None, 0, 1, 0, 0, 1))
            return
        xs = X.view(-1)[: capacity * n_in]
        ts = T.view(-1)[: capacity * n_out]
        self._check(self.lib.hbpc_mlp_collect(self.h, _ptr(xs, capacity * n_in, torch.float32),
                                              _ptr(ts, capacity * n_out, torch.float32), int(capacity),
                                              int(per_event), int(seed), PAIRS[source], int(every)))

    def mlp_collected(self):
        return int(self.lib.hbpc_mlp_collected(self.h))

    def train_mlp(self, X, T, count, **cfg):
        """Adam training on `count` pairs; cfg overrides the library defaults."""
        import torch
        n_in, _, n_out, _ = self.mlp_shape()
        c = HbpcTrainCfg()
        self.lib.hbpc_default_train_cfg(ctypes.byref(c))
        for k, v in cfg.items():
            if k == "precision" and isinstance(v, str):
                v = MLP_PRECISION[v]
            setattr(c, k, v)
        log = HbpcTrainLog()
        xs = X.view(-1)[: count * n_in]
        ts = T.view(-1)[: count * n_out]
        self._check(self.lib.hbpc_train_mlp(self.h, _ptr(xs, count * n_in, torch.float32),
                                            _ptr(ts, count * n_out, torch.float32), int(count),
                                            ctypes.byref(c), ctypes.byref(log)))
        return {"steps": log.steps, "loss_first": log.loss_first, "loss_last": log.loss_last, "ms": log.ms}
