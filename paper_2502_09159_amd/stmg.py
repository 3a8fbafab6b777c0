"""ctypes binding of the C ABI in include/stmg.h (argument marshalling only).

Vectors are torch tensors on the GPU (float64, contiguous, the layout of
Eq. (DefX)); their device pointers are handed to the library.  Every call
raises StmgError on a non-zero status.  There is no fallback: if libstmg.so is
missing or fails to load, importing this module raises.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstmg.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} not built; run python -m paper_2502_09159_amd.build")
lib = ctypes.CDLL(LIB_PATH)

STATUS = {0: "STMG_OK", -1: "STMG_EINVAL", -2: "STMG_ENOMEM", -3: "STMG_EDEVICE", -4: "STMG_ENOCONV",
          -5: "STMG_ESINGULAR", -6: "STMG_EUNSUPPORTED"}
FP64, MIXED_FP32 = 0, 1
OPT_APPLY_SUBINTERVALS, OPT_NET_CHUNK, OPT_APPLY_LOOP_ORDER, OPT_INJECT_NONFINITE = 1, 2, 3, 4  # stmg_option
VANKA_FACTORED, VANKA_DENSE, VANKA_DECOUPLED, VANKA_AUTO = 0, 1, 2, 3
LOCAL_EXACT, LOCAL_DIAGONAL = 0, 1

NU_FN = ctypes.CFUNCTYPE(None, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                         ctypes.c_void_p)


class Params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n_cells_1d", ctypes.c_int), ("n_coarse_1d", ctypes.c_int),
                ("deform_amp", ctypes.c_double), ("r", ctypes.c_int), ("k", ctypes.c_int),
                ("n_sub", ctypes.c_int), ("tau", ctypes.c_double), ("nu", ctypes.c_double),
                ("nu_fn", NU_FN), ("nu_user", ctypes.c_void_p), ("r_min", ctypes.c_int),
                ("k_min", ctypes.c_int), ("time_h_coarsening", ctypes.c_int), ("placement", ctypes.c_int),
                ("nu_pre", ctypes.c_int),
                ("nu_post", ctypes.c_int), ("omega", ctypes.c_double), ("precision", ctypes.c_int),
                ("vanka_mode", ctypes.c_int), ("local_solver", ctypes.c_int), ("device", ctypes.c_int),
                ("stream", ctypes.c_void_p)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("rel_residual", ctypes.c_double), ("t_solve_s", ctypes.c_double),
                ("t_smoother_s", ctypes.c_double), ("t_mg_other_s", ctypes.c_double),
                ("t_operator_s", ctypes.c_double), ("t_other_s", ctypes.c_double),
                ("learned_disabled", ctypes.c_int), ("history_len", ctypes.c_int),
                ("history", ctypes.POINTER(ctypes.c_double)), ("vcycle_fallbacks", ctypes.c_int),
                ("learned_steps", ctypes.c_int)]


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_sig = {
    "stmg_default_params": [ctypes.POINTER(Params)],
    "stmg_hierarchy": [ctypes.POINTER(Params), ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
    "stmg_setup": [ctypes.POINTER(Params), ctypes.POINTER(_P)],
    "stmg_destroy": [_P],
    "stmg_set_phase_timing": [_P, ctypes.c_int],
    "stmg_sizes": [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                   ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int)],
    "stmg_apply_operator": [_P, ctypes.c_int, _P, _P],
    "stmg_apply_operator_vcycle_precision": [_P, ctypes.c_int, _P, _P],
    "stmg_set_option": [_P, ctypes.c_int, ctypes.c_int64],
    "stmg_residual": [_P, ctypes.c_int, _P, _P, _P],
    "stmg_smooth": [_P, ctypes.c_int, _P, _P, ctypes.c_int],
    "stmg_vanka_correction": [_P, ctypes.c_int, _P, _P],
    "stmg_vanka_correction_noalloc": [_P, ctypes.c_int, _P, _P],
    "stmg_kernel_time": [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)],
    "stmg_restrict": [_P, ctypes.c_int, _P, _P],
    "stmg_prolongate": [_P, ctypes.c_int, _P, _P],
    "stmg_coarse_solve": [_P, _P, _P],
    "stmg_vcycle": [_P, _P, _P],
    "stmg_solve": [_P, _P, _P, ctypes.c_double, ctypes.c_int, ctypes.POINTER(SolveInfo)],
    "stmg_project_pressure_mean_zero": [_P, _P],
    "stmg_time_nodes": [_P, _D],
    "stmg_slab_rhs": [_P, _P, _P, _P, _P],
    "stmg_slab_end_value": [_P, _P, _P],
    "stmg_solve_slab": [_P, _P, _P, _P, _P, ctypes.c_double, ctypes.c_int, ctypes.POINTER(SolveInfo)],
    "stmg_march": [_P, ctypes.c_int, _P, _P, _P, _P, ctypes.c_double, ctypes.c_int,
                   ctypes.POINTER(ctypes.c_int)],
    "stmg_learned_load": [_P, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t],
    "stmg_learned_weights": [_P, ctypes.POINTER(ctypes.c_float), ctypes.c_size_t],
    "stmg_learned_enable": [_P, ctypes.c_int],
    "stmg_learned_record": [_P, _P, _P, _P, _P],
    "stmg_learned_train_pairs": [_P, _P, _P, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_float, ctypes.POINTER(ctypes.c_float)],
    "stmg_learned_train": [_P, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_float,
                           ctypes.POINTER(ctypes.c_float)],
    "stmg_learned_correction": [_P, ctypes.c_int, _P, _P],
    "stmg_learned_gradient": [_P, ctypes.c_int, _P, _P, ctypes.POINTER(ctypes.c_float),
                              ctypes.POINTER(ctypes.c_double)],
}
NET_PARAMS = 52704
RESTART = 64  # STMG_RESTART: FGMRES restart length of stmg_solve
for _name, _args in _sig.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
lib.stmg_last_error.argtypes = [_P]
lib.stmg_last_error.restype = ctypes.c_char_p

EXPORTED = list(_sig) + ["stmg_last_error"]


class StmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def _check(code, ctx=None):
    if code != 0:
        msg = lib.stmg_last_error(ctx).decode() if ctx else ""
        raise StmgError(code, msg)


def default_params(**kw):
    p = Params()
    _check(lib.stmg_default_params(ctypes.byref(p)))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def hierarchy(**kw):
    p = default_params(**kw)
    buf = (ctypes.c_int * 256)()
    n = ctypes.c_int()
    _check(lib.stmg_hierarchy(ctypes.byref(p), 64, buf, ctypes.byref(n)))
    return [tuple(buf[4 * i:4 * i + 4]) for i in range(n.value)]


def _ptr(t, n=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} entries, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """Owns one library context (stmg_setup .. stmg_destroy)."""

    def __init__(self, nu_fn=None, **kw):
        self._keep = None
        if nu_fn is not None:
            import numpy as np

            def cb(npts, xyz, out, user):
                d = kw.get("dim", 3)
                pts = np.ctypeslib.as_array(xyz, shape=(npts * d,)).reshape(npts, d)
                vals = np.ctypeslib.as_array(out, shape=(npts,))
                vals[:] = nu_fn(pts)

            self._keep = NU_FN(cb)
            kw["nu_fn"] = self._keep
        if "stream" not in kw:
            kw["stream"] = torch.cuda.current_stream().cuda_stream
        self.params = default_params(**kw)
        ctx = ctypes.c_void_p()
        code = lib.stmg_setup(ctypes.byref(self.params), ctypes.byref(ctx))
        if code != 0:
            raise StmgError(code, "setup failed")
        self.ctx = ctx
        self.n_levels = self.sizes(0)[3]

    def close(self):
        if getattr(self, "ctx", None):
            lib.stmg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sizes(self, level=0):
        nd, nv, npr, nl = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int()
        _check(lib.stmg_sizes(self.ctx, level, ctypes.byref(nd), ctypes.byref(nv), ctypes.byref(npr),
                              ctypes.byref(nl)), self.ctx)
        return nd.value, nv.value, npr.value, nl.value

    def ndofs(self, level=0):
        return self.sizes(level)[0]

    def vector(self, level=0):
        return torch.zeros(self.ndofs(level), dtype=torch.float64, device="cuda")

    def set_phase_timing(self, on=True):
        _check(lib.stmg_set_phase_timing(self.ctx, int(on)), self.ctx)

    def apply(self, x, y, level=0):
        n = self.ndofs(level)
        _check(lib.stmg_apply_operator(self.ctx, level, _ptr(x, n), _ptr(y, n)), self.ctx)

    def apply_vcycle_precision(self, x, y, level=0):
        """y = S x with the operator of the V-cycle (FP32 in a mixed context)."""
        n = self.ndofs(level)
        _check(lib.stmg_apply_operator_vcycle_precision(self.ctx, level, _ptr(x, n), _ptr(y, n)), self.ctx)

    def set_option(self, option, value):
        _check(lib.stmg_set_option(self.ctx, int(option), int(value)), self.ctx)

    def residual(self, b, x, r, level=0):
        n = self.ndofs(level)
        _check(lib.stmg_residual(self.ctx, level, _ptr(b, n), _ptr(x, n), _ptr(r, n)), self.ctx)

    def smooth(self, b, x, steps=1, level=0):
        n = self.ndofs(level)
        _check(lib.stmg_smooth(self.ctx, level, _ptr(b, n), _ptr(x, n), steps), self.ctx)

    def vanka_correction(self, r, x, level=0):
        n = self.ndofs(level)
        _check(lib.stmg_vanka_correction(self.ctx, level, _ptr(r, n), _ptr(x, n)), self.ctx)

    def vanka_correction_noalloc(self, r, x, level=0):
        """stmg_vanka_correction with the library's fixed scratch buffer (no allocation)."""
        n = self.ndofs(level)
        _check(lib.stmg_vanka_correction_noalloc(self.ctx, level, _ptr(r, n), _ptr(x, n)), self.ctx)

    def kernel_time(self, which, level=0, reps=10):
        """Mean device time (ms) of one application of kernel class `which` on
        `level`: 0 Vanka correction, 1 operator residual, 2 the Vanka local
        solves alone, 3 the operator's cell kernel alone."""
        ms = ctypes.c_double()
        _check(lib.stmg_kernel_time(self.ctx, which, level, reps, ctypes.byref(ms)), self.ctx)
        return ms.value

    def restrict(self, fine, coarse, level=0):
        _check(lib.stmg_restrict(self.ctx, level, _ptr(fine, self.ndofs(level)),
                                 _ptr(coarse, self.ndofs(level + 1))), self.ctx)

    def prolongate(self, coarse, fine, level=0):
        _check(lib.stmg_prolongate(self.ctx, level, _ptr(coarse, self.ndofs(level + 1)),
                                   _ptr(fine, self.ndofs(level))), self.ctx)

    def coarse_solve(self, b, x):
        n = self.ndofs(self.n_levels - 1)
        _check(lib.stmg_coarse_solve(self.ctx, _ptr(b, n), _ptr(x, n)), self.ctx)

    def vcycle(self, b, x):
        n = self.ndofs(0)
        _check(lib.stmg_vcycle(self.ctx, _ptr(b, n), _ptr(x, n)), self.ctx)

    def project_pressure(self, x):
        _check(lib.stmg_project_pressure_mean_zero(self.ctx, _ptr(x, self.ndofs(0))), self.ctx)

    # ------------------------------------------------------- time marching
    def time_nodes(self):
        import numpy as np
        t = np.zeros(self.params.k + 1)
        _check(lib.stmg_time_nodes(self.ctx, t.ctypes.data_as(_D)), self.ctx)
        return t

    @staticmethod
    def _optr(t, n):
        return ctypes.c_void_p(None) if t is None else _ptr(t, n)

    def slab_rhs(self, b, f=None, v0=None, g=None):
        n = self.ndofs(0)
        nv = self.sizes(0)[1]
        _check(lib.stmg_slab_rhs(self.ctx, self._optr(f, n), self._optr(v0, nv), self._optr(g, n), _ptr(b, n)),
               self.ctx)

    def slab_end_value(self, x):
        n, nv = self.ndofs(0), self.sizes(0)[1]
        v = torch.empty(nv, dtype=torch.float64, device="cuda")
        _check(lib.stmg_slab_end_value(self.ctx, _ptr(x, n), _ptr(v, nv)), self.ctx)
        return v

    def solve_slab(self, x, f=None, v0=None, g=None, rtol=1e-8, max_it=100):
        n, nv = self.ndofs(0), self.sizes(0)[1]
        info = SolveInfo()
        _check(lib.stmg_solve_slab(self.ctx, self._optr(f, n), self._optr(v0, nv), self._optr(g, n), _ptr(x, n),
                                   rtol, max_it, ctypes.byref(info)), self.ctx)
        return dict(iterations=info.iterations, rel_residual=info.rel_residual, t_solve_s=info.t_solve_s)

    def march(self, n_slabs, x, f=None, g=None, v0=None, rtol=1e-8, max_it=100):
        """x, f, g: (n_slabs * n_dofs) device arrays; returns the iterations per slab."""
        import numpy as np
        n, nv = self.ndofs(0), self.sizes(0)[1]
        its = np.zeros(n_slabs, dtype=np.int32)
        _check(lib.stmg_march(self.ctx, n_slabs, self._optr(f, n * n_slabs), self._optr(g, n * n_slabs),
                              self._optr(v0, nv), _ptr(x, n * n_slabs), rtol, max_it,
                              its.ctypes.data_as(ctypes.POINTER(ctypes.c_int))), self.ctx)
        return its

    # ---------------------------------------------------------- learned
    def learned_load(self, weights):
        import numpy as np
        w = np.ascontiguousarray(weights, dtype=np.float32).ravel()
        if w.size != NET_PARAMS:
            raise ValueError(f"expected {NET_PARAMS} weights")
        _check(lib.stmg_learned_load(self.ctx, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), w.size), self.ctx)

    def learned_weights(self):
        import numpy as np
        w = np.zeros(NET_PARAMS, dtype=np.float32)
        _check(lib.stmg_learned_weights(self.ctx, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), w.size),
               self.ctx)
        return w

    def learned_enable(self, on=True, element_levels_only=False):
        """on: the correction on every level it reaches (directly or through
        the next level); element_levels_only: only on levels with the
        network's element."""
        code = 0 if not on else (2 if element_levels_only else 1)
        _check(lib.stmg_learned_enable(self.ctx, code), self.ctx)

    def learned_record(self, b, xstar):
        n = self.ndofs(0)
        r = torch.empty(2 * n, dtype=torch.float64, device="cuda")
        e = torch.empty(2 * n, dtype=torch.float64, device="cuda")
        _check(lib.stmg_learned_record(self.ctx, _ptr(b, n), _ptr(xstar, n), ctypes.c_void_p(r.data_ptr()),
                                       ctypes.c_void_p(e.data_ptr())), self.ctx)
        return r.view(2, n), e.view(2, n)

    def learned_train(self, r_pairs, e_pairs, seed=0, epochs=1, batch=4096, lr=1e-3):
        import numpy as np
        for t in (r_pairs, e_pairs):
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or t.dim() != 2:
                raise TypeError("pairs must be contiguous float32 CUDA tensors of shape (n_pairs, n_dofs)")
        n_pairs = r_pairs.shape[0]
        d, n, r, k, N = (self.params.dim, self.params.n_cells_1d, self.params.r, self.params.k, self.params.n_sub)
        cells = N * n ** d
        steps = epochs * n_pairs * ((cells + batch - 1) // batch)
        hist = np.zeros(steps, dtype=np.float32)
        _check(lib.stmg_learned_train_pairs(self.ctx, ctypes.c_void_p(r_pairs.data_ptr()),
                                            ctypes.c_void_p(e_pairs.data_ptr()), n_pairs, seed, epochs, batch, lr,
                                            hist.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), self.ctx)
        return hist

    def learned_train_seeded(self, n_pairs, seed=0, epochs=20, lr=1e-3):
        """stmg_learned_train: pairs from random forcings generated and
        solved inside the library, then Adam; returns the trained weights."""
        import numpy as np
        w = np.zeros(NET_PARAMS, dtype=np.float32)
        _check(lib.stmg_learned_train(self.ctx, n_pairs, seed, epochs, lr,
                                      w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), self.ctx)
        return w

    def learned_correction(self, r, level=0):
        n = self.ndofs(level)
        u = torch.empty(n, dtype=torch.float64, device="cuda")
        _check(lib.stmg_learned_correction(self.ctx, level, _ptr(r, n), _ptr(u, n)), self.ctx)
        return u

    def learned_gradient(self, r, e, level=0):
        import numpy as np
        n = self.ndofs(level)
        g = np.zeros(NET_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        _check(lib.stmg_learned_gradient(self.ctx, level, _ptr(r, n), _ptr(e, n),
                                         g.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(loss)),
               self.ctx)
        return g, loss.value

    def solve(self, b, x, rtol=1e-8, max_it=100, raise_on_noconv=True):
        n = self.ndofs(0)
        info = SolveInfo()
        code = lib.stmg_solve(self.ctx, _ptr(b, n), _ptr(x, n), rtol, max_it, ctypes.byref(info))
        if code != 0 and (raise_on_noconv or code != -4):
            _check(code, self.ctx)
        hist = [info.history[i] for i in range(info.history_len)]
        return dict(iterations=info.iterations, rel_residual=info.rel_residual, t_solve_s=info.t_solve_s,
                    t_smoother_s=info.t_smoother_s, t_mg_other_s=info.t_mg_other_s,
                    t_operator_s=info.t_operator_s, t_other_s=info.t_other_s,
                    learned_disabled=info.learned_disabled, vcycle_fallbacks=info.vcycle_fallbacks,
                    learned_steps=info.learned_steps,
                    history=hist, status=code)
