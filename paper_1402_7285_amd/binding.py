"""ctypes binding of libscocg.so (argument marshalling only).

Every computation runs in the HIP library; this module converts NumPy
arrays to pointers, wraps the opaque handles, and uses torch for device
buffers and streams.  Loading fails loudly if the library is not built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libscocg.so")

# return codes (include/scocg.h)
OK, W_PARTIAL, W_S_DIAG = 0, 1, 2
E_ARG, E_SHAPE, E_NOT_SYMMETRIC, E_DEVICE, E_NOMEM, E_UNSUPPORTED = -1, -2, -3, -4, -5, -6
CONVERGED, MAXITER, BREAKDOWN, NONFINITE, ABORTED = 0, 1, 2, 3, 4
FP64, FP32, FP32_BF16 = 0, 1, 2
OUT_SELECTED_G, OUT_FULL_X = 0, 1
METHOD_COCG, METHOD_QMR, METHOD_COCG_LANCZOS = 0, 1, 2
NSTAT = 8
STAT_NAMES = ("outer", "sum_upd", "inner", "switches", "M", "blocks", "replacements", "fallback")

EXPORTS = (
    "scocg_last_error", "scocg_version", "scocg_matrix_from_bsr", "scocg_matrix_from_csr",
    "scocg_matrix_free", "scocg_problem_create", "scocg_problem_free", "scocg_options_default",
    "scocg_plan_create", "scocg_plan_free", "scocg_plan_out_count", "scocg_plan_out_offsets", "scocg_plan_info",
    "scocg_plan_run", "scocg_plan_stats", "scocg_solve", "scocg_plan_capture", "scocg_plan_replay",
    "scocg_autotune", "scocg_features", "scocg_mlp_nparams", "scocg_mlp_work_floats", "scocg_mlp_forward",
    "scocg_mlp_train_step", "scocg_plan_integrate", "scocg_matrix_from_mtx", "scocg_matrix_shape",
    "scocg_matrix_export_bsr", "scocg_solve_device", "scocg_sync", "scocg_mlp_cfg_default",
    "scocg_mlp_model_floats", "scocg_mlp_train", "scocg_mlp_predict", "scocg_plan_cohp", "scocg_autotune_team",
    "scocg_solve_device_noalloc", "scocg_plan_set_order", "scocg_schedule",
)


class ScocgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"scocg error {code}: {msg}")
        self.code = code


class scocg_z(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class scocg_options(C.Structure):
    _fields_ = [("tol", C.c_double), ("maxiter", C.c_int32), ("precision", C.c_int32),
                ("replace_every", C.c_int32), ("inner_maxiter", C.c_int32), ("inner_tol", C.c_double),
                ("inner_tol_lo", C.c_double), ("seed_index", C.c_int32), ("threads", C.c_int32),
                ("slots", C.c_int32), ("audit", C.c_int32), ("projected", C.c_int32), ("method", C.c_int32),
                ("team_size", C.c_int32), ("panel_width", C.c_int32), ("team_registers", C.c_int32)]


class scocg_rhs_spec(C.Structure):
    _fields_ = [("cluster_ptr", C.c_void_p), ("cluster_atoms", C.c_void_p), ("out_mode", C.c_int32),
                ("out_ptr", C.c_void_p), ("out_rows", C.c_void_p), ("order", C.c_void_p)]


_VP = C.c_void_p
_LIB = None


class scocg_mlp_cfg(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("val_frac", C.c_float),
                ("seed", C.c_uint64), ("init_weights", C.c_void_p)]


def _declare(lib):
    i32, i64, st = C.c_int32, C.c_int64, C.c_int32
    sig = {
        "scocg_last_error": (C.c_char_p, []),
        "scocg_version": (C.c_char_p, []),
        "scocg_matrix_from_bsr": (st, [i64, i32, _VP, _VP, _VP, C.POINTER(_VP)]),
        "scocg_matrix_from_csr": (st, [i64, _VP, _VP, _VP, i32, C.POINTER(_VP)]),
        "scocg_matrix_free": (None, [_VP]),
        "scocg_matrix_from_mtx": (st, [C.c_char_p, i32, C.POINTER(_VP)]),
        "scocg_matrix_shape": (st, [_VP, C.POINTER(i64), C.POINTER(i32), C.POINTER(i64)]),
        "scocg_matrix_export_bsr": (st, [_VP, _VP, _VP, _VP]),
        "scocg_problem_create": (st, [_VP, _VP, C.POINTER(_VP)]),
        "scocg_problem_free": (None, [_VP]),
        "scocg_options_default": (None, [C.POINTER(scocg_options)]),
        "scocg_plan_create": (st, [_VP, C.POINTER(scocg_options), i32, _VP, i32, _VP,
                                   C.POINTER(scocg_rhs_spec), C.POINTER(_VP)]),
        "scocg_plan_free": (None, [_VP]),
        "scocg_plan_out_count": (i64, [_VP]),
        "scocg_plan_out_offsets": (st, [_VP, _VP]),
        "scocg_plan_info": (st, [_VP, _VP]),
        "scocg_plan_run": (st, [_VP, _VP, _VP, _VP, _VP, _VP]),
        "scocg_plan_stats": (st, [_VP, _VP]),
        "scocg_plan_capture": (st, [_VP, _VP, _VP, _VP, _VP, _VP]),
        "scocg_plan_replay": (st, [_VP, _VP]),
        "scocg_features": (st, [_VP, _VP, _VP]),
        "scocg_plan_integrate": (st, [_VP, _VP, _VP, _VP, C.c_double, C.c_double, _VP, _VP]),
        "scocg_plan_cohp": (st, [_VP, _VP, _VP, _VP]),
        "scocg_mlp_nparams": (i64, []),
        "scocg_mlp_work_floats": (i64, []),
        "scocg_mlp_forward": (st, [_VP, _VP, i64, _VP, _VP]),
        "scocg_mlp_train_step": (st, [_VP, _VP, _VP, _VP, _VP, _VP, i64, C.c_float, i32, _VP, _VP, _VP, _VP]),
        "scocg_autotune": (st, [_VP, C.POINTER(scocg_options), i32, _VP, i32, _VP, C.POINTER(scocg_rhs_spec),
                                i32, C.POINTER(i32), C.POINTER(i32), C.POINTER(C.c_double)]),
        "scocg_autotune_team": (st, [_VP, C.POINTER(scocg_options), i32, _VP, i32, _VP, C.POINTER(scocg_rhs_spec),
                                     i32, C.POINTER(scocg_options), C.POINTER(C.c_double)]),
        "scocg_solve": (st, [_VP, C.POINTER(scocg_options), i32, _VP, i32, _VP,
                             C.POINTER(scocg_rhs_spec), _VP, _VP, _VP, _VP]),
        "scocg_solve_device": (st, [_VP, C.POINTER(scocg_options), i32, _VP, i32, _VP,
                                    C.POINTER(scocg_rhs_spec), _VP, _VP, _VP, _VP, _VP]),
        "scocg_solve_device_noalloc": (st, [_VP, C.POINTER(scocg_options), i32, _VP, i32, _VP,
                                            C.POINTER(scocg_rhs_spec), _VP, _VP, _VP, _VP, _VP]),
        "scocg_sync": (st, [_VP]),
        "scocg_mlp_cfg_default": (None, [C.POINTER(scocg_mlp_cfg)]),
        "scocg_mlp_model_floats": (i64, []),
        "scocg_mlp_train": (st, [_VP, _VP, i64, C.POINTER(scocg_mlp_cfg), _VP, C.POINTER(C.c_double)]),
        "scocg_mlp_predict": (st, [_VP, _VP, i64, _VP]),
        "scocg_plan_set_order": (st, [_VP, _VP]),
        "scocg_schedule": (st, [_VP, _VP, _VP, _VP]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def load(path: str = LIB_PATH):
    """Load libscocg.so; raises if it is missing (no fallback exists)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built: run `python -m paper_1402_7285_amd.build`")
        _LIB = _declare(C.CDLL(path))
    return _LIB


def _check(code):
    if code < 0:
        raise ScocgError(code, load().scocg_last_error().decode())
    return code


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _tptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


# ---------------------------------------------------------------------------
# thin wrappers with the C names
# ---------------------------------------------------------------------------

def scocg_matrix_from_bsr(nbrows, bdim, rowptr, colidx, vals):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    colidx = np.ascontiguousarray(colidx, dtype=np.int32)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    h = _VP()
    _check(load().scocg_matrix_from_bsr(int(nbrows), int(bdim), _ptr(rowptr), _ptr(colidx), _ptr(vals), C.byref(h)))
    return h


def scocg_matrix_from_csr(n, rowptr, colidx, vals, bdim):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    colidx = np.ascontiguousarray(colidx, dtype=np.int32)
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    h = _VP()
    _check(load().scocg_matrix_from_csr(int(n), _ptr(rowptr), _ptr(colidx), _ptr(vals), int(bdim), C.byref(h)))
    return h


def scocg_matrix_free(h):
    load().scocg_matrix_free(h)


def scocg_problem_create(H, S=None):
    h = _VP()
    code = _check(load().scocg_problem_create(H, S, C.byref(h)))
    return h, code


def scocg_problem_free(h):
    load().scocg_problem_free(h)


def scocg_options_default(**overrides) -> scocg_options:
    o = scocg_options()
    load().scocg_options_default(C.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


@dataclass
class _Spec:
    struct: scocg_rhs_spec
    keep: tuple


def make_spec(cluster_ptr=None, cluster_atoms=None, out_ptr=None, out_rows=None, full_x=False, order=None):
    arrs = (
        None if cluster_ptr is None else np.ascontiguousarray(cluster_ptr, dtype=np.int64),
        None if cluster_atoms is None else np.ascontiguousarray(cluster_atoms, dtype=np.int32),
        None if out_ptr is None else np.ascontiguousarray(out_ptr, dtype=np.int64),
        None if out_rows is None else np.ascontiguousarray(out_rows, dtype=np.int32),
        None if order is None else np.ascontiguousarray(order, dtype=np.int32),
    )
    s = scocg_rhs_spec(_ptr(arrs[0]), _ptr(arrs[1]), OUT_FULL_X if full_x else OUT_SELECTED_G,
                       _ptr(arrs[2]), _ptr(arrs[3]), _ptr(arrs[4]))
    return _Spec(s, arrs)


def _shifts(z):
    z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128))
    return z, z.ctypes.data_as(C.c_void_p)


def scocg_plan_create(problem, opt: scocg_options, shifts, rhs_index, spec: _Spec):
    z, zp = _shifts(shifts)
    rhs = np.ascontiguousarray(rhs_index, dtype=np.int32)
    h = _VP()
    _check(load().scocg_plan_create(problem, C.byref(opt), int(z.size), zp, int(rhs.size), _ptr(rhs),
                                    C.byref(spec.struct), C.byref(h)))
    return h


def scocg_plan_free(h):
    load().scocg_plan_free(h)


def scocg_plan_out_count(h) -> int:
    return int(load().scocg_plan_out_count(h))


def scocg_plan_out_offsets(h, nrhs) -> np.ndarray:
    off = np.zeros(nrhs + 1, dtype=np.int64)
    _check(load().scocg_plan_out_offsets(h, _ptr(off)))
    return off


NINFO = 10
INFO_NAMES = ("slots", "threads", "Mp", "slot_bytes", "seed0", "lds_bytes", "precision", "global", "team_size",
              "panel_width")


def scocg_plan_info(h) -> dict:
    info = np.zeros(NINFO, dtype=np.int64)
    _check(load().scocg_plan_info(h, _ptr(info)))
    return dict(zip(INFO_NAMES, (int(v) for v in info)))


def scocg_plan_run(h, stream, out, iters=None, status=None, resid=None):
    """Device buffers are torch CUDA tensors; stream a torch.cuda.Stream or None."""
    sp = None if stream is None else C.c_void_p(stream.cuda_stream)
    return _check(load().scocg_plan_run(h, sp, _tptr(out), _tptr(iters), _tptr(status), _tptr(resid)))


def scocg_plan_capture(h, stream, out, iters=None, status=None, resid=None):
    return _check(load().scocg_plan_capture(h, C.c_void_p(stream.cuda_stream), _tptr(out), _tptr(iters),
                                            _tptr(status), _tptr(resid)))


def scocg_plan_replay(h, stream):
    return _check(load().scocg_plan_replay(h, C.c_void_p(stream.cuda_stream)))


def scocg_autotune(problem, opt, shifts, rhs_index, spec: "_Spec", probe_iters):
    z, zp = _shifts(shifts)
    rhs = np.ascontiguousarray(rhs_index, dtype=np.int32)
    t, sl, sec = C.c_int32(0), C.c_int32(0), C.c_double(0.0)
    _check(load().scocg_autotune(problem, C.byref(opt), int(z.size), zp, int(rhs.size), _ptr(rhs),
                                 C.byref(spec.struct), int(probe_iters), C.byref(t), C.byref(sl), C.byref(sec)))
    return int(t.value), int(sl.value), float(sec.value)


def scocg_autotune_team(problem, opt, shifts, rhs_index, spec: "_Spec", probe_iters):
    """Team-solver launch search; returns (best options struct, probe seconds)."""
    z, zp = _shifts(shifts)
    rhs = np.ascontiguousarray(rhs_index, dtype=np.int32)
    best = scocg_options()
    sec = C.c_double(0.0)
    _check(load().scocg_autotune_team(problem, C.byref(opt), int(z.size), zp, int(rhs.size), _ptr(rhs),
                                      C.byref(spec.struct), int(probe_iters), C.byref(best), C.byref(sec)))
    return best, float(sec.value)


def _sp(stream):
    return None if stream is None else C.c_void_p(stream.cuda_stream)


def scocg_plan_integrate(h, G, weights, mu, kT, rho, ldos=None, stream=None):
    return _check(load().scocg_plan_integrate(h, _sp(stream), _tptr(G), _tptr(weights), float(mu), float(kT),
                                              _tptr(rho), _tptr(ldos)))


def scocg_plan_cohp(h, rho, cohp, stream=None):
    return _check(load().scocg_plan_cohp(h, _sp(stream), _tptr(rho), _tptr(cohp)))


def scocg_features(h, feats, stream=None):
    return _check(load().scocg_features(h, _tptr(feats), _sp(stream)))


def scocg_mlp_nparams() -> int:
    return int(load().scocg_mlp_nparams())


def scocg_mlp_work_floats() -> int:
    return int(load().scocg_mlp_work_floats())


def scocg_mlp_forward(w, x, y, stream=None):
    return _check(load().scocg_mlp_forward(_tptr(w), _tptr(x), int(x.shape[0]), _tptr(y), _sp(stream)))


def scocg_mlp_train_step(w, m, v, x, t, idx, lr, step, loss, grad, work, stream=None):
    n = int(idx.shape[0]) if idx is not None else int(x.shape[0])
    return _check(load().scocg_mlp_train_step(_tptr(w), _tptr(m), _tptr(v), _tptr(x), _tptr(t), _tptr(idx), n,
                                              float(lr), int(step), _tptr(loss), _tptr(grad), _tptr(work),
                                              _sp(stream)))


def scocg_plan_stats(h, nrhs) -> np.ndarray:
    st = np.zeros((nrhs, NSTAT), dtype=np.int64)
    _check(load().scocg_plan_stats(h, _ptr(st)))
    return st


def scocg_solve(problem, opt, shifts, rhs_index, spec: _Spec, nout_total):
    """Host-buffer convenience call; returns (out, iters, status, resid, code)."""
    z, zp = _shifts(shifts)
    rhs = np.ascontiguousarray(rhs_index, dtype=np.int32)
    K, R = z.size, rhs.size
    out = np.zeros(max(1, nout_total), dtype=np.complex128)
    iters = np.zeros(R * K, dtype=np.int32)
    status = np.zeros(R * K, dtype=np.int8)
    resid = np.zeros(R * K, dtype=np.float64)
    code = _check(load().scocg_solve(problem, C.byref(opt), int(K), zp, int(R), _ptr(rhs), C.byref(spec.struct),
                                     _ptr(out), _ptr(iters), _ptr(status), _ptr(resid)))
    return out[:nout_total], iters.reshape(R, K), status.reshape(R, K), resid.reshape(R, K), code


def scocg_solve_device(problem, opt, shifts, rhs_index, spec: _Spec, out, iters=None, status=None, resid=None,
                       stream=None):
    """Enqueue a solve into caller-owned torch CUDA tensors on ``stream``
    (a torch.cuda.Stream or None); finish it with ``scocg_sync(problem)``."""
    z, zp = _shifts(shifts)
    rhs = np.ascontiguousarray(rhs_index, dtype=np.int32)
    return _check(load().scocg_solve_device(problem, C.byref(opt), int(z.size), zp, int(rhs.size), _ptr(rhs),
                                            C.byref(spec.struct), _tptr(out), _tptr(iters), _tptr(status),
                                            _tptr(resid), _sp(stream)))


def scocg_solve_device_noalloc(problem, opt, shifts, rhs_index, spec: _Spec, out, iters=None, status=None,
                               resid=None, stream=None):
    """The allocation-free device-buffer solve (one-workgroup Lanczos-basis
    solver on the library's fixed per-device array); enqueued on ``stream``."""
    z, zp = _shifts(shifts)
    rhs = np.ascontiguousarray(rhs_index, dtype=np.int32)
    return _check(load().scocg_solve_device_noalloc(problem, C.byref(opt), int(z.size), zp, int(rhs.size),
                                                    _ptr(rhs), C.byref(spec.struct), _tptr(out), _tptr(iters),
                                                    _tptr(status), _tptr(resid), _sp(stream)))


def scocg_sync(problem):
    """Wait for the problem's pending device-buffer solves; returns OK or W_PARTIAL."""
    return _check(load().scocg_sync(problem))


def scocg_mlp_cfg_default(**overrides) -> scocg_mlp_cfg:
    cfg = scocg_mlp_cfg()
    load().scocg_mlp_cfg_default(C.byref(cfg))
    for k, v in overrides.items():
        setattr(cfg, k, v)
    return cfg


def scocg_mlp_model_floats() -> int:
    return int(load().scocg_mlp_model_floats())


def scocg_mlp_train(feats, log_iters, init_weights=None, **cfg_overrides):
    """Whole training run on host arrays; returns (model float32
    [scocg_mlp_model_floats()], best validation loss)."""
    F = np.ascontiguousarray(feats, dtype=np.float32)
    t = np.ascontiguousarray(log_iters, dtype=np.float32)
    if F.ndim != 2 or F.shape[1] != 16 or t.shape != (F.shape[0],):
        raise ValueError("feats must be [n, 16] and log_iters [n]")
    w0 = None if init_weights is None else np.ascontiguousarray(init_weights, dtype=np.float32)
    cfg = scocg_mlp_cfg_default(**cfg_overrides)
    cfg.init_weights = None if w0 is None else w0.ctypes.data
    model = np.zeros(scocg_mlp_model_floats(), dtype=np.float32)
    vl = C.c_double(0.0)
    _check(load().scocg_mlp_train(_ptr(F), _ptr(t), int(F.shape[0]), C.byref(cfg), _ptr(model), C.byref(vl)))
    return model, float(vl.value)


def scocg_mlp_predict(model, feats):
    """Predictions of a scocg_mlp_train model for host features [n, 16]."""
    m = np.ascontiguousarray(model, dtype=np.float32)
    F = np.ascontiguousarray(feats, dtype=np.float32)
    if m.size != scocg_mlp_model_floats() or F.ndim != 2 or F.shape[1] != 16:
        raise ValueError("model size or feature shape")
    y = np.zeros(F.shape[0], dtype=np.float32)
    _check(load().scocg_mlp_predict(_ptr(m), _ptr(F), int(F.shape[0]), _ptr(y)))
    return y


# ---------------------------------------------------------------------------
# object wrappers
# ---------------------------------------------------------------------------

class Matrix:
    def __init__(self, nbrows, bdim, rowptr, colidx, vals):
        self.h = scocg_matrix_from_bsr(nbrows, bdim, rowptr, colidx, vals)

    @classmethod
    def from_bsr(cls, A):
        """From any object with nbrows, bdim, rowptr, colidx, vals attributes."""
        if isinstance(A, Matrix):
            return A
        return cls(A.nbrows, A.bdim, A.rowptr, A.colidx, A.vals)

    @classmethod
    def from_mtx(cls, path, bdim=1):
        """Read a Matrix Market file (real coordinate, symmetric or general)."""
        m = cls.__new__(cls)
        h = _VP()
        _check(load().scocg_matrix_from_mtx(os.fsencode(path), int(bdim), C.byref(h)))
        m.h = h
        return m

    def shape(self):
        """(block rows, block dimension, stored blocks)."""
        nb, bd, nblk = C.c_int64(), C.c_int32(), C.c_int64()
        _check(load().scocg_matrix_shape(self.h, C.byref(nb), C.byref(bd), C.byref(nblk)))
        return nb.value, bd.value, nblk.value

    def export(self):
        """The stored BSR arrays as an object with nbrows, bdim, rowptr, colidx, vals."""
        nb, bd, nblk = self.shape()
        rp = np.empty(nb + 1, dtype=np.int64)
        ci = np.empty(max(1, nblk), dtype=np.int32)
        vv = np.empty((max(1, nblk), bd, bd), dtype=np.float64)
        _check(load().scocg_matrix_export_bsr(self.h, rp.ctypes.data, ci.ctypes.data, vv.ctypes.data))

        class _B:
            pass
        out = _B()
        out.nbrows, out.bdim, out.rowptr, out.colidx, out.vals = nb, bd, rp, ci[:nblk], vv[:nblk]
        out.n = nb * bd
        return out

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None:
            scocg_matrix_free(self.h)
            self.h = None


class Problem:
    """H and S resident on the current device (S None means S = I)."""

    def __init__(self, H, S=None):
        self.Hm = Matrix.from_bsr(H)
        self.Sm = Matrix.from_bsr(S) if S is not None else None
        self.h, self.code = scocg_problem_create(self.Hm.h, self.Sm.h if self.Sm else None)

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None:
            scocg_problem_free(self.h)
            self.h = None


class Plan:
    """Everything a solve reads, resident on the device; ``run`` enqueues the solve."""

    def __init__(self, problem: Problem, shifts, rhs, cluster_ptr=None, cluster_atoms=None,
                 out_ptr=None, out_rows=None, full_x=False, order=None, **options):
        self.problem = problem
        self.shifts = np.asarray(shifts, dtype=np.complex128)
        self.rhs = np.asarray(rhs, dtype=np.int32)
        self.K, self.nrhs = self.shifts.size, self.rhs.size
        self.opt = scocg_options_default(**options)
        self.spec = make_spec(cluster_ptr, cluster_atoms, out_ptr, out_rows, full_x, order)
        self.h = scocg_plan_create(problem.h, self.opt, self.shifts, self.rhs, self.spec)
        self.out_count = scocg_plan_out_count(self.h)
        self.out_offsets = scocg_plan_out_offsets(self.h, self.nrhs)
        self.info = scocg_plan_info(self.h)
        self.slots = self.info["slots"]

    def alloc_outputs(self, device="cuda"):
        import torch
        R, K = self.nrhs, self.K
        return dict(
            out=torch.empty(max(1, self.out_count), dtype=torch.complex128, device=device),
            iters=torch.empty((R, K), dtype=torch.int32, device=device),
            status=torch.empty((R, K), dtype=torch.int8, device=device),
            resid=torch.empty((R, K), dtype=torch.float64, device=device),
        )

    def run(self, bufs, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        return scocg_plan_run(self.h, stream, bufs["out"], bufs["iters"], bufs["status"], bufs["resid"])

    def stats(self) -> np.ndarray:
        return scocg_plan_stats(self.h, self.nrhs)

    def integrate(self, bufs, weights, mu, kT, stream=None):
        """Density-matrix rows and local DOS from the G of the last run in
        ``bufs``: returns (rho [rows] float64, ldos [nrhs, K] float64),
        torch CUDA tensors.  ``weights``: K quadrature weights (array-like)."""
        import torch
        w = torch.as_tensor(np.asarray(weights, dtype=np.float64)).to("cuda")
        rows = int(self.out_offsets[-1])                  # output rows (out_count is rows x K)
        rho = torch.empty(max(1, rows), dtype=torch.float64, device="cuda")
        ldos = torch.empty((max(1, self.nrhs), self.K), dtype=torch.float64, device="cuda")
        if stream is None:
            stream = torch.cuda.current_stream()
        scocg_plan_integrate(self.h, bufs["out"], w, mu, kT, rho, ldos, stream)
        return rho[:rows], ldos[: self.nrhs]

    def cohp(self, rho, stream=None):
        """Integrated COHP H_{row(o), j} rho[o] of every output row, from the
        ``rho`` that ``integrate`` returned (torch CUDA tensor [rows])."""
        import torch
        rows = int(self.out_offsets[-1])
        out = torch.empty(max(1, rows), dtype=torch.float64, device="cuda")
        if stream is None:
            stream = torch.cuda.current_stream()
        scocg_plan_cohp(self.h, rho, out, stream)
        return out[:rows]

    def set_order(self, order=None):
        """Replace the work-queue order (host permutation of 0..nrhs-1; None = index order)."""
        o = None if order is None else np.ascontiguousarray(order, dtype=np.int32)
        if o is not None and o.shape != (self.nrhs,):
            raise ValueError("order must have nrhs entries")
        _check(load().scocg_plan_set_order(self.h, None if o is None else _ptr(o)))

    def schedule(self, model=None):
        """Learned binning: order the queue by decreasing predicted cost (model from
        scocg_mlp_train; None = by local-pattern size).  Returns (order, cost)."""
        m = None
        if model is not None:
            m = np.ascontiguousarray(model, dtype=np.float32)
            if m.size != scocg_mlp_model_floats():
                raise ValueError("model size")
        order = np.zeros(max(1, self.nrhs), dtype=np.int32)
        cost = np.zeros(max(1, self.nrhs), dtype=np.float32)
        _check(load().scocg_schedule(self.h, None if m is None else _ptr(m), _ptr(order), _ptr(cost)))
        return order[: self.nrhs], cost[: self.nrhs]

    def features(self):
        """[nrhs, 16] FP32 features computed on the device (torch tensor)."""
        import torch
        f = torch.empty((max(1, self.nrhs), 16), dtype=torch.float32, device="cuda")
        scocg_features(self.h, f, torch.cuda.current_stream())
        return f[: self.nrhs]

    def capture(self, bufs, stream):
        """Record the run into a HIP graph bound to ``bufs`` on ``stream`` (non-default)."""
        return scocg_plan_capture(self.h, stream, bufs["out"], bufs["iters"], bufs["status"], bufs["resid"])

    def replay(self, stream):
        return scocg_plan_replay(self.h, stream)

    def solve(self):
        """Run once and return host results: dict(G=list of [K, nout] arrays, iters, status, resid)."""
        import torch
        bufs = self.alloc_outputs()
        self.run(bufs)
        torch.cuda.synchronize()
        out = bufs["out"].cpu().numpy()
        G = []
        for r in range(self.nrhs):
            a, b = self.out_offsets[r] * self.K, self.out_offsets[r + 1] * self.K
            G.append(out[a:b].reshape(self.K, -1))
        return dict(G=G, iters=bufs["iters"].cpu().numpy(), status=bufs["status"].cpu().numpy(),
                    resid=bufs["resid"].cpu().numpy(), stats=self.stats())

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None:
            scocg_plan_free(self.h)
            self.h = None


def autotune(problem: Problem, shifts, rhs, probe_iters=200, cache_path=None, key_extra="", **plan_kwargs):
    """Pick the launch shape for this problem by timing short probe solves on
    the device: (threads, slots) of the one-workgroup solvers, or, for the
    Lanczos-basis methods, (threads, slots, team_size, panel_width) of the
    team solver (which includes the one-workgroup shape as team_size -1).
    Results are cached in a JSON file keyed by the GPU architecture and the
    problem shape."""
    import json
    import torch
    opts = {k: v for k, v in plan_kwargs.items() if hasattr(scocg_options, k)}
    spec_kw = {k: v for k, v in plan_kwargs.items() if not hasattr(scocg_options, k)}
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName
    shifts = np.asarray(shifts, dtype=np.complex128)
    rhs = np.asarray(rhs, dtype=np.int32)
    key = f"{arch}|K{shifts.size}|R{rhs.size}|{sorted(opts.items())}|{key_extra}"
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            return cache[key]
    opt = scocg_options_default(**opts)
    spec = make_spec(**spec_kw)
    if opt.method in (METHOD_QMR, METHOD_COCG_LANCZOS) and opt.team_size != -1:
        best, sec = scocg_autotune_team(problem.h, opt, shifts, rhs, spec, probe_iters)
        res = {"threads": int(best.threads), "slots": int(best.slots), "team_size": int(best.team_size),
               "panel_width": int(best.panel_width), "probe_seconds": sec, "probe_iters": probe_iters}
    else:
        t, sl, sec = scocg_autotune(problem.h, opt, shifts, rhs, spec, probe_iters)
        res = {"threads": t, "slots": sl, "probe_seconds": sec, "probe_iters": probe_iters}
    if cache_path:
        cache[key] = res
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return res
