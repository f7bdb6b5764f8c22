"""MI355X engine for exact KDE bandwidth-selection pair sums.

A thin ctypes binding over the C ABI declared in include/kde_bw.h (built as
libkde_bw.so next to this file).  Every function named ``kde_*`` here has the
same name, arguments and meaning as the C entry point; this module only
marshals arguments.  All arithmetic of the selectors runs in the library's
HIP kernels: there is no Python or CPU fallback, and importing the package
fails if the library has not been built.

Method: Andrzejewski, Gramacki, Gramacki, arXiv 1505.01998, Section 4.4
(normal-reference rule, direct plug-in, LSCV_h objective over a grid).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkde_bw.so")

KDE_OK, KDE_E_INVAL, KDE_E_DEGENERATE, KDE_E_NOMEM, KDE_E_DEVICE, KDE_E_BUSY, KDE_E_CANCELLED = range(7)
KDE_F32, KDE_F64 = 0, 1
KDE_PREC_MIXED, KDE_PREC_FP64 = 0, 1
KDE_MAX_N = 1 << 30
KDE_MAX_NH = 65536
KDE_MAX_BATCH = 65535
KDE_MAX_D = 16
KDE_MAX_H_EVAL = 65536
KDE_NOALLOC_SCRATCH_BYTES = 32 << 20
KDE_GRID_EXPLICIT, KDE_GRID_PAPER, KDE_GRID_LOG_ROT = 0, 1, 2
KDE_METHOD_ROT, KDE_METHOD_PLUGIN, KDE_METHOD_LSCV = 1, 2, 4

STATUS_NAMES = {
    KDE_OK: "KDE_OK",
    KDE_E_INVAL: "KDE_E_INVAL",
    KDE_E_DEGENERATE: "KDE_E_DEGENERATE",
    KDE_E_NOMEM: "KDE_E_NOMEM",
    KDE_E_DEVICE: "KDE_E_DEVICE",
    KDE_E_BUSY: "KDE_E_BUSY",
    KDE_E_CANCELLED: "KDE_E_CANCELLED",
}

# Every symbol the header declares; tests check that the library exports them.
EXPORTS = (
    "kde_ctx_create", "kde_ctx_destroy", "kde_last_error", "kde_ctx_set_stream", "kde_ctx_set_precision",
    "kde_ctx_set_option", "kde_ctx_set_timing", "kde_ctx_kernel_time", "kde_bw_rot", "kde_bw_plugin",
    "kde_lscv_curve", "kde_lscv_sums", "kde_lscv_item_sums", "kde_bw_lscv", "kde_batch",
    "kde_server_start", "kde_submit", "kde_poll", "kde_wait", "kde_server_stop", "kde_autotune",
    "kde_ctx_graph_stats", "kde_request_footprint", "kde_plan_items", "kde_bw_lscv_min", "kde_density",
    "kde_range_aggregates", "kde_lscv_md_curve", "kde_bw_lscv_md", "kde_lscv_H_eval", "kde_bw_lscv_H",
    "kde_density_H", "kde_range_aggregates_2d", "kde_cancel", "kde_job_create", "kde_job_run",
    "kde_job_progress", "kde_job_result", "kde_job_checkpoint_bytes", "kde_job_checkpoint", "kde_job_resume",
    "kde_job_destroy", "kde_lscv_ceiling", "kde_lscv_H_prepare", "kde_lscv_H_eval_prepared", "kde_lscv_H_release",
    "kde_issue_rates", "kde_lscv_curve_noalloc",
)


class KdeError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class kde_column(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("n", ctypes.c_int64), ("dtype", ctypes.c_int),
                ("on_device", ctypes.c_int)]


class kde_plugin_info(ctypes.Structure):
    _fields_ = [
        ("sigma", ctypes.c_double),
        ("h_rot", ctypes.c_double),
        ("stages", ctypes.c_int),
        ("g", ctypes.c_double * 3),
        ("psi", ctypes.c_double * 3),
        ("kappa", ctypes.c_double * 3),
        ("precision_used", ctypes.c_int * 3),
        ("h", ctypes.c_double),
    ]


class kde_tune_info(ctypes.Structure):
    _fields_ = [("hc", ctypes.c_int32), ("tj", ctypes.c_int32), ("evals_per_s", ctypes.c_double * 5),
                ("parity", ctypes.c_int32 * 5), ("pad0", ctypes.c_int32)]


# variants of the persistent LSCV sweep, in the order of kde_tune_info's arrays
TUNE_VARIANTS = ((8, 512), (16, 256), (16, 512), (16, 1024), (32, 512))


class kde_issue_info(ctypes.Structure):
    _fields_ = [("clock_hz", ctypes.c_double), ("cus", ctypes.c_int32), ("pad0", ctypes.c_int32),
                ("add_f32", ctypes.c_double), ("mul_f32", ctypes.c_double), ("fma_f32", ctypes.c_double),
                ("exp_f32", ctypes.c_double), ("lscv_mix", ctypes.c_double), ("lscv_mix_zero", ctypes.c_double)]


class kde_lscv_min_info(ctypes.Structure):
    _fields_ = [("g", ctypes.c_double), ("iterations", ctypes.c_int32), ("pad0", ctypes.c_int32),
                ("evaluated", ctypes.c_int64), ("bracket_lo", ctypes.c_double), ("bracket_hi", ctypes.c_double)]


class kde_matrix(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int32), ("dtype", ctypes.c_int),
                ("on_device", ctypes.c_int)]


class kde_lscv_H_info(ctypes.Structure):
    _fields_ = [("g", ctypes.c_double), ("evals", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("pad0", ctypes.c_int32)]


class kde_grid(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("h", ctypes.POINTER(ctypes.c_double)), ("n_h", ctypes.c_int32),
                ("lo", ctypes.c_double), ("hi", ctypes.c_double)]


class kde_request(ctypes.Structure):
    _fields_ = [("x", kde_column), ("methods", ctypes.c_uint), ("stages", ctypes.c_int), ("grid", kde_grid)]


class kde_result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("sigma", ctypes.c_double),
        ("h_rot", ctypes.c_double),
        ("h_plugin", ctypes.c_double),
        ("h_lscv", ctypes.c_double),
        ("k_lscv", ctypes.c_int32),
        ("at_edge", ctypes.c_int),
        ("plugin", kde_plugin_info),
        ("g_out", ctypes.POINTER(ctypes.c_double)),
        ("gscale_out", ctypes.POINTER(ctypes.c_double)),
        ("t_queue_s", ctypes.c_double),
        ("t_service_s", ctypes.c_double),
        ("lscv_evals_dense", ctypes.c_double),
        ("lscv_evals", ctypes.c_double),
    ]


def _load():
    # PyTorch ships its own HIP runtime under the same soname as the system
    # one.  Loading torch first makes the dynamic loader bind this library to
    # that already-loaded runtime, so a process that also uses torch for
    # device buffers and streams holds exactly one HIP runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python paper_1505_01998_amd/build.py (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    PD = ctypes.POINTER(ctypes.c_double)
    I = ctypes.c_int
    I32 = ctypes.c_int32
    I64 = ctypes.c_int64
    lib.kde_ctx_create.argtypes = [I, I, ctypes.POINTER(P)]
    lib.kde_ctx_destroy.argtypes = [P]
    lib.kde_ctx_destroy.restype = None
    lib.kde_last_error.argtypes = [P]
    lib.kde_last_error.restype = ctypes.c_char_p
    lib.kde_ctx_set_stream.argtypes = [P, P]
    lib.kde_ctx_set_precision.argtypes = [P, I]
    lib.kde_ctx_set_option.argtypes = [P, ctypes.c_char_p, I64]
    lib.kde_ctx_set_timing.argtypes = [P, I]
    lib.kde_ctx_kernel_time.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(I64), PD, PD]
    lib.kde_bw_rot.argtypes = [P, kde_column, PD]
    lib.kde_bw_plugin.argtypes = [P, kde_column, I, PD, ctypes.POINTER(kde_plugin_info)]
    lib.kde_lscv_curve.argtypes = [P, kde_column, PD, I32, PD, PD, PD]
    lib.kde_lscv_curve_noalloc.argtypes = [P, kde_column, PD, I32, PD, PD]
    lib.kde_lscv_sums.argtypes = [P, kde_column, PD, I32, PD, PD]
    lib.kde_lscv_item_sums.argtypes = [P, kde_column, PD, I32, ctypes.POINTER(I32), I32, ctypes.POINTER(I32),
                                       ctypes.POINTER(I32), PD]
    lib.kde_bw_lscv.argtypes = [P, kde_column, PD, I32, PD, ctypes.POINTER(I32), ctypes.POINTER(I)]
    lib.kde_batch.argtypes = [P, ctypes.POINTER(kde_request), I32, ctypes.POINTER(kde_result)]
    lib.kde_server_start.argtypes = [P, ctypes.c_uint64, I32]
    lib.kde_submit.argtypes = [P, ctypes.POINTER(kde_request), ctypes.POINTER(ctypes.c_uint64)]
    lib.kde_poll.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(kde_result)]
    lib.kde_wait.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(kde_result), ctypes.c_double]
    lib.kde_server_stop.argtypes = [P]
    lib.kde_cancel.argtypes = [P, ctypes.c_uint64]
    lib.kde_job_create.argtypes = [P, ctypes.POINTER(kde_request), ctypes.POINTER(P)]
    lib.kde_job_run.argtypes = [P, ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
    lib.kde_job_progress.argtypes = [P, PD, PD, ctypes.POINTER(ctypes.c_int)]
    lib.kde_job_result.argtypes = [P, ctypes.POINTER(kde_result)]
    lib.kde_job_checkpoint_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_uint64)]
    lib.kde_job_checkpoint.argtypes = [P, ctypes.c_void_p, ctypes.c_uint64]
    lib.kde_job_resume.argtypes = [P, ctypes.c_void_p, ctypes.c_uint64]
    lib.kde_job_destroy.argtypes = [P]
    lib.kde_job_destroy.restype = None
    lib.kde_autotune.argtypes = [P, I64, I32, ctypes.POINTER(kde_tune_info)]
    lib.kde_lscv_ceiling.argtypes = [P, I32, PD]
    lib.kde_issue_rates.argtypes = [P, ctypes.POINTER(kde_issue_info)]
    lib.kde_density.argtypes = [P, kde_column, ctypes.c_double, PD, I32, PD]
    lib.kde_lscv_md_curve.argtypes = [P, kde_matrix, PD, I32, PD, PD, PD]
    lib.kde_bw_lscv_md.argtypes = [P, kde_matrix, PD, I32, PD, ctypes.POINTER(I32)]
    lib.kde_lscv_H_eval.argtypes = [P, kde_matrix, PD, I32, PD, PD]
    lib.kde_lscv_H_prepare.argtypes = [P, kde_matrix, ctypes.POINTER(ctypes.c_void_p)]
    lib.kde_lscv_H_eval_prepared.argtypes = [ctypes.c_void_p, PD, I32, PD, PD]
    lib.kde_lscv_H_release.argtypes = [ctypes.c_void_p]
    lib.kde_density_H.argtypes = [P, kde_matrix, PD, PD, I32, PD]
    lib.kde_range_aggregates_2d.argtypes = [P, kde_matrix, PD, PD, I32, PD, PD, PD, PD, PD]
    lib.kde_bw_lscv_H.argtypes = [P, kde_matrix, ctypes.c_double, ctypes.c_double, I32, PD,
                                  ctypes.POINTER(kde_lscv_H_info)]
    lib.kde_range_aggregates.argtypes = [P, kde_column, ctypes.c_double, PD, PD, I32, PD, PD, PD]
    lib.kde_bw_lscv_min.argtypes = [P, kde_column, ctypes.c_double, ctypes.c_double, ctypes.c_double, I32, PD,
                                    ctypes.POINTER(kde_lscv_min_info)]
    lib.kde_ctx_graph_stats.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64)]
    lib.kde_request_footprint.argtypes = [P, ctypes.POINTER(kde_request), ctypes.POINTER(ctypes.c_uint64)]
    lib.kde_plan_items.argtypes = [I64, I32, I64, I32, ctypes.POINTER(I32), ctypes.POINTER(I32),
                                   ctypes.POINTER(I32), ctypes.POINTER(I32), PD]
    for name in EXPORTS:
        if name not in ("kde_ctx_destroy", "kde_last_error", "kde_job_destroy", "kde_lscv_H_release"):
            getattr(lib, name).restype = ctypes.c_int
    lib.kde_lscv_H_release.restype = None
    return lib


lib = _load()


# ---------------------------------------------------------------- argument marshalling
def _pd(a):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_column(x):
    """Return (kde_column, keepalive) for a numpy array (host) or a torch CUDA tensor (device)."""
    if hasattr(x, "data_ptr") and hasattr(x, "is_cuda"):
        if x.dim() != 1 or not x.is_contiguous():
            raise ValueError("device column must be a contiguous 1-D tensor")
        import torch

        if x.dtype == torch.float32:
            dt = KDE_F32
        elif x.dtype == torch.float64:
            dt = KDE_F64
        else:
            raise ValueError("device column must be float32 or float64")
        return kde_column(x.data_ptr(), x.numel(), dt, 1 if x.is_cuda else 0), x
    a = np.asarray(x)
    if a.dtype not in (np.float32, np.float64):
        a = a.astype(np.float64)
    a = np.ascontiguousarray(a)
    if a.ndim != 1:
        raise ValueError("sample column must be one-dimensional")
    return kde_column(a.ctypes.data, a.size, KDE_F32 if a.dtype == np.float32 else KDE_F64, 0), a


def _grid(h_grid):
    if h_grid is None:
        return None
    return np.ascontiguousarray(np.asarray(h_grid, dtype=np.float64).ravel())


# ---------------------------------------------------------------- C-ABI functions, same names
def kde_ctx_create(device: int = 0, prec: int = KDE_PREC_MIXED) -> ctypes.c_void_p:
    out = ctypes.c_void_p()
    st = lib.kde_ctx_create(int(device), int(prec), ctypes.byref(out))
    if st != KDE_OK:
        raise KdeError(st, "kde_ctx_create failed")
    return out


def kde_ctx_destroy(ctx) -> None:
    lib.kde_ctx_destroy(ctx)


def kde_last_error(ctx) -> str:
    return lib.kde_last_error(ctx).decode()


def _check(ctx, st):
    if st != KDE_OK:
        raise KdeError(st, kde_last_error(ctx))


def kde_ctx_set_stream(ctx, hip_stream) -> None:
    _check(ctx, lib.kde_ctx_set_stream(ctx, hip_stream))


def kde_ctx_set_precision(ctx, prec: int) -> None:
    _check(ctx, lib.kde_ctx_set_precision(ctx, int(prec)))


def kde_ctx_set_option(ctx, key: str, value: int) -> None:
    _check(ctx, lib.kde_ctx_set_option(ctx, key.encode(), int(value)))


def kde_ctx_set_timing(ctx, enable: bool) -> None:
    _check(ctx, lib.kde_ctx_set_timing(ctx, 1 if enable else 0))


def kde_ctx_kernel_time(ctx, family: str):
    """(launches, total_ms, evals) of a pair-kernel family since timing was enabled."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    ev = ctypes.c_double()
    _check(ctx, lib.kde_ctx_kernel_time(ctx, family.encode(), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(ev)))
    return n.value, ms.value, ev.value


def kde_plan_items(n: int, n_h: int = 128, seg: int = -1):
    """Work items of the i < j triangle of n samples for the LSCV pass over n_h
    bandwidths (n_h = 0: a plug-in stage): arrays (row_begin, j_begin, j_end,
    pairs), longest first."""
    m = ctypes.c_int32()
    st = lib.kde_plan_items(int(n), int(n_h), int(seg), 0, ctypes.byref(m), None, None, None, None)
    if st != KDE_OK:
        raise KdeError(st, "kde_plan_items: invalid arguments")
    k = m.value
    i0, jb, je = (np.empty(k, np.int32) for _ in range(3))
    pr = np.empty(k, np.float64)
    P32 = ctypes.POINTER(ctypes.c_int32)
    st = lib.kde_plan_items(int(n), int(n_h), int(seg), k, ctypes.byref(m), i0.ctypes.data_as(P32),
                            jb.ctypes.data_as(P32), je.ctypes.data_as(P32), _pd(pr))
    if st != KDE_OK:
        raise KdeError(st, "kde_plan_items failed")
    return i0, jb, je, pr


def kde_request_footprint(req, ctx=None) -> int:
    """Device bytes a Request needs (its column block), under ctx's options or the defaults."""
    r, keep, _ = _make_request(req)
    b = ctypes.c_uint64()
    st = lib.kde_request_footprint(ctx, ctypes.byref(r), ctypes.byref(b))
    del keep
    if st != KDE_OK:
        raise KdeError(st, "kde_request_footprint: invalid request" if st == KDE_E_INVAL else "busy")
    return b.value


def make_matrix(x):
    """(kde_matrix, keepalive) for an n x d numpy array or CUDA tensor (row-major)."""
    if hasattr(x, "is_cuda") and x.is_cuda:
        t = x.contiguous()
        if t.dim() != 2:
            raise ValueError("a sample matrix is n x d")
        dt = {"torch.float32": KDE_F32, "torch.float64": KDE_F64}[str(t.dtype)]
        return kde_matrix(t.data_ptr(), t.shape[0], t.shape[1], dt, 1), t
    a = np.asarray(x)
    if a.dtype not in (np.float32, np.float64):
        a = a.astype(np.float64)
    a = np.ascontiguousarray(a)
    if a.ndim != 2:
        raise ValueError("a sample matrix is n x d")
    return kde_matrix(a.ctypes.data, a.shape[0], a.shape[1], KDE_F64 if a.dtype == np.float64 else KDE_F32, 0), a


def kde_lscv_md_curve(ctx, x, h_grid=None, n_h: int = 0):
    """(g, gscale, grid) of the d-dimensional LSCV_h objective."""
    m, keep = make_matrix(x)
    gr = None if h_grid is None else _grid(h_grid)
    k = gr.size if gr is not None else (n_h if n_h > 0 else 150)
    g, gs, grid = (np.empty(k, np.float64) for _ in range(3))
    _check(ctx, lib.kde_lscv_md_curve(ctx, m, _pd(gr), int(k), _pd(g), _pd(gs), _pd(grid)))
    del keep
    return g, gs, grid


def kde_bw_lscv_md(ctx, x, h_grid=None, n_h: int = 0):
    """(h, k) -- the grid point minimising the d-dimensional g(h)."""
    m, keep = make_matrix(x)
    gr = None if h_grid is None else _grid(h_grid)
    k = gr.size if gr is not None else int(n_h)
    h = ctypes.c_double()
    kk = ctypes.c_int32()
    _check(ctx, lib.kde_bw_lscv_md(ctx, m, _pd(gr), int(k), ctypes.byref(h), ctypes.byref(kk)))
    del keep
    return h.value, kk.value


def kde_lscv_H_eval(ctx, x, H):
    """(g, gscale) of LSCV_H at bandwidth matrices H (m x d x d, or one d x d)."""
    m, keep = make_matrix(x)
    d = m.d
    Hs = np.ascontiguousarray(np.asarray(H, np.float64))
    if Hs.ndim == 2:
        Hs = Hs[None]
    if Hs.ndim != 3 or Hs.shape[1:] != (d, d):
        raise ValueError("H must be m x d x d for d-dimensional samples")
    k = Hs.shape[0]
    g, gs = np.empty(k, np.float64), np.empty(k, np.float64)
    _check(ctx, lib.kde_lscv_H_eval(ctx, m, _pd(Hs.ravel()), int(k), _pd(g), _pd(gs)))
    del keep
    return g, gs


def _H_stack(H, d):
    Hs = np.ascontiguousarray(np.asarray(H, np.float64))
    if Hs.ndim == 2:
        Hs = Hs[None]
    if Hs.ndim != 3 or Hs.shape[1:] != (d, d):
        raise ValueError("H must be m x d x d for d-dimensional samples")
    return Hs


class HPrep:
    """A sample staged once for repeated LSCV_H evaluations
    (kde_lscv_H_prepare / kde_lscv_H_eval_prepared / kde_lscv_H_release)."""

    def __init__(self, ctx, x):
        m, keep = make_matrix(x)
        self.ctx, self.d = ctx, m.d
        self.handle = None
        h = ctypes.c_void_p()
        _check(ctx, lib.kde_lscv_H_prepare(ctx, m, ctypes.byref(h)))
        del keep
        self.handle = h
        _dependents(ctx).add(self)

    def eval(self, H):
        """(g, gscale) at bandwidth matrices H (m x d x d, or one d x d)."""
        Hs = _H_stack(H, self.d)
        k = Hs.shape[0]
        g, gs = np.empty(k, np.float64), np.empty(k, np.float64)
        _check(self.ctx, lib.kde_lscv_H_eval_prepared(self.handle, _pd(Hs.ravel()), int(k), _pd(g), _pd(gs)))
        return g, gs

    def close(self):
        if self.handle:
            lib.kde_lscv_H_release(self.handle)
            self.handle = None

    def _forget(self):
        # the context was destroyed, which released the handle
        self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# Handles created on each context (by its address): kde_ctx_destroy releases
# them, so Context.close tells them to forget theirs first.
_DEPENDENTS = {}


def _dependents(ctx):
    import weakref

    key = ctx.value if isinstance(ctx, ctypes.c_void_p) else int(ctx)
    return _DEPENDENTS.setdefault(key, weakref.WeakSet())


def kde_lscv_H_prepare(ctx, x) -> HPrep:
    """Stages x once for repeated LSCV_H evaluations."""
    return HPrep(ctx, x)


def kde_lscv_H_eval_prepared(prep: HPrep, H):
    """(g, gscale) at bandwidth matrices H over a prepared sample."""
    return prep.eval(H)


def kde_lscv_H_release(prep: HPrep) -> None:
    prep.close()


def kde_density_H(ctx, x, H, points):
    """Density estimate with bandwidth matrix H at points (m x d host array)."""
    m, keep = make_matrix(x)
    d = m.d
    Hm = np.ascontiguousarray(np.asarray(H, np.float64).reshape(d, d))
    p = np.ascontiguousarray(np.asarray(points, np.float64).reshape(-1, d))
    out = np.empty(p.shape[0], np.float64)
    _check(ctx, lib.kde_density_H(ctx, m, _pd(Hm.ravel()), _pd(p.ravel()), int(p.shape[0]), _pd(out)))
    del keep
    return out


def kde_range_aggregates_2d(ctx, x, H, boxes):
    """(count, sum_x, sum_y, avg_x, avg_y) over boxes (rows a, b, c, d) for n x 2 samples."""
    m, keep = make_matrix(x)
    Hm = np.ascontiguousarray(np.asarray(H, np.float64).reshape(2, 2))
    bx = np.ascontiguousarray(np.asarray(boxes, np.float64).reshape(-1, 4))
    q = bx.shape[0]
    outs = [np.empty(q, np.float64) for _ in range(5)]
    _check(ctx, lib.kde_range_aggregates_2d(ctx, m, _pd(Hm.ravel()), _pd(bx.ravel()), int(q), *(_pd(o) for o in outs)))
    del keep
    return tuple(outs)


def kde_bw_lscv_H(ctx, x, ftol: float = 1e-10, xtol: float = 1e-6, max_evals: int = 2000):
    """(H, info) -- the Nelder-Mead LSCV_H bandwidth matrix."""
    m, keep = make_matrix(x)
    H = np.empty(m.d * m.d, np.float64)
    info = kde_lscv_H_info()
    _check(ctx, lib.kde_bw_lscv_H(ctx, m, float(ftol), float(xtol), int(max_evals), _pd(H), ctypes.byref(info)))
    del keep
    return H.reshape(m.d, m.d), info


def kde_density(ctx, x, h: float, points):
    """Density estimate f(points) at bandwidth h."""
    col, keep = make_column(x)
    q = np.ascontiguousarray(np.asarray(points, np.float64).ravel())
    out = np.empty(q.size, np.float64)
    _check(ctx, lib.kde_density(ctx, col, float(h), _pd(q), int(q.size), _pd(out)))
    del keep
    return out


def kde_range_aggregates(ctx, x, h: float, lo, hi):
    """(count, sum, avg) arrays over the ranges [lo[k], hi[k]]."""
    col, keep = make_column(x)
    a = np.ascontiguousarray(np.asarray(lo, np.float64).ravel())
    b = np.ascontiguousarray(np.asarray(hi, np.float64).ravel())
    if a.size != b.size:
        raise ValueError("lo and hi differ in length")
    cnt, sm, av = (np.empty(a.size, np.float64) for _ in range(3))
    _check(ctx, lib.kde_range_aggregates(ctx, col, float(h), _pd(a), _pd(b), int(a.size), _pd(cnt), _pd(sm), _pd(av)))
    del keep
    return cnt, sm, av


def kde_bw_lscv_min(ctx, x, h_lo: float, h_hi: float, rel_tol: float = 1e-4, points: int = 16):
    """(h, info dict) -- LSCV bandwidth by the log-spaced k-section search."""
    col, keep = make_column(x)
    h = ctypes.c_double()
    info = kde_lscv_min_info()
    _check(ctx, lib.kde_bw_lscv_min(ctx, col, float(h_lo), float(h_hi), float(rel_tol), int(points), ctypes.byref(h),
                                    ctypes.byref(info)))
    del keep
    return h.value, {"g": info.g, "iterations": info.iterations, "evaluated": info.evaluated,
                     "bracket": (info.bracket_lo, info.bracket_hi)}


def kde_ctx_graph_stats(ctx):
    """(captures, replays) of the graph option."""
    a = ctypes.c_int64()
    b = ctypes.c_int64()
    _check(ctx, lib.kde_ctx_graph_stats(ctx, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def kde_autotune(ctx, n: int, n_h: int):
    """((hc, tj), {(hc, tj): rate}, {(hc, tj): parity}) -- the persistent LSCV
    sweep variant (bandwidths per block, samples per LDS tile) the tile
    autotuner picks for a column of n samples and an n_h-point grid, with the
    measured pair-term evaluations per second of each variant and whether its
    partial sums passed the bitwise parity gate."""
    t = kde_tune_info()
    _check(ctx, lib.kde_autotune(ctx, int(n), int(n_h), ctypes.byref(t)))
    rates = {v: t.evals_per_s[k] for k, v in enumerate(TUNE_VARIANTS)}
    parity = {v: bool(t.parity[k]) for k, v in enumerate(TUNE_VARIANTS)}
    return (t.hc, t.tj), rates, parity


def kde_lscv_ceiling(ctx, hc: int = 16) -> float:
    """Pair-term evaluations per second of the LSCV sweep's inner loop run
    from one LDS tile (no staging, barriers, masks or partial sums)."""
    r = ctypes.c_double()
    _check(ctx, lib.kde_lscv_ceiling(ctx, int(hc), ctypes.byref(r)))
    return r.value


def kde_issue_rates(ctx) -> dict:
    """Measured vector-ALU issue rates of the device, per clock and per CU:
    {"clock_hz", "cus", "add_f32", "mul_f32", "fma_f32", "exp_f32",
    "lscv_mix", "lscv_mix_zero"}."""
    r = kde_issue_info()
    _check(ctx, lib.kde_issue_rates(ctx, ctypes.byref(r)))
    return {k: getattr(r, k) for k, _ in kde_issue_info._fields_ if k != "pad0"}


def kde_bw_rot(ctx, x) -> float:
    col, keep = make_column(x)
    h = ctypes.c_double()
    _check(ctx, lib.kde_bw_rot(ctx, col, ctypes.byref(h)))
    del keep
    return h.value


@dataclass
class PluginInfo:
    sigma: float
    h_rot: float
    stages: int
    g: tuple
    psi: tuple
    kappa: tuple
    precision_used: tuple
    h: float


def kde_bw_plugin(ctx, x, stages: int = 2):
    """(h, PluginInfo)."""
    col, keep = make_column(x)
    h = ctypes.c_double()
    info = kde_plugin_info()
    _check(ctx, lib.kde_bw_plugin(ctx, col, int(stages), ctypes.byref(h), ctypes.byref(info)))
    del keep
    return h.value, PluginInfo(info.sigma, info.h_rot, info.stages, tuple(info.g), tuple(info.psi),
                               tuple(info.kappa), tuple(info.precision_used), info.h)


def kde_lscv_curve(ctx, x, h_grid=None, n_h: int = 0):
    """(g, gscale, grid) as float64 arrays."""
    col, keep = make_column(x)
    gr = _grid(h_grid)
    m = gr.size if gr is not None else (n_h if n_h > 0 else 150)
    g = np.empty(m, np.float64)
    gs = np.empty(m, np.float64)
    grid_used = np.empty(m, np.float64)
    _check(ctx, lib.kde_lscv_curve(ctx, col, _pd(gr), int(m), _pd(g), _pd(gs), _pd(grid_used)))
    del keep
    return g, gs, grid_used


def kde_lscv_curve_noalloc(ctx, x, h_grid=None, n_h: int = 0):
    """(g, gscale) as float64 arrays, computed in the library's fixed device scratch (no allocation)."""
    col, keep = make_column(x)
    gr = _grid(h_grid)
    m = gr.size if gr is not None else (n_h if n_h > 0 else 150)
    g = np.empty(m, np.float64)
    gs = np.empty(m, np.float64)
    _check(ctx, lib.kde_lscv_curve_noalloc(ctx, col, _pd(gr), int(m), _pd(g), _pd(gs)))
    del keep
    return g, gs


def kde_lscv_sums(ctx, x, h_grid):
    """(s1, s2): pair sums of exp(-D^2/(4h^2)) and exp(-D^2/(2h^2))."""
    col, keep = make_column(x)
    gr = _grid(h_grid)
    s1 = np.empty(gr.size, np.float64)
    s2 = np.empty(gr.size, np.float64)
    _check(ctx, lib.kde_lscv_sums(ctx, col, _pd(gr), int(gr.size), _pd(s1), _pd(s2)))
    del keep
    return s1, s2


def kde_lscv_item_sums(ctx, x, h_grid, sel=()):
    """(n_items, ranges[n_sel, 3] = (i_begin, j_begin, j_end), sums[n_sel, n_h, 2]) of selected work items."""
    col, keep = make_column(x)
    gr = _grid(h_grid)
    sel_a = np.ascontiguousarray(np.asarray(sel, dtype=np.int32))
    m = sel_a.size
    n_items = ctypes.c_int32()
    ranges = np.zeros((max(m, 1), 3), np.int32)
    sums = np.zeros((max(m, 1), gr.size, 2), np.float64)
    P32 = ctypes.POINTER(ctypes.c_int32)
    _check(ctx, lib.kde_lscv_item_sums(ctx, col, _pd(gr), int(gr.size), sel_a.ctypes.data_as(P32) if m else None,
                                       int(m), ctypes.byref(n_items), ranges.ctypes.data_as(P32),
                                       sums.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    del keep
    return n_items.value, ranges[:m], sums[:m]


def kde_bw_lscv(ctx, x, h_grid=None, n_h: int = 0):
    """(h, k, at_edge)."""
    col, keep = make_column(x)
    gr = _grid(h_grid)
    m = gr.size if gr is not None else n_h
    h = ctypes.c_double()
    k = ctypes.c_int32()
    e = ctypes.c_int()
    _check(ctx, lib.kde_bw_lscv(ctx, col, _pd(gr), int(m), ctypes.byref(h), ctypes.byref(k), ctypes.byref(e)))
    del keep
    return h.value, k.value, bool(e.value)


@dataclass
class Request:
    """One bandwidth-selection request: a sample column and what to compute.

    grid: an explicit array of h (data units), or ("log_rot", lo, hi, n_h) for
    n_h log-spaced points over h_rot * [lo, hi], or ("paper", n_h) for the
    paper's default grid.
    """
    x: object
    methods: int = KDE_METHOD_ROT | KDE_METHOD_PLUGIN | KDE_METHOD_LSCV
    stages: int = 3
    grid: object = ("paper", 150)


@dataclass
class Result:
    status: int
    sigma: float
    h_rot: float
    h_plugin: float
    h_lscv: float
    k_lscv: int
    at_edge: bool
    plugin: PluginInfo
    g: np.ndarray
    gscale: np.ndarray
    t_queue_s: float = 0.0
    t_service_s: float = 0.0
    lscv_evals_dense: float = 0.0
    lscv_evals: float = 0.0


def _make_request(r: Request):
    """(kde_request, keepalive list, n_h)."""
    col, keep = make_column(r.x)
    req = kde_request()
    req.x = col
    req.methods = int(r.methods)
    req.stages = int(r.stages)
    keeps = [keep]
    g = r.grid
    if isinstance(g, tuple) and g and g[0] == "log_rot":
        req.grid.kind = KDE_GRID_LOG_ROT
        req.grid.lo, req.grid.hi, req.grid.n_h = float(g[1]), float(g[2]), int(g[3])
    elif isinstance(g, tuple) and g and g[0] == "paper":
        req.grid.kind = KDE_GRID_PAPER
        req.grid.n_h = int(g[1])
    else:
        ga = _grid(g)
        req.grid.kind = KDE_GRID_EXPLICIT
        req.grid.h = _pd(ga)
        req.grid.n_h = ga.size
        keeps.append(ga)
    return req, keeps, int(req.grid.n_h)


def _unpack_result(res: kde_result, g, gs) -> Result:
    p = res.plugin
    info = PluginInfo(p.sigma, p.h_rot, p.stages, tuple(p.g), tuple(p.psi), tuple(p.kappa),
                      tuple(p.precision_used), p.h)
    return Result(res.status, res.sigma, res.h_rot, res.h_plugin, res.h_lscv, res.k_lscv, bool(res.at_edge), info,
                  g, gs, res.t_queue_s, res.t_service_s, res.lscv_evals_dense, res.lscv_evals)


def kde_batch(ctx, requests):
    """Run a list of Request as one job; returns a list of Result (per-request status)."""
    m = len(requests)
    reqs = (kde_request * max(m, 1))()
    outs = (kde_result * max(m, 1))()
    keeps, bufs = [], []
    for k, r in enumerate(requests):
        req, kp, n_h = _make_request(r)
        reqs[k] = req
        keeps.append(kp)
        lscv = (r.methods & KDE_METHOD_LSCV) != 0
        g = np.full(n_h, np.nan) if lscv else None
        gs = np.full(n_h, np.nan) if lscv else None
        bufs.append((g, gs))
        outs[k].g_out = _pd(g)
        outs[k].gscale_out = _pd(gs)
    _check(ctx, lib.kde_batch(ctx, reqs, m, outs))
    del keeps
    return [_unpack_result(outs[k], *bufs[k]) for k in range(m)]


def kde_server_start(ctx, hbm_budget_bytes: int, max_slots: int) -> None:
    _check(ctx, lib.kde_server_start(ctx, int(hbm_budget_bytes), int(max_slots)))


def kde_submit(ctx, request: Request):
    """Submit a Request to the context's server; returns (ticket, n_h or 0). Inputs are copied."""
    req, keep, n_h = _make_request(request)
    t = ctypes.c_uint64()
    _check(ctx, lib.kde_submit(ctx, ctypes.byref(req), ctypes.byref(t)))
    del keep
    return t.value, (n_h if request.methods & KDE_METHOD_LSCV else 0)


def _collect(ctx, fn, ticket, n_h, *extra):
    out = kde_result()
    g = np.full(n_h, np.nan) if n_h else None
    gs = np.full(n_h, np.nan) if n_h else None
    out.g_out = _pd(g)
    out.gscale_out = _pd(gs)
    st = fn(ctx, ticket, ctypes.byref(out), *extra)
    if st == KDE_E_BUSY:
        return None
    _check(ctx, st)
    return _unpack_result(out, g, gs)


def kde_poll(ctx, ticket: int, n_h: int = 0):
    """Result when done, None while pending."""
    return _collect(ctx, lib.kde_poll, ticket, n_h)


def kde_wait(ctx, ticket: int, n_h: int = 0, timeout_s: float = -1.0):
    """Result when done (blocking up to timeout_s; < 0 = no limit), None on timeout."""
    return _collect(ctx, lib.kde_wait, ticket, n_h, float(timeout_s))


def kde_server_stop(ctx) -> None:
    _check(ctx, lib.kde_server_stop(ctx))


def kde_cancel(ctx, ticket: int) -> None:
    _check(ctx, lib.kde_cancel(ctx, int(ticket)))


def kde_job_create(ctx, request: Request):
    """(job handle, n_h or 0): a resumable job for one request; inputs are copied."""
    req, keep, n_h = _make_request(request)
    job = ctypes.c_void_p()
    _check(ctx, lib.kde_job_create(ctx, ctypes.byref(req), ctypes.byref(job)))
    del keep
    return job, (n_h if request.methods & KDE_METHOD_LSCV else 0)


def kde_job_run(ctx, job, max_evals: float) -> bool:
    """Runs the next slice of about max_evals pair-term evaluations; True once finished."""
    done = ctypes.c_int()
    _check(ctx, lib.kde_job_run(job, float(max_evals), ctypes.byref(done)))
    return bool(done.value)


def kde_job_progress(job):
    """(evaluations issued, evaluations in all, finished)."""
    a, b, d = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
    st = lib.kde_job_progress(job, ctypes.byref(a), ctypes.byref(b), ctypes.byref(d))
    if st != KDE_OK:
        raise KdeError(st, "kde_job_progress")
    return a.value, b.value, bool(d.value)


def kde_job_result(ctx, job, n_h: int = 0):
    """Result of a finished job, None before."""
    return _collect(ctx, lambda _c, _j, out: lib.kde_job_result(_j, out), job, n_h)


def kde_job_checkpoint_bytes(job) -> int:
    b = ctypes.c_uint64()
    st = lib.kde_job_checkpoint_bytes(job, ctypes.byref(b))
    if st != KDE_OK:
        raise KdeError(st, "kde_job_checkpoint_bytes")
    return b.value


def kde_job_checkpoint(ctx, job) -> np.ndarray:
    """The job's checkpoint as a uint8 array."""
    buf = np.empty(kde_job_checkpoint_bytes(job), np.uint8)
    _check(ctx, lib.kde_job_checkpoint(job, buf.ctypes.data, buf.size))
    return buf


def kde_job_resume(ctx, job, buf) -> None:
    b = np.ascontiguousarray(np.asarray(buf, np.uint8))
    _check(ctx, lib.kde_job_resume(job, b.ctypes.data, b.size))


def kde_job_destroy(job) -> None:
    lib.kde_job_destroy(job)


class Job:
    """A resumable request on a Context; closing the context releases it."""

    def __init__(self, context, request: Request):
        self.ctx = context.ctx
        self.job = None
        self.job, self.n_h = kde_job_create(self.ctx, request)
        _dependents(self.ctx).add(self)

    def run(self, max_evals: float) -> bool:
        return kde_job_run(self.ctx, self.job, max_evals)

    def run_to_end(self, slice_evals: float = 4e12):
        while not self.run(slice_evals):
            pass
        return self.result()

    def progress(self):
        return kde_job_progress(self.job)

    def result(self):
        return kde_job_result(self.ctx, self.job, self.n_h)

    def checkpoint(self) -> np.ndarray:
        return kde_job_checkpoint(self.ctx, self.job)

    def resume(self, buf) -> None:
        kde_job_resume(self.ctx, self.job, buf)

    def close(self):
        if self.job:
            kde_job_destroy(self.job)
            self.job = None

    def _forget(self):
        self.job = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Context:
    """Owns a kde_ctx; methods forward to the kde_* functions above."""

    def __init__(self, device: int = 0, precision: str = "mixed"):
        self.ctx = kde_ctx_create(device, KDE_PREC_FP64 if precision == "fp64" else KDE_PREC_MIXED)

    def close(self):
        if self.ctx:
            key = self.ctx.value if isinstance(self.ctx, ctypes.c_void_p) else int(self.ctx)
            for dep in list(_DEPENDENTS.pop(key, ())):
                dep._forget()
            kde_ctx_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_precision(self, precision: str):
        kde_ctx_set_precision(self.ctx, KDE_PREC_FP64 if precision == "fp64" else KDE_PREC_MIXED)

    def set_option(self, key, value):
        kde_ctx_set_option(self.ctx, key, value)

    def set_timing(self, enable=True):
        kde_ctx_set_timing(self.ctx, enable)

    def kernel_time(self, family):
        return kde_ctx_kernel_time(self.ctx, family)

    def bw_rot(self, x):
        return kde_bw_rot(self.ctx, x)

    def bw_plugin(self, x, stages=2):
        return kde_bw_plugin(self.ctx, x, stages)

    def autotune(self, n, n_h):
        return kde_autotune(self.ctx, n, n_h)

    def lscv_ceiling(self, hc=16):
        return kde_lscv_ceiling(self.ctx, hc)

    def issue_rates(self):
        return kde_issue_rates(self.ctx)

    def graph_stats(self):
        return kde_ctx_graph_stats(self.ctx)

    def bw_lscv_min(self, x, h_lo, h_hi, rel_tol=1e-4, points=16):
        return kde_bw_lscv_min(self.ctx, x, h_lo, h_hi, rel_tol, points)

    def density(self, x, h, points):
        return kde_density(self.ctx, x, h, points)

    def lscv_md_curve(self, x, h_grid=None, n_h=0):
        return kde_lscv_md_curve(self.ctx, x, h_grid, n_h)

    def bw_lscv_md(self, x, h_grid=None, n_h=0):
        return kde_bw_lscv_md(self.ctx, x, h_grid, n_h)

    def lscv_H_eval(self, x, H):
        return kde_lscv_H_eval(self.ctx, x, H)

    def lscv_H_prepare(self, x):
        return HPrep(self.ctx, x)

    def bw_lscv_H(self, x, ftol=1e-10, xtol=1e-6, max_evals=2000):
        return kde_bw_lscv_H(self.ctx, x, ftol, xtol, max_evals)

    def density_H(self, x, H, points):
        return kde_density_H(self.ctx, x, H, points)

    def range_aggregates_2d(self, x, H, boxes):
        return kde_range_aggregates_2d(self.ctx, x, H, boxes)

    def range_aggregates(self, x, h, lo, hi):
        return kde_range_aggregates(self.ctx, x, h, lo, hi)

    def footprint(self, req):
        return kde_request_footprint(req, self.ctx)

    def lscv_curve(self, x, h_grid=None, n_h=0):
        return kde_lscv_curve(self.ctx, x, h_grid, n_h)

    def lscv_curve_noalloc(self, x, h_grid=None, n_h=0):
        return kde_lscv_curve_noalloc(self.ctx, x, h_grid, n_h)

    def lscv_sums(self, x, h_grid):
        return kde_lscv_sums(self.ctx, x, h_grid)

    def lscv_item_sums(self, x, h_grid, sel=()):
        return kde_lscv_item_sums(self.ctx, x, h_grid, sel)

    def bw_lscv(self, x, h_grid=None, n_h=0):
        return kde_bw_lscv(self.ctx, x, h_grid, n_h)

    def batch(self, requests):
        return kde_batch(self.ctx, requests)

    # serving
    def server_start(self, hbm_budget_bytes: int, max_slots: int):
        self._tickets = {}
        kde_server_start(self.ctx, hbm_budget_bytes, max_slots)

    def submit(self, request: Request) -> int:
        t, n_h = kde_submit(self.ctx, request)
        self._tickets[t] = n_h
        return t

    def poll(self, ticket: int):
        r = kde_poll(self.ctx, ticket, self._tickets.get(ticket, 0))
        if r is not None:
            self._tickets.pop(ticket, None)
        return r

    def wait(self, ticket: int, timeout_s: float = -1.0):
        r = kde_wait(self.ctx, ticket, self._tickets.get(ticket, 0), timeout_s)
        if r is not None:
            self._tickets.pop(ticket, None)
        return r

    def cancel(self, ticket: int):
        kde_cancel(self.ctx, ticket)

    def server_stop(self):
        kde_server_stop(self.ctx)
