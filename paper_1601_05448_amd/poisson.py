"""Python binding of libpoisson (``include/poisson.h``): argument marshalling only.

Every function has the name of the C entry point it calls.  Field arguments are
contiguous float64 torch tensors on the current HIP device (their data_ptr is
handed to the library); all arithmetic of the solve runs in the library's HIP
kernels.  The library must be built (``python -m paper_1601_05448_amd.build``);
if it is missing, loading fails loudly: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass
from typing import Optional, Sequence

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpoisson.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "poisson.h")

POISSON_OK = 0
POISSON_EINVAL = -1
POISSON_ENOMEM = -2
POISSON_EDOMAIN = -3
POISSON_ENOCONV = -4
POISSON_EDIVERGED = -5
POISSON_EHIP = -6
POISSON_ETOOBIG = -7
POISSON_EBUSY = -8
POISSON_ENOTFOUND = -9

POISSON_FP64 = 0
POISSON_FP32_REFINE = 1
POISSON_COEF_RHO_FACE_MEAN = 0
POISSON_COEF_INVRHO_FACE_MEAN = 1
POISSON_W_RHO = 0
POISSON_W_DIAG = 1
POISSON_BC_PERIODIC = 0
POISSON_BC_WALLS_X = 1


class poisson_opts(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double), ("lz", ctypes.c_double),
                ("precision", ctypes.c_int), ("coef", ctypes.c_int), ("weight", ctypes.c_int),
                ("max_iter", ctypes.c_int), ("stream", ctypes.c_void_p), ("inner_tol", ctypes.c_double),
                ("use_graphs", ctypes.c_int), ("bc_x", ctypes.c_int)]


class poisson_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("outer_iters", ctypes.c_int),
                ("rel_resid", ctypes.c_double), ("b_mean_removed", ctypes.c_double),
                ("b_norm", ctypes.c_double), ("rho_min", ctypes.c_double), ("rho_max", ctypes.c_double),
                ("err_bound_rel", ctypes.c_double), ("ms", ctypes.c_double), ("p1_sweeps", ctypes.c_int),
                ("queue_ms", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class PoissonError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {poisson_strerror(code)} ({code})")
        self.code = code


_lib: Optional[ctypes.CDLL] = None


def declared_functions() -> list:
    """Names of the functions include/poisson.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(poisson_\w+)\s*\(", text)))


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1601_05448_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d, ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    pd = ctypes.POINTER(ctypes.c_double)
    lib.poisson_create.argtypes = [ctypes.POINTER(poisson_opts), ctypes.POINTER(vp)]
    lib.poisson_solve.argtypes = [vp, vp, vp, vp, d]
    lib.poisson_solve_noalloc.argtypes = [ctypes.POINTER(poisson_opts), vp, vp, vp, d, ctypes.POINTER(poisson_stats)]
    lib.poisson_get_stats.argtypes = [vp, ctypes.POINTER(poisson_stats)]
    lib.poisson_get_history.argtypes = [vp, pd, i]
    lib.poisson_destroy.argtypes = [vp]
    lib.poisson_destroy.restype = None
    lib.poisson_strerror.argtypes = [i]
    lib.poisson_strerror.restype = ctypes.c_char_p
    lib.poisson_apply.argtypes = [vp, vp, vp, vp]
    lib.poisson_residual.argtypes = [vp, vp, vp, vp, vp, pd, pd]
    lib.poisson_lap_pinv.argtypes = [vp, vp, vp]
    lib.poisson_lap_pinv_fp32.argtypes = [vp, vp, vp]
    lib.poisson_time_sweep.argtypes = [vp, i, i, vp, vp, vp, i, pd]
    lib.poisson_kernel_timer.argtypes = [vp, i, i]
    lib.poisson_kernel_timer_read.argtypes = [vp, pd, ctypes.POINTER(ll)]
    lib.poisson_divergence.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.poisson_project.argtypes = [vp, vp, vp, vp, vp, vp, d, vp, d, pd]
    lib.poisson_deposit.argtypes = [vp, i, vp, vp, vp]
    lib.poisson_interpolate.argtypes = [vp, i, vp, vp, vp]
    if hasattr(lib, "poisson_server_create"):
        lib.poisson_server_create.argtypes = [ctypes.c_size_t, i, i, i, i, i, vp, ctypes.POINTER(vp)]
        lib.poisson_server_submit.argtypes = [vp, i, i, i, d, d, d, i, vp, vp, vp, d, ctypes.POINTER(ll)]
        lib.poisson_server_tick.argtypes = [vp]
        lib.poisson_server_poll.argtypes = [vp, ll, ctypes.POINTER(poisson_stats)]
        lib.poisson_server_destroy.argtypes = [vp]
        lib.poisson_server_destroy.restype = None
        lib.poisson_server_footprint.argtypes = [vp, i, i, i, i, ctypes.POINTER(ctypes.c_size_t)]
        lib.poisson_server_use_graphs.argtypes = [vp, i]
    _lib = lib
    return lib


def poisson_strerror(code: int) -> str:
    return load().poisson_strerror(code).decode()


def _ptr(t) -> Optional[int]:
    """Device address of a contiguous float64 torch tensor (None passes NULL)."""
    if t is None:
        return None
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError("fields must be torch tensors")
    if t.dtype != torch.float64 or not t.is_contiguous() or t.device.type != "cuda":
        raise ValueError("fields must be contiguous float64 tensors on the GPU")
    return t.data_ptr()


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    return int(getattr(stream, "cuda_stream", stream))


def poisson_create(shape: Sequence[int], lengths: Sequence[float], precision: int = POISSON_FP64,
                   coef: int = POISSON_COEF_RHO_FACE_MEAN, weight: int = POISSON_W_RHO,
                   max_iter: int = 0, stream=None, inner_tol: float = 0.0, use_graphs: bool = False,
                   bc_x: int = POISSON_BC_PERIODIC) -> int:
    """Handle for grid `shape` = (nz, ny, nx) on box `lengths` = (lx, ly, lz);
    `bc_x` = POISSON_BC_WALLS_X for zero-flux walls at both ends of x."""
    nz, ny, nx = (int(v) for v in shape)
    o = poisson_opts(nx, ny, nz, float(lengths[0]), float(lengths[1]), float(lengths[2]),
                     precision, coef, weight, max_iter, _stream_ptr(stream), float(inner_tol),
                     1 if use_graphs else 0, int(bc_x))
    h = ctypes.c_void_p()
    rc = load().poisson_create(ctypes.byref(o), ctypes.byref(h))
    if rc != POISSON_OK:
        raise PoissonError(rc, "poisson_create")
    return h.value


def poisson_solve(h: int, rho, b, p, tol: float) -> int:
    """Solve in place into p; returns the status code (raises on argument errors)."""
    rc = load().poisson_solve(h, _ptr(rho), _ptr(b), _ptr(p), float(tol))
    if rc in (POISSON_EINVAL, POISSON_ENOMEM, POISSON_EHIP):
        raise PoissonError(rc, "poisson_solve")
    return rc


def poisson_solve_noalloc(shape: Sequence[int], lengths: Sequence[float], rho, b, p, tol: float,
                          precision: int = POISSON_FP64, coef: int = POISSON_COEF_RHO_FACE_MEAN,
                          weight: int = POISSON_W_RHO, max_iter: int = 0, stream=None, inner_tol: float = 0.0,
                          bc_x: int = POISSON_BC_PERIODIC) -> dict:
    """The allocation-free solve (no handle): returns the stats dict with the
    status under "code" (raises on argument errors)."""
    nz, ny, nx = (int(v) for v in shape)
    o = poisson_opts(nx, ny, nz, float(lengths[0]), float(lengths[1]), float(lengths[2]),
                     precision, coef, weight, max_iter, _stream_ptr(stream), float(inner_tol), 0, int(bc_x))
    st = poisson_stats()
    rc = load().poisson_solve_noalloc(ctypes.byref(o), _ptr(rho), _ptr(b), _ptr(p), float(tol), ctypes.byref(st))
    if rc in (POISSON_EINVAL, POISSON_ENOMEM, POISSON_EHIP):
        raise PoissonError(rc, "poisson_solve_noalloc")
    out = st.as_dict()
    out["code"] = rc
    return out


def poisson_get_stats(h: int) -> dict:
    s = poisson_stats()
    rc = load().poisson_get_stats(h, ctypes.byref(s))
    if rc != POISSON_OK:
        raise PoissonError(rc, "poisson_get_stats")
    return s.as_dict()


def poisson_get_history(h: int, cap: int = 256) -> list:
    buf = (ctypes.c_double * cap)()
    n = load().poisson_get_history(h, buf, cap)
    if n < 0:
        raise PoissonError(n, "poisson_get_history")
    return [buf[k] for k in range(min(n, cap))]


def poisson_destroy(h: Optional[int]) -> None:
    load().poisson_destroy(h)


def poisson_apply(h: int, rho, p, out) -> None:
    rc = load().poisson_apply(h, _ptr(rho), _ptr(p), _ptr(out))
    if rc != POISSON_OK:
        raise PoissonError(rc, "poisson_apply")


def poisson_residual(h: int, rho, b, p, r=None):
    """Returns (||r||, ||b - mean b||); writes r if given."""
    rn, bn = ctypes.c_double(), ctypes.c_double()
    rc = load().poisson_residual(h, _ptr(rho), _ptr(b), _ptr(p), _ptr(r), ctypes.byref(rn), ctypes.byref(bn))
    if rc != POISSON_OK:
        raise PoissonError(rc, "poisson_residual")
    return rn.value, bn.value


def poisson_lap_pinv(h: int, q, delta) -> None:
    rc = load().poisson_lap_pinv(h, _ptr(q), _ptr(delta))
    if rc != POISSON_OK:
        raise PoissonError(rc, "poisson_lap_pinv")


def poisson_lap_pinv_fp32(h: int, q, delta) -> None:
    rc = load().poisson_lap_pinv_fp32(h, _ptr(q), _ptr(delta))
    if rc != POISSON_OK:
        raise PoissonError(rc, "poisson_lap_pinv_fp32")


def poisson_divergence(h: int, rho, mx, my, mz, out) -> None:
    rc = load().poisson_divergence(h, _ptr(rho), _ptr(mx), _ptr(my), _ptr(mz), _ptr(out))
    if rc != POISSON_OK:
        raise PoissonError(rc, "poisson_divergence")


def poisson_project(h: int, rho, mx, my, mz, rhs_div, c_dt: float, p, tol: float) -> tuple:
    """One pressure projection; mx, my, mz and p in/out.  Returns (status, chi):
    POISSON_OK or POISSON_ENOCONV (momentum corrected); other codes raise."""
    chi = ctypes.c_double()
    rc = load().poisson_project(h, _ptr(rho), _ptr(mx), _ptr(my), _ptr(mz), _ptr(rhs_div), float(c_dt), _ptr(p),
                                float(tol), ctypes.byref(chi))
    if rc not in (POISSON_OK, POISSON_ENOCONV):
        raise PoissonError(rc, "poisson_project")
    return rc, chi.value


def poisson_deposit(h: int, pos, q, out) -> None:
    """out = P(q): pos (n_p, 3) device positions, q (n_p,) or None."""
    n = int(pos.shape[0]) if pos is not None else 0
    rc = load().poisson_deposit(h, n, _ptr(pos), _ptr(q), _ptr(out))
    if rc != POISSON_OK:
        raise PoissonError(rc, "poisson_deposit")


def poisson_interpolate(h: int, pos, field, out) -> None:
    n = int(pos.shape[0]) if pos is not None else 0
    rc = load().poisson_interpolate(h, n, _ptr(pos), _ptr(field), _ptr(out))
    if rc != POISSON_OK:
        raise PoissonError(rc, "poisson_interpolate")


def poisson_time_sweep(h: int, sweep: int, fp32: bool, rho, b, p, reps: int) -> float:
    """Average milliseconds of one sweep (1, 2, 3, 5, or 6 = FP64 outer residual
    of a FP32_REFINE handle); p is overwritten."""
    ms = ctypes.c_double()
    rc = load().poisson_time_sweep(h, sweep, 1 if fp32 else 0, _ptr(rho), _ptr(b), _ptr(p), reps, ctypes.byref(ms))
    if rc != POISSON_OK:
        raise PoissonError(rc, "poisson_time_sweep")
    return ms.value


def poisson_kernel_timer(h: int, sweep: int, fp32: bool = False) -> None:
    """Bracket every later launch of `sweep` (1, 2, 3, 5; 0 = off) inside solves
    with HIP events; resets the sums."""
    rc = load().poisson_kernel_timer(h, sweep, 1 if fp32 else 0)
    if rc != POISSON_OK:
        raise PoissonError(rc, "poisson_kernel_timer")


def poisson_kernel_timer_read(h: int) -> tuple:
    """(summed milliseconds, bracketed launches) since the timer was set."""
    ms, n = ctypes.c_double(), ctypes.c_longlong()
    rc = load().poisson_kernel_timer_read(h, ctypes.byref(ms), ctypes.byref(n))
    if rc != POISSON_OK:
        raise PoissonError(rc, "poisson_kernel_timer_read")
    return ms.value, n.value


# ---- serving -------------------------------------------------------------------


def poisson_server_create(budget_bytes: int, max_slots: int, precision: int = POISSON_FP64,
                          coef: int = POISSON_COEF_RHO_FACE_MEAN, weight: int = POISSON_W_RHO,
                          max_iter: int = 0, stream=None) -> int:
    h = ctypes.c_void_p()
    rc = load().poisson_server_create(int(budget_bytes), int(max_slots), precision, coef, weight, max_iter,
                                      _stream_ptr(stream), ctypes.byref(h))
    if rc != POISSON_OK:
        raise PoissonError(rc, "poisson_server_create")
    return h.value


def poisson_server_submit(s: int, shape: Sequence[int], lengths: Sequence[float], rho, b, p,
                          tol: float, bc_x: int = POISSON_BC_PERIODIC) -> int:
    nz, ny, nx = (int(v) for v in shape)
    rid = ctypes.c_longlong()
    rc = load().poisson_server_submit(s, nx, ny, nz, float(lengths[0]), float(lengths[1]), float(lengths[2]),
                                      int(bc_x), _ptr(rho), _ptr(b), _ptr(p), float(tol), ctypes.byref(rid))
    if rc != POISSON_OK:
        raise PoissonError(rc, "poisson_server_submit")
    return rid.value


def poisson_server_tick(s: int) -> int:
    rc = load().poisson_server_tick(s)
    if rc < 0:
        raise PoissonError(rc, "poisson_server_tick")
    return rc


def poisson_server_poll(s: int, rid: int) -> Optional[dict]:
    """Stats dict if the request is done, None while pending."""
    st = poisson_stats()
    rc = load().poisson_server_poll(s, rid, ctypes.byref(st))
    if rc < 0:
        raise PoissonError(rc, "poisson_server_poll")
    return st.as_dict() if rc == 0 else None


def poisson_server_use_graphs(s: int, on: bool) -> None:
    rc = load().poisson_server_use_graphs(s, 1 if on else 0)
    if rc != POISSON_OK:
        raise PoissonError(rc, "poisson_server_use_graphs")


def poisson_server_footprint(s: int, shape: Sequence[int], bc_x: int = POISSON_BC_PERIODIC) -> int:
    """Bytes a request on this grid holds against the server's budget while admitted."""
    nz, ny, nx = (int(v) for v in shape)
    out = ctypes.c_size_t()
    rc = load().poisson_server_footprint(s, nx, ny, nz, int(bc_x), ctypes.byref(out))
    if rc != POISSON_OK:
        raise PoissonError(rc, "poisson_server_footprint")
    return out.value


def poisson_server_destroy(s: Optional[int]) -> None:
    load().poisson_server_destroy(s)


@dataclass
class Solver:
    """Owning wrapper of a handle: Solver(shape, lengths).solve(rho, b, p, tol)."""
    shape: Sequence[int]
    lengths: Sequence[float]
    precision: int = POISSON_FP64
    coef: int = POISSON_COEF_RHO_FACE_MEAN
    weight: int = POISSON_W_RHO
    max_iter: int = 0
    stream: object = None
    inner_tol: float = 0.0
    use_graphs: bool = False
    bc_x: int = POISSON_BC_PERIODIC

    def __post_init__(self):
        self.h = poisson_create(self.shape, self.lengths, self.precision, self.coef, self.weight,
                                self.max_iter, self.stream, self.inner_tol, self.use_graphs, self.bc_x)

    def solve(self, rho, b, p, tol: float = 1e-10) -> dict:
        rc = poisson_solve(self.h, rho, b, p, tol)
        st = poisson_get_stats(self.h)
        st["code"] = rc
        return st

    def history(self) -> list:
        return poisson_get_history(self.h)

    def close(self) -> None:
        if getattr(self, "h", None):
            poisson_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
