"""ctypes binding of the FP64 CPU oracle (``oracle/poisson_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark use it to check the GPU library.  The product path never
imports it, and this module imports nothing from the product.

Each function cites the part of Pouransari, Mortazavi & Mani (arXiv:1601.05448)
that it follows; see the C source for the discrete definitions.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "poisson_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ENOMEM, EDOMAIN, ENOCONV, EDIVERGED = 0, -1, -2, -3, -4, -5

COEF_RHO_FACE_MEAN = 0  # beta = 2 / (rho_a + rho_b)
COEF_INVRHO_FACE_MEAN = 1  # beta = (1/rho_a + 1/rho_b) / 2
WEIGHT_RHO = 0  # w = rho, the multiplier of eq. (Pois)
WEIGHT_DIAG = 1  # w = 1 / mean of the six face coefficients
BC_PERIODIC = 0  # periodic in x (and always in y, z)
BC_WALLS_X = 1  # zero-flux walls at both ends of x: the inflow-outflow duct


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: plain IEEE FP64, no FMA contraction."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib: Optional[ctypes.CDLL] = None


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    _lib = _configure(ctypes.CDLL(_LIB_PATH))
    return _lib


@contextlib.contextmanager
def use_library(path: str):
    """Route every call through another build of the oracle source, e.g. a copy
    with a planted mistake, to show that the pins catch it."""
    global _lib
    saved = _lib
    _lib = _configure(ctypes.CDLL(path))
    try:
        yield
    finally:
        _lib = saved


def _configure(lib: ctypes.CDLL) -> ctypes.CDLL:
    i, d, pd, pi = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)
    pdd = ctypes.POINTER(ctypes.c_double)
    grid = [i, i, i, d, d, d]
    lib.oracle_apply_bc.argtypes = grid + [i, i, pd, pd, pd]
    lib.oracle_fft1d.argtypes = [i, pd, pd, i]
    lib.oracle_lap_pinv_bc.argtypes = grid + [i, pd, pd]
    lib.oracle_residual_bc.argtypes = grid + [i, i, pd, pd, pd, pd, pdd, pdd, pdd]
    lib.oracle_solve_bc.argtypes = grid + [i, i, i, pd, pd, pd, d, i, pi, pdd, pdd, pd]
    lib.oracle_cg_bc.argtypes = grid + [i, i, pd, pd, pd, d, i, pi, pdd]
    lib.oracle_dense_bc.argtypes = grid + [i, i, pd, pd, pd]
    lib.oracle_error_bound_bc.argtypes = grid + [i, d, d]
    lib.oracle_error_bound_bc.restype = d
    lib.oracle_divergence_bc.argtypes = grid + [i, i, pd, pd, pd, pd, pd]
    lib.oracle_project_bc.argtypes = grid + [i, i, i, pd, pd, pd, pd, pd, d, pd, d, i, pi, pdd, pdd]
    lib.oracle_deposit.argtypes = grid + [i, pd, pd, pd]
    lib.oracle_interpolate.argtypes = grid + [i, pd, pd, pd]
    return lib


def _f64(a: np.ndarray, shape) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {a.shape}")
    return a


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _grid(shape, lengths):
    nz, ny, nx = shape
    lx, ly, lz = lengths
    return nx, ny, nz, lx / nx, ly / ny, lz / nz


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed with code {code}")
        self.code = code


def _check(rc: int, what: str, allow=(OK,)):
    if rc not in allow:
        raise OracleError(rc, what)
    return rc


def apply(rho: Optional[np.ndarray], p: np.ndarray, lengths=(2 * np.pi,) * 3,
          coef: int = COEF_RHO_FACE_MEAN, bcx: int = BC_PERIODIC) -> np.ndarray:
    """A p: flux-form second-order div((1/rho) grad p), periodic, or with
    zero-flux walls in x (bcx = 1, the duct of section "Boundary and initial
    conditions") (section "Poisson equation"; staggered grid of section
    "Spatial discretization").  rho=None means rho = 1, i.e. the 7-point
    Laplacian."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    shape = p.shape
    rho = None if rho is None else _f64(rho, shape)
    out = np.empty(shape)
    _check(_load().oracle_apply_bc(*_grid(shape, lengths), coef, bcx, _ptr(rho), _ptr(p), _ptr(out)), "apply")
    return out


def fft1d(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """Textbook radix-2/3 DFT, sum_j x_j exp(sign 2 pi i jk/n), unnormalised."""
    x = np.asarray(x, dtype=np.complex128)
    re = np.ascontiguousarray(x.real)
    im = np.ascontiguousarray(x.imag)
    _check(_load().oracle_fft1d(x.size, _ptr(re), _ptr(im), sign), "fft1d")
    return re + 1j * im


def lap_pinv(q: np.ndarray, lengths=(2 * np.pi,) * 3, bcx: int = BC_PERIODIC) -> np.ndarray:
    """L^+ q: zero-mean solution of the constant-coefficient problem, by
    Fourier transform in the periodic directions and, with walls in x, a
    tridiagonal solve along x per (k_y, k_z) mode (section "Poisson
    equation")."""
    q = np.ascontiguousarray(q, dtype=np.float64)
    out = np.empty(q.shape)
    _check(_load().oracle_lap_pinv_bc(*_grid(q.shape, lengths), bcx, _ptr(q), _ptr(out)), "lap_pinv")
    return out


def residual(rho, b, p, lengths=(2 * np.pi,) * 3, coef: int = COEF_RHO_FACE_MEAN,
             want_field: bool = False, bcx: int = BC_PERIODIC):
    """(b - mean b) - A p and its norms: the O(n) verifier (compatibility
    constant chi of Appendix A removes the mean of the right-hand side).
    Returns dict(b_mean, b_norm, r_norm, rel[, r])."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    shape = b.shape
    rho, p = _f64(rho, shape), _f64(p, shape)
    r = np.empty(shape) if want_field else None
    bm, bn, rn = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(_load().oracle_residual_bc(*_grid(shape, lengths), coef, bcx, _ptr(rho), _ptr(b), _ptr(p),
                                   _ptr(r), ctypes.byref(bm), ctypes.byref(bn), ctypes.byref(rn)),
           "residual")
    out = dict(b_mean=bm.value, b_norm=bn.value, r_norm=rn.value,
               rel=(rn.value / bn.value) if bn.value > 0 else 0.0)
    if want_field:
        out["r"] = r
    return out


def solve(rho, b, p0=None, lengths=(2 * np.pi,) * 3, coef: int = COEF_RHO_FACE_MEAN,
          weight: int = WEIGHT_RHO, tol: float = 1e-13, max_iter: int = 10000,
          allow_noconv: bool = False, bcx: int = BC_PERIODIC, allow_diverged: bool = False):
    """The paper's iteration (section "Poisson equation", eq. (Pois)):
    r = b~ - A p, q = w r, dp = L^+ q, p += dp, until ||r||/||b~|| <= tol.
    Returns dict(p, iters, rel, b_mean, history, code); allow_noconv and
    allow_diverged return the cap and divergence codes instead of raising."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    shape = b.shape
    rho = _f64(rho, shape)
    p = np.zeros(shape) if p0 is None else np.array(p0, dtype=np.float64, order="C", copy=True)
    hist = np.zeros(max_iter + 1)
    it, rel, bm = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
    rc = _load().oracle_solve_bc(*_grid(shape, lengths), coef, bcx, weight, _ptr(rho), _ptr(b), _ptr(p),
                              tol, max_iter, ctypes.byref(it), ctypes.byref(rel), ctypes.byref(bm),
                              _ptr(hist))
    _check(rc, "solve", allow=(OK,) + ((ENOCONV,) if allow_noconv else ()) + ((EDIVERGED,) if allow_diverged else ()))
    return dict(p=p, iters=it.value, rel=rel.value, b_mean=bm.value,
                history=hist[: it.value + 1].copy(), code=rc)


def cg(rho, b, lengths=(2 * np.pi,) * 3, coef: int = COEF_RHO_FACE_MEAN, tol: float = 1e-13,
       max_iter: int = 100000, bcx: int = BC_PERIODIC):
    """Conjugate gradients on -A over zero-mean fields: an independent
    algorithm for cross-checking the iteration."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    shape = b.shape
    rho = _f64(rho, shape)
    p = np.empty(shape)
    it, rel = ctypes.c_int(), ctypes.c_double()
    _check(_load().oracle_cg_bc(*_grid(shape, lengths), coef, bcx, _ptr(rho), _ptr(b), _ptr(p), tol,
                             max_iter, ctypes.byref(it), ctypes.byref(rel)), "cg")
    return dict(p=p, iters=it.value, rel=rel.value)


def dense(rho, b, lengths=(2 * np.pi,) * 3, coef: int = COEF_RHO_FACE_MEAN, bcx: int = BC_PERIODIC) -> np.ndarray:
    """Brute-force bordered dense solve (Gaussian elimination) for tiny grids."""
    b = np.ascontiguousarray(b, dtype=np.float64)
    shape = b.shape
    rho = _f64(rho, shape)
    p = np.empty(shape)
    _check(_load().oracle_dense_bc(*_grid(shape, lengths), coef, bcx, _ptr(rho), _ptr(b), _ptr(p)), "dense")
    return p


def error_bound(shape, lengths, rho_max: float, r_norm: float, bcx: int = BC_PERIODIC) -> float:
    """Upper bound on ||p - p*||_2 from ||r||_2, valid in both coefficient modes."""
    return _load().oracle_error_bound_bc(*_grid(shape, lengths), bcx, rho_max, r_norm)


def divergence(rho, mx, my, mz, lengths=(2 * np.pi,) * 3, coef: int = COEF_RHO_FACE_MEAN,
               bcx: int = BC_PERIODIC) -> np.ndarray:
    """div(u) of face momentum m (m_d[c] on the face between c and c + e_d),
    u = m / rho_face with 1/rho_face the operator's face coefficient; periodic,
    or closed at both x ends with walls (appendix A, the divergence of the
    predicted momentum over rho)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    shape = rho.shape
    ms = [_f64(m, shape) for m in (mx, my, mz)]
    out = np.empty(shape)
    _check(_load().oracle_divergence_bc(*_grid(shape, lengths), coef, bcx, _ptr(rho), *(_ptr(m) for m in ms),
                                        _ptr(out)), "divergence")
    return out


def project(rho, mx, my, mz, rhs_div, c_dt: float, p0=None, lengths=(2 * np.pi,) * 3,
            coef: int = COEF_RHO_FACE_MEAN, weight: int = WEIGHT_RHO, tol: float = 1e-13,
            max_iter: int = 10000, bcx: int = BC_PERIODIC):
    """One pressure projection (appendix A): RHS^Pois from the predicted face
    momentum and the divergence target, chi from its mean, the solve, and the
    momentum correction -C dt grad p (not across the closed x end faces with
    walls).  Returns dict(p, mx, my, mz, chi, iters, rel, code); the inputs are
    not modified."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    shape = rho.shape
    ms = [np.array(m, dtype=np.float64, order="C", copy=True) for m in (mx, my, mz)]
    for m in ms:
        if m.shape != shape:
            raise ValueError("momentum shape")
    rd = _f64(rhs_div, shape)
    p = np.zeros(shape) if p0 is None else np.array(p0, dtype=np.float64, order="C", copy=True)
    it, rel, chi = ctypes.c_int(), ctypes.c_double(), ctypes.c_double()
    rc = _load().oracle_project_bc(*_grid(shape, lengths), coef, bcx, weight, _ptr(rho), *(_ptr(m) for m in ms),
                                   _ptr(rd), float(c_dt), _ptr(p), tol, max_iter, ctypes.byref(it), ctypes.byref(rel),
                                   ctypes.byref(chi))
    _check(rc, "project", allow=(OK, ENOCONV))
    return dict(p=p, mx=ms[0], my=ms[1], mz=ms[2], chi=chi.value, iters=it.value, rel=rel.value, code=rc)


def deposit(shape, pos, q=None, lengths=(2 * np.pi,) * 3) -> np.ndarray:
    """P(q): particle values projected to the cell centres per unit volume with
    trilinear (cloud-in-cell) weights, periodic (section "Physical model").
    pos: (n_p, 3) positions (x, y, z); q: (n_p,) or None for ones."""
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    qq = None if q is None else np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    if qq is not None and qq.size != pos.shape[0]:
        raise ValueError("q length")
    out = np.empty(tuple(shape))
    _check(_load().oracle_deposit(*_grid(tuple(shape), lengths), pos.shape[0], _ptr(pos), _ptr(qq), _ptr(out)),
           "deposit")
    return out


def interpolate(field, pos, lengths=(2 * np.pi,) * 3) -> np.ndarray:
    """I(field)(x_p): trilinear interpolation of a cell-centred field at the
    particle positions, periodic (section "Physical model")."""
    field = np.ascontiguousarray(field, dtype=np.float64)
    pos = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
    out = np.empty(pos.shape[0])
    _check(_load().oracle_interpolate(*_grid(field.shape, lengths), pos.shape[0], _ptr(pos), _ptr(field),
                                      _ptr(out)), "interpolate")
    return out
