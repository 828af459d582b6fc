"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/poisson.h declares, and rejects invalid options before
touching the device."""
import ctypes

import pytest

from paper_1601_05448_amd import poisson as P


def test_library_exports_every_declared_function():
    lib = P.load()
    declared = P.declared_functions()
    assert "poisson_solve" in declared and "poisson_create" in declared
    missing = [n for n in declared if not hasattr(lib, n)]
    assert not missing, f"declared in include/poisson.h but not exported: {missing}"


def test_strerror_covers_every_code():
    for code in range(0, -10, -1):
        assert P.poisson_strerror(code) != "unknown status"
    assert P.poisson_strerror(12345) == "unknown status"


def _create(**kw):
    o = dict(nx=32, ny=32, nz=32, lx=6.28, ly=6.28, lz=6.28, precision=0, coef=0, weight=0, max_iter=0,
             stream=None)
    o.update(kw)
    opts = P.poisson_opts(**o)
    h = ctypes.c_void_p()
    rc = P.load().poisson_create(ctypes.byref(opts), ctypes.byref(h))
    return rc, h.value


@pytest.mark.parametrize("kw", [dict(nx=5), dict(ny=7), dict(nz=2), dict(nx=2048), dict(nx=9), dict(nx=3),
                                dict(nx=72), dict(ny=144), dict(nz=288),
                                dict(lx=0.0), dict(ly=-1.0), dict(lz=float("nan")), dict(precision=2),
                                dict(coef=5), dict(weight=-1), dict(bc_x=2), dict(bc_x=-1)])
def test_create_rejects_invalid_options(kw):
    rc, h = _create(**kw)
    assert rc == P.POISSON_EINVAL and h is None


def test_null_arguments_rejected():
    lib = P.load()
    assert lib.poisson_create(None, None) == P.POISSON_EINVAL
    assert lib.poisson_solve(None, None, None, None, 1e-10) == P.POISSON_EINVAL
    assert lib.poisson_get_stats(None, None) == P.POISSON_EINVAL
    assert lib.poisson_lap_pinv_fp32(None, None, None) == P.POISSON_EINVAL
    lib.poisson_destroy(None)  # NULL is allowed


def test_server_footprint_argument_checks():
    lib = P.load()
    out = ctypes.c_size_t()
    assert lib.poisson_server_footprint(None, 32, 32, 32, 0, ctypes.byref(out)) == P.POISSON_EINVAL


@pytest.mark.parametrize("args", [(0, 4, 0, 0, 0), (1 << 30, 0, 0, 0, 0), (1 << 30, 4, 7, 0, 0),
                                  (1 << 30, 4, 0, 3, 0), (1 << 30, 4, 0, 0, 9)])
def test_server_create_rejects_invalid_options(args):
    budget, slots, prec, coef, weight = args
    h = ctypes.c_void_p()
    rc = P.load().poisson_server_create(budget, slots, prec, coef, weight, 0, None, ctypes.byref(h))
    assert rc == P.POISSON_EINVAL and h.value is None
