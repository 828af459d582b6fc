"""Planted mistakes in the oracle must each fail at least one pin.

Each case copies the oracle's C source, makes one plausible mistake in it (a
wrong coefficient, a flipped sign, a wrong neighbour index, swapped spacings, a
dropped mean removal, a wrong FFT twiddle ...), builds the copy with gcc into a
temporary directory and runs the pins of test_oracle_pins against it.  The real
oracle is untouched; everything happens on the CPU.
"""
import os
import subprocess

import pytest

import oracle
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "poisson_oracle.c")

MUTANTS = {
    "face coefficient halved": ("return 2.0 / (ra + rb);", "return 1.0 / (ra + rb);"),
    "flux difference sign": ("acc += (bp * (p[cp] - p[c]) - bm * (p[c] - p[cm])) / h2[d];",
                             "acc += (bp * (p[cp] - p[c]) + bm * (p[c] - p[cm])) / h2[d];"),
    "minus face uses the centre density twice": (
        "face_beta(coef, rho[c], rho[*nb]) : face_beta(coef, rho[*nb], rho[c]);",
        "face_beta(coef, rho[c], rho[*nb]) : face_beta(coef, rho[c], rho[c]);"),
    "spacings swapped y<->z": ("const double h2[3] = {hx * hx, hy * hy, hz * hz};",
                               "const double h2[3] = {hx * hx, hz * hz, hy * hy};"),
    "x minus neighbour wrong": ("if (d == 0) ii += side;", "if (d == 0) ii += (side < 0 ? 2 * side : side);"),
    "symbol factor": ("return -4.0 * s * s / (h * h);\n}\n\n/* delta = L^+ q : the zero-mean",
                      "return -2.0 * s * s / (h * h);\n}\n\n/* delta = L^+ q : the zero-mean"),
    "symbol axes transposed": ("symbol_1d(i, nx, hx) + symbol_1d(j, ny, hy)", "symbol_1d(i, nx, hx) + symbol_1d(j, ny, hx)"),
    "zero mode kept": ("                    F[c] = 0.0;\n                    continue;",
                       "                    continue;"),
    "weight inverted": ("w[c] = rho[c];", "w[c] = 1.0 / rho[c];"),
    "update sign": ("p[c] += dp[c];\n    }\ndone:", "p[c] -= 0.5 * dp[c];\n    }\ndone:"),
    "mean of b not removed": ("for (size_t c = 0; c < n; ++c) bt[c] = b[c] - bm;",
                              "for (size_t c = 0; c < n; ++c) bt[c] = b[c];"),
    "twiddle sign ignored": ("tw[t] = cos(a) + (double)sign * sin(a) * I;", "tw[t] = cos(a) - sin(a) * I;"),
    "radix-3 combine index": ("const long t = ((long)q * (long)K) % n;", "const long t = ((long)q * (long)(K % m)) % n;"),
    "gauge not fixed": ("for (size_t c = 0; c < n; ++c) p[c] -= pm;\n    }\n    make_weight",
                        "(void)pm;\n    }\n    make_weight"),
    "wall face kept": ("if (d == 0 && bcx == 1 && (ii < 0 || ii >= nx)) {",
                       "if (d == 0 && bcx == 1 && (ii < 0 || ii >= nx) && 0) {"),
    "wall end of the tridiagonal": ("const double b = ((i == 0 || i == n - 1) ? -a : -2.0 * a) + c;",
                                    "const double b = -2.0 * a + c;"),
    "tridiagonal back substitution": ("x[i] = (x[i] - a * x[i + 1]) / dmod[i];",
                                      "x[i] = (x[i] + a * x[i + 1]) / dmod[i];"),
    "divergence minus face": ("acc += (bp * m[d][c] - bm * m[d][cm]) / h[d];",
                              "acc += (bp * m[d][c] - bm * m[d][cp]) / h[d];"),
    "divergence target dropped": ("b[c] = (b[c] - rhs_div[c]) / c_dt;", "b[c] = b[c] / c_dt;"),
    "chi sign": ("*chi_out = -c_dt * mean_of(b, n);", "*chi_out = c_dt * mean_of(b, n);"),
    "deposit weights swapped": ("    *w0 = 1.0 - f;\n    *w1 = f;", "    *w0 = f;\n    *w1 = 1.0 - f;"),
    "deposit upper neighbour": ("*i1 = (int)((a + 1) % n);", "*i1 = (int)((a + n - 1) % n);"),
    "deposit not per unit volume": ("const double inv_v = 1.0 / (hx * hy * hz);", "const double inv_v = 1.0 / (hx * hy);"),
    "interpolation drops a corner": ("for (int a = 0; a < 2; ++a) acc += wx[a]", "for (int a = 0; a < 1; ++a) acc += wx[a]"),
    "momentum correction sign": ("m[d][c] -= c_dt * (p[cp] - p[c]) / h[d];",
                                 "m[d][c] += c_dt * (p[cp] - p[c]) / h[d];"),
    "correction across the closed x face": ("(void)face_coef(nx, ny, nz, coef, bcx, NULL, i, j, k, d, +1, &cp);",
                                            "(void)face_coef(nx, ny, nz, coef, 0, NULL, i, j, k, d, +1, &cp);"),
    "divergence ignores the walls": (
        "int rc = oracle_divergence_bc(nx, ny, nz, hx, hy, hz, coef, bcx, rho, mx, my, mz, b);",
        "int rc = oracle_divergence_bc(nx, ny, nz, hx, hy, hz, coef, 0, rho, mx, my, mz, b);"),
}


def _caught(lib_path):
    with oracle.use_library(lib_path):
        for pin in pins.ALL_PINS:
            try:
                pin()
            except (AssertionError, oracle.OracleError, FloatingPointError):
                return pin.__name__
    return None


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name!r} not unique in the oracle source"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o",
                    str(lib), str(mut), "-lm"], check=True)
    import numpy as np
    with np.errstate(all="ignore"):
        who = _caught(str(lib))
    assert who is not None, f"no pin caught the planted mistake {name!r}"
