/*
 * poisson_oracle.c -- plain, slow, single-threaded FP64 reference ("the oracle")
 * for the periodic variable-coefficient pressure Poisson solve
 *
 *        div( (1/rho) grad p ) = f                      (section "Poisson equation")
 *
 * of Pouransari, Mortazavi & Mani, "Parallel variable-density particle-laden
 * turbulence simulation" (arXiv:1601.05448).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker against which the GPU
 * library is checked.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant with the GPU path and includes nothing from it.
 *
 * Conventions (all readings of the paper are listed in the design notes):
 *   - Grid (nx, ny, nz), uniform spacing h_d = L_d / N_d, triply periodic
 *     (section "Boundary and initial conditions", configuration 1), or, with
 *     bcx = 1, periodic in y and z and bounded in x by walls through which
 *     the pressure flux is zero (the inflow-outflow duct of configuration 2;
 *     the paper gives the convective condition for the flow, and the
 *     pressure condition read here is the homogeneous Neumann one).
 *   - Scalars (rho, p, f) live at cell centres, fluxes on faces (section
 *     "Spatial discretization", staggered-grid figure).  Storage is
 *     [nz][ny][nx], x fastest: idx = (k*ny + j)*nx + i.
 *   - Discrete operator, second order (section "Spatial discretization"):
 *        (A p)_c = sum_d [ beta_{c+1/2} (p_{c+e_d} - p_c)
 *                        - beta_{c-1/2} (p_c - p_{c-e_d}) ] / h_d^2
 *     with the face coefficient beta (the paper never writes it out):
 *        coef 0: beta = 2 / (rho_a + rho_b)      1/rho of the face-averaged rho
 *        coef 1: beta = (1/rho_a + 1/rho_b) / 2  face average of 1/rho
 *   - Compatibility: the right-hand side is made zero-mean by subtracting its
 *     domain mean (the constant chi of Appendix A); p is returned zero-mean.
 *   - The paper's iteration (section "Poisson equation", eq. (Pois)): with
 *     p = p_g + dp, drop the term rho grad(1/rho).grad dp, solve the remaining
 *     constant-coefficient Poisson problem by Fourier transform in the periodic
 *     directions, set p_g <- p_g + dp, and repeat until convergence.  In
 *     residual form one step is
 *        r  = f~ - A p_g,     q = w * r,     L dp = q,     p_g += dp
 *     with w = rho (weight 0, the multiplier of eq. (Pois)) or w = 1/mean of the
 *     six face coefficients (weight 1).  L is the constant-coefficient 7-point
 *     Laplacian, inverted on zero-mean fields through its discrete Fourier
 *     symbol  sum_d -4 sin^2(pi k_d / N_d) / h_d^2; with walls in x, by Fourier
 *     transform in y and z and a tridiagonal solve along x per (k_y, k_z)
 *     mode, as the paper does in its non-periodic direction.
 *
 * Compiled with -O2 -ffp-contract=off: IEEE double, round to nearest, no FMA
 * contraction, no fast-math.
 */
#include <complex.h>
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_EDOMAIN (-3)
#define OR_ENOCONV (-4)
#define OR_EDIVERGED (-5)

typedef double complex cplx;

static const double OR_PI = 3.14159265358979323846264338327950288;

/* ------------------------------------------------------------------------ */
/* grid helpers                                                             */
/* ------------------------------------------------------------------------ */

static size_t cell(int nx, int ny, int i, int j, int k) {
    return ((size_t)k * (size_t)ny + (size_t)j) * (size_t)nx + (size_t)i;
}

static int wrap(int i, int n) { return (i % n + n) % n; }

static double mean_of(const double* a, size_t n);

static int is_2a3b(int n) {
    if (n < 1) return 0;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

static int check_grid(int nx, int ny, int nz, double hx, double hy, double hz) {
    if (nx < 2 || ny < 2 || nz < 2) return OR_EINVAL;
    if (!(hx > 0.0) || !(hy > 0.0) || !(hz > 0.0)) return OR_EINVAL;
    return OR_OK;
}

/* Face coefficient between two cells with densities ra and rb. */
static double face_beta(int coef, double ra, double rb) {
    if (coef == 0) return 2.0 / (ra + rb);
    return 0.5 * (1.0 / ra + 1.0 / rb);
}

/* ------------------------------------------------------------------------ */
/* operator                                                                 */
/* ------------------------------------------------------------------------ */

/* Face coefficient of the face between cell c and its neighbour at offset +1
 * (side = +1) or -1 (side = -1) along direction d; 0 for a wall face (bcx = 1,
 * d = 0, beyond the first or last cell), else beta of the two densities (1
 * when rho is NULL). */
static double face_coef(int nx, int ny, int nz, int coef, int bcx, const double* rho, int i, int j, int k,
                        int d, int side, size_t* nb) {
    const int n3[3] = {nx, ny, nz};
    int ii = i, jj = j, kk = k;
    if (d == 0) ii += side;
    if (d == 1) jj += side;
    if (d == 2) kk += side;
    if (d == 0 && bcx == 1 && (ii < 0 || ii >= nx)) {
        *nb = cell(nx, ny, i, j, k);
        return 0.0;
    }
    *nb = cell(nx, ny, wrap(ii, n3[0]), wrap(jj, n3[1]), wrap(kk, n3[2]));
    if (!rho) return 1.0;
    const size_t c = cell(nx, ny, i, j, k);
    return side > 0 ? face_beta(coef, rho[c], rho[*nb]) : face_beta(coef, rho[*nb], rho[c]);
}

/* out = A p : the second-order flux-form discretisation of div((1/rho) grad p)
 * on the staggered grid, periodic, or with zero-flux walls in x (bcx = 1).
 * rho may be NULL, meaning rho = 1 (then A is the constant-coefficient 7-point
 * Laplacian L). */
int oracle_apply_bc(int nx, int ny, int nz, double hx, double hy, double hz, int coef, int bcx,
                    const double* rho, const double* p, double* out) {
    if (check_grid(nx, ny, nz, hx, hy, hz) != OR_OK || (coef != 0 && coef != 1) || (bcx != 0 && bcx != 1) ||
        !p || !out)
        return OR_EINVAL;
    const double h2[3] = {hx * hx, hy * hy, hz * hz};
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t c = cell(nx, ny, i, j, k);
                double acc = 0.0;
                for (int d = 0; d < 3; ++d) {
                    size_t cp, cm;
                    const double bp = face_coef(nx, ny, nz, coef, bcx, rho, i, j, k, d, +1, &cp);
                    const double bm = face_coef(nx, ny, nz, coef, bcx, rho, i, j, k, d, -1, &cm);
                    acc += (bp * (p[cp] - p[c]) - bm * (p[c] - p[cm])) / h2[d];
                }
                out[c] = acc;
            }
    return OR_OK;
}

int oracle_apply(int nx, int ny, int nz, double hx, double hy, double hz, int coef,
                 const double* rho, const double* p, double* out) {
    return oracle_apply_bc(nx, ny, nz, hx, hy, hz, coef, 0, rho, p, out);
}

/* ------------------------------------------------------------------------ */
/* textbook complex FFT, lengths 2^a 3^b (recursive Cooley-Tukey, DIT)       */
/* ------------------------------------------------------------------------ */

/* X[K] = sum_j x[j*stride] * tw[(j*K*tstep) mod N], with tw[t] = exp(sign*2*pi*i*t/N)
 * and n = N/tstep.  Split j = r*j' + q (r = 2 or 3): X[K] = sum_q w^{qK} Y_q[K mod m]. */
static void fft_rec(const cplx* x, size_t stride, cplx* X, int n, const cplx* tw, int N,
                    int tstep, cplx* scratch) {
    if (n == 1) {
        X[0] = x[0];
        return;
    }
    const int r = (n % 2 == 0) ? 2 : 3;
    const int m = n / r;
    for (int q = 0; q < r; ++q)
        fft_rec(x + (size_t)q * stride, stride * (size_t)r, X + (size_t)q * m, m, tw, N,
                tstep * r, scratch);
    for (int K = 0; K < n; ++K) {
        cplx acc = 0.0;
        for (int q = 0; q < r; ++q) {
            const long t = ((long)q * (long)K) % n;
            acc += tw[(size_t)t * (size_t)tstep % (size_t)N] * X[(size_t)q * m + (size_t)(K % m)];
        }
        scratch[K] = acc;
    }
    memcpy(X, scratch, (size_t)n * sizeof(cplx));
}

static cplx* make_twiddles(int n, int sign) {
    cplx* tw = (cplx*)malloc((size_t)n * sizeof(cplx));
    if (!tw) return NULL;
    for (int t = 0; t < n; ++t) {
        const double a = 2.0 * OR_PI * (double)t / (double)n;
        tw[t] = cos(a) + (double)sign * sin(a) * I;
    }
    return tw;
}

/* In-place 1-D DFT of a line of length n (2^a 3^b), elements at stride. */
static int fft_line(cplx* data, size_t stride, int n, const cplx* tw, cplx* in, cplx* out,
                    cplx* scratch) {
    for (int j = 0; j < n; ++j) in[j] = data[(size_t)j * stride];
    fft_rec(in, 1, out, n, tw, n, 1, scratch);
    for (int j = 0; j < n; ++j) data[(size_t)j * stride] = out[j];
    return OR_OK;
}

/* Exported for pinning: in-place complex DFT of length n, sign -1 forward
 * (exp(-2 pi i jk/n)), +1 backward (unnormalised). */
int oracle_fft1d(int n, double* re, double* im, int sign) {
    if (!is_2a3b(n) || (sign != 1 && sign != -1) || !re || !im) return OR_EINVAL;
    cplx* buf = (cplx*)malloc(4 * (size_t)n * sizeof(cplx));
    cplx* tw = make_twiddles(n, sign);
    if (!buf || !tw) {
        free(buf);
        free(tw);
        return OR_ENOMEM;
    }
    cplx* line = buf;
    for (int j = 0; j < n; ++j) line[j] = re[j] + im[j] * I;
    fft_line(line, 1, n, tw, buf + n, buf + 2 * (size_t)n, buf + 3 * (size_t)n);
    for (int j = 0; j < n; ++j) {
        re[j] = creal(line[j]);
        im[j] = cimag(line[j]);
    }
    free(buf);
    free(tw);
    return OR_OK;
}

/* 3-D DFT of a complex [nz][ny][nx] array along x, then y, then z. */
static int fft3(cplx* a, int nx, int ny, int nz, int sign) {
    const int nmax = nx > ny ? (nx > nz ? nx : nz) : (ny > nz ? ny : nz);
    cplx* buf = (cplx*)malloc(3 * (size_t)nmax * sizeof(cplx));
    cplx* twx = make_twiddles(nx, sign);
    cplx* twy = make_twiddles(ny, sign);
    cplx* twz = make_twiddles(nz, sign);
    if (!buf || !twx || !twy || !twz) {
        free(buf); free(twx); free(twy); free(twz);
        return OR_ENOMEM;
    }
    cplx *in = buf, *out = buf + nmax, *scr = buf + 2 * (size_t)nmax;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) fft_line(a + cell(nx, ny, 0, j, k), 1, nx, twx, in, out, scr);
    for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nx; ++i) fft_line(a + cell(nx, ny, i, 0, k), (size_t)nx, ny, twy, in, out, scr);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            fft_line(a + cell(nx, ny, i, j, 0), (size_t)nx * (size_t)ny, nz, twz, in, out, scr);
    free(buf); free(twx); free(twy); free(twz);
    return OR_OK;
}

/* Discrete symbol of the 1-D periodic second difference: -4 sin^2(pi k/N)/h^2. */
static double symbol_1d(int k, int n, double h) {
    const double s = sin(OR_PI * (double)k / (double)n);
    return -4.0 * s * s / (h * h);
}

/* delta = L^+ q : the zero-mean solution of L delta = q - mean(q), where L is the
 * constant-coefficient periodic 7-point Laplacian (the inner solve of eq. (Pois)
 * "by Fourier transform in the periodic directions").  Forward 3-D DFT, divide by
 * the discrete symbol, zero the k = 0 mode, backward 3-D DFT, scale 1/n. */
int oracle_lap_pinv(int nx, int ny, int nz, double hx, double hy, double hz, const double* q,
                    double* delta) {
    if (check_grid(nx, ny, nz, hx, hy, hz) != OR_OK || !q || !delta) return OR_EINVAL;
    if (!is_2a3b(nx) || !is_2a3b(ny) || !is_2a3b(nz)) return OR_EINVAL;
    const size_t n = (size_t)nx * ny * nz;
    cplx* F = (cplx*)malloc(n * sizeof(cplx));
    if (!F) return OR_ENOMEM;
    for (size_t c = 0; c < n; ++c) F[c] = q[c];
    int rc = fft3(F, nx, ny, nz, -1);
    if (rc != OR_OK) { free(F); return rc; }
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t c = cell(nx, ny, i, j, k);
                if (i == 0 && j == 0 && k == 0) {
                    F[c] = 0.0;
                    continue;
                }
                const double lam = symbol_1d(i, nx, hx) + symbol_1d(j, ny, hy) + symbol_1d(k, nz, hz);
                F[c] /= lam;
            }
    rc = fft3(F, nx, ny, nz, +1);
    if (rc != OR_OK) { free(F); return rc; }
    for (size_t c = 0; c < n; ++c) delta[c] = creal(F[c]) / (double)n;
    free(F);
    return OR_OK;
}

/* Symbol of the 1-D second difference between zero-flux walls (cell centres,
 * mirror ghost cells): -4 sin^2(pi k/(2N))/h^2, k = 0..N-1, eigenvectors
 * cos(pi k (i + 1/2)/N).  Used by the pins and the error bound; the solve below
 * does not use it. */
static double symbol_wall_1d(int k, int n, double h) {
    const double s = sin(OR_PI * (double)k / (2.0 * (double)n));
    return -4.0 * s * s / (h * h);
}

/* Solve (D + c) x = q along one x-line, D the wall second difference (tridiagonal:
 * 1/h^2 off the diagonal, -2/h^2 on it, -1/h^2 at the two ends), c = the y and z
 * symbols of the mode (c < 0), q complex: the Thomas algorithm (the matrix is
 * strictly diagonally dominant, no pivoting needed).  For c = 0 the matrix is
 * singular; then q has zero sum, and the solution with x_0 = 0 follows from the
 * face fluxes g_{i+1/2} = h sum_{j<=i} q_j (g = 0 at both walls):
 * x_{i+1} = x_i + h g_{i+1/2}.  dmod: scratch of n doubles. */
static void tridiag_wall(int n, double h, double c, const cplx* q, double* dmod, cplx* x) {
    const double a = 1.0 / (h * h);
    if (c == 0.0) {
        cplx g = 0.0;
        x[0] = 0.0;
        for (int i = 0; i + 1 < n; ++i) {
            g += h * q[i];
            x[i + 1] = x[i] + h * g;
        }
        return;
    }
    for (int i = 0; i < n; ++i) {
        const double b = ((i == 0 || i == n - 1) ? -a : -2.0 * a) + c;
        if (i == 0) {
            dmod[0] = b;
            x[0] = q[0];
        } else {
            const double m = a / dmod[i - 1];
            dmod[i] = b - m * a;
            x[i] = q[i] - m * x[i - 1];
        }
    }
    x[n - 1] /= dmod[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = (x[i] - a * x[i + 1]) / dmod[i];
}

/* delta = L^+ q with zero-flux walls in x: the zero-mean solution of
 * L delta = q - mean(q).  Forward DFT along y and z, a tridiagonal solve along
 * x for every (k_y, k_z) mode, backward DFT along z and y, scale 1/(ny nz). */
static int lap_pinv_wall(int nx, int ny, int nz, double hx, double hy, double hz, const double* q, double* delta) {
    const size_t n = (size_t)nx * ny * nz;
    const int nmax = nx > ny ? (nx > nz ? nx : nz) : (ny > nz ? ny : nz);
    cplx* F = (cplx*)malloc(n * sizeof(cplx));
    cplx* buf = (cplx*)malloc(3 * (size_t)nmax * sizeof(cplx));
    cplx* line = (cplx*)malloc(2 * (size_t)nx * sizeof(cplx));
    double* dmod = (double*)malloc((size_t)nx * sizeof(double));
    cplx* twy = make_twiddles(ny, -1);
    cplx* twz = make_twiddles(nz, -1);
    cplx* twyb = make_twiddles(ny, +1);
    cplx* twzb = make_twiddles(nz, +1);
    if (!F || !buf || !line || !dmod || !twy || !twz || !twyb || !twzb) {
        free(F); free(buf); free(line); free(dmod); free(twy); free(twz); free(twyb); free(twzb);
        return OR_ENOMEM;
    }
    const double qm = mean_of(q, n);
    for (size_t c = 0; c < n; ++c) F[c] = q[c] - qm;
    cplx *in = buf, *out = buf + nmax, *scr = buf + 2 * (size_t)nmax;
    for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nx; ++i) fft_line(F + cell(nx, ny, i, 0, k), (size_t)nx, ny, twy, in, out, scr);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            fft_line(F + cell(nx, ny, i, j, 0), (size_t)nx * (size_t)ny, nz, twz, in, out, scr);
    cplx *rhs = line, *x = line + nx;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j) {
            const double c = symbol_1d(j, ny, hy) + symbol_1d(k, nz, hz);
            for (int i = 0; i < nx; ++i) rhs[i] = F[cell(nx, ny, i, j, k)];
            tridiag_wall(nx, hx, c, rhs, dmod, x);
            for (int i = 0; i < nx; ++i) F[cell(nx, ny, i, j, k)] = x[i];
        }
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i)
            fft_line(F + cell(nx, ny, i, j, 0), (size_t)nx * (size_t)ny, nz, twzb, in, out, scr);
    for (int k = 0; k < nz; ++k)
        for (int i = 0; i < nx; ++i) fft_line(F + cell(nx, ny, i, 0, k), (size_t)nx, ny, twyb, in, out, scr);
    for (size_t c = 0; c < n; ++c) delta[c] = creal(F[c]) / ((double)ny * (double)nz);
    const double dm = mean_of(delta, n);
    for (size_t c = 0; c < n; ++c) delta[c] -= dm;
    free(F); free(buf); free(line); free(dmod); free(twy); free(twz); free(twyb); free(twzb);
    return OR_OK;
}

int oracle_lap_pinv_bc(int nx, int ny, int nz, double hx, double hy, double hz, int bcx, const double* q,
                       double* delta) {
    if (bcx == 0) return oracle_lap_pinv(nx, ny, nz, hx, hy, hz, q, delta);
    if (bcx != 1 || check_grid(nx, ny, nz, hx, hy, hz) != OR_OK || !q || !delta) return OR_EINVAL;
    if (!is_2a3b(ny) || !is_2a3b(nz)) return OR_EINVAL;
    return lap_pinv_wall(nx, ny, nz, hx, hy, hz, q, delta);
}

/* ------------------------------------------------------------------------ */
/* reductions                                                               */
/* ------------------------------------------------------------------------ */

static double mean_of(const double* a, size_t n) {
    double s = 0.0;
    for (size_t c = 0; c < n; ++c) s += a[c];
    return s / (double)n;
}

static double norm2_of(const double* a, size_t n) {
    double s = 0.0;
    for (size_t c = 0; c < n; ++c) s += a[c] * a[c];
    return sqrt(s);
}

static int check_fields(const double* rho, const double* b, size_t n) {
    for (size_t c = 0; c < n; ++c) {
        if (!isfinite(rho[c]) || !(rho[c] > 0.0)) return OR_EDOMAIN;
        if (!isfinite(b[c])) return OR_EDOMAIN;
    }
    return OR_OK;
}

/* r = (b - mean(b)) - A p.  Returns through the pointers the removed mean of b,
 * ||b - mean(b)||_2 and ||r||_2.  r may be NULL.  This is the O(n) verifier
 * used on any solution, including ones the full oracle solve would take too
 * long to produce. */
int oracle_residual_bc(int nx, int ny, int nz, double hx, double hy, double hz, int coef, int bcx,
                       const double* rho, const double* b, const double* p, double* r,
                       double* b_mean, double* b_norm, double* r_norm) {
    if (check_grid(nx, ny, nz, hx, hy, hz) != OR_OK || (coef != 0 && coef != 1) || (bcx != 0 && bcx != 1) ||
        !rho || !b || !p)
        return OR_EINVAL;
    const size_t n = (size_t)nx * ny * nz;
    double* Ap = (double*)malloc(n * sizeof(double));
    if (!Ap) return OR_ENOMEM;
    oracle_apply_bc(nx, ny, nz, hx, hy, hz, coef, bcx, rho, p, Ap);
    const double bm = mean_of(b, n);
    double sb = 0.0, sr = 0.0;
    for (size_t c = 0; c < n; ++c) {
        const double bt = b[c] - bm;
        const double rc = bt - Ap[c];
        sb += bt * bt;
        sr += rc * rc;
        if (r) r[c] = rc;
    }
    free(Ap);
    if (b_mean) *b_mean = bm;
    if (b_norm) *b_norm = sqrt(sb);
    if (r_norm) *r_norm = sqrt(sr);
    return OR_OK;
}

int oracle_residual(int nx, int ny, int nz, double hx, double hy, double hz, int coef,
                    const double* rho, const double* b, const double* p, double* r,
                    double* b_mean, double* b_norm, double* r_norm) {
    return oracle_residual_bc(nx, ny, nz, hx, hy, hz, coef, 0, rho, b, p, r, b_mean, b_norm, r_norm);
}

/* ------------------------------------------------------------------------ */
/* the paper's iteration                                                    */
/* ------------------------------------------------------------------------ */

/* Weight multiplying the residual before the constant-coefficient solve.
 * weight 0: w = rho (the multiplier in eq. (Pois)); weight 1: w = 1 / (mean of
 * the six face coefficients around the cell). */
static void make_weight(int nx, int ny, int nz, int coef, int bcx, int weight, const double* rho,
                        double* w) {
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t c = cell(nx, ny, i, j, k);
                if (weight == 0) {
                    w[c] = rho[c];
                    continue;
                }
                /* a wall face counts with coefficient 0 */
                double s = 0.0;
                size_t nb;
                for (int d = 0; d < 3; ++d) {
                    s += face_coef(nx, ny, nz, coef, bcx, rho, i, j, k, d, +1, &nb);
                    s += face_coef(nx, ny, nz, coef, bcx, rho, i, j, k, d, -1, &nb);
                }
                w[c] = 6.0 / s;
            }
}

/* The paper's solver.  p is in/out: on entry the estimate p_g, on exit the
 * zero-mean iterate whose relative residual ||r||/||b~|| is <= tol.
 * Iterates: r = b~ - A p; stop if small; p += L^+ (w r).
 * history (may be NULL, length max_iter+1) receives ||r_k|| / ||b~||.
 * Returns OR_OK, OR_ENOCONV (p = last iterate), OR_EDIVERGED (relative residual
 * above 1e8 or not finite), OR_EDOMAIN, OR_EINVAL, OR_ENOMEM. */
int oracle_solve_bc(int nx, int ny, int nz, double hx, double hy, double hz, int coef, int bcx, int weight,
                    const double* rho, const double* b, double* p, double tol, int max_iter,
                    int* iters_out, double* rel_out, double* b_mean_out, double* history) {
    if (check_grid(nx, ny, nz, hx, hy, hz) != OR_OK || (bcx != 0 && bcx != 1)) return OR_EINVAL;
    if ((bcx == 0 && !is_2a3b(nx)) || !is_2a3b(ny) || !is_2a3b(nz)) return OR_EINVAL;
    if ((coef != 0 && coef != 1) || (weight != 0 && weight != 1)) return OR_EINVAL;
    if (!rho || !b || !p || !(tol > 0.0) || max_iter < 0) return OR_EINVAL;
    const size_t n = (size_t)nx * ny * nz;
    if (check_fields(rho, b, n) != OR_OK) return OR_EDOMAIN;

    double* bt = (double*)malloc(n * sizeof(double));
    double* r = (double*)malloc(n * sizeof(double));
    double* w = (double*)malloc(n * sizeof(double));
    double* dp = (double*)malloc(n * sizeof(double));
    if (!bt || !r || !w || !dp) {
        free(bt); free(r); free(w); free(dp);
        return OR_ENOMEM;
    }
    /* compatibility: remove the domain mean of the right-hand side */
    const double bm = mean_of(b, n);
    for (size_t c = 0; c < n; ++c) bt[c] = b[c] - bm;
    const double bn = norm2_of(bt, n);
    if (b_mean_out) *b_mean_out = bm;

    int rc = OR_OK, it = 0;
    double rel = 0.0;
    if (bn == 0.0) {
        for (size_t c = 0; c < n; ++c) p[c] = 0.0;
        if (history) history[0] = 0.0;
        goto done;
    }
    /* gauge: the solution is the zero-mean one */
    {
        const double pm = mean_of(p, n);
        for (size_t c = 0; c < n; ++c) p[c] -= pm;
    }
    make_weight(nx, ny, nz, coef, bcx, weight, rho, w);
    for (it = 0;; ++it) {
        oracle_apply_bc(nx, ny, nz, hx, hy, hz, coef, bcx, rho, p, r);
        for (size_t c = 0; c < n; ++c) r[c] = bt[c] - r[c];
        rel = norm2_of(r, n) / bn;
        if (history) history[it] = rel;
        if (rel <= tol) break;
        if (!isfinite(rel) || rel > 1e8) { /* the iteration is not contracting */
            rc = OR_EDIVERGED;
            break;
        }
        if (it == max_iter) {
            rc = OR_ENOCONV;
            break;
        }
        for (size_t c = 0; c < n; ++c) r[c] *= w[c];
        rc = oracle_lap_pinv_bc(nx, ny, nz, hx, hy, hz, bcx, r, dp);
        if (rc != OR_OK) break;
        for (size_t c = 0; c < n; ++c) p[c] += dp[c];
    }
done:
    if (iters_out) *iters_out = it;
    if (rel_out) *rel_out = rel;
    free(bt); free(r); free(w); free(dp);
    return rc;
}

int oracle_solve(int nx, int ny, int nz, double hx, double hy, double hz, int coef, int weight,
                 const double* rho, const double* b, double* p, double tol, int max_iter,
                 int* iters_out, double* rel_out, double* b_mean_out, double* history) {
    return oracle_solve_bc(nx, ny, nz, hx, hy, hz, coef, 0, weight, rho, b, p, tol, max_iter, iters_out, rel_out,
                           b_mean_out, history);
}

/* ------------------------------------------------------------------------ */
/* independent cross-checks                                                 */
/* ------------------------------------------------------------------------ */

/* Conjugate gradients on the symmetric positive semi-definite -A, restricted
 * to zero-mean vectors: solves -A p = -(b - mean b) from p = 0.  An algorithm
 * unrelated to the paper's iteration, used to cross-check it. */
int oracle_cg_bc(int nx, int ny, int nz, double hx, double hy, double hz, int coef, int bcx,
                 const double* rho, const double* b, double* p, double tol, int max_iter,
                 int* iters_out, double* rel_out) {
    if (check_grid(nx, ny, nz, hx, hy, hz) != OR_OK || (coef != 0 && coef != 1) || (bcx != 0 && bcx != 1))
        return OR_EINVAL;
    if (!rho || !b || !p || !(tol > 0.0) || max_iter < 0) return OR_EINVAL;
    const size_t n = (size_t)nx * ny * nz;
    if (check_fields(rho, b, n) != OR_OK) return OR_EDOMAIN;
    double* r = (double*)malloc(n * sizeof(double));
    double* d = (double*)malloc(n * sizeof(double));
    double* Ad = (double*)malloc(n * sizeof(double));
    if (!r || !d || !Ad) {
        free(r); free(d); free(Ad);
        return OR_ENOMEM;
    }
    const double bm = mean_of(b, n);
    for (size_t c = 0; c < n; ++c) {
        p[c] = 0.0;
        r[c] = -(b[c] - bm); /* residual of -A p = -b~ at p = 0 */
        d[c] = r[c];
    }
    const double bn = norm2_of(r, n);
    double rr = bn * bn;
    int it = 0, rc = OR_OK;
    double rel = bn > 0.0 ? 1.0 : 0.0;
    while (bn > 0.0 && rel > tol) {
        if (it == max_iter) {
            rc = OR_ENOCONV;
            break;
        }
        oracle_apply_bc(nx, ny, nz, hx, hy, hz, coef, bcx, rho, d, Ad);
        double dAd = 0.0;
        for (size_t c = 0; c < n; ++c) dAd += d[c] * (-Ad[c]);
        const double alpha = rr / dAd;
        double rr_new = 0.0;
        for (size_t c = 0; c < n; ++c) {
            p[c] += alpha * d[c];
            r[c] -= alpha * (-Ad[c]);
            rr_new += r[c] * r[c];
        }
        const double beta = rr_new / rr;
        rr = rr_new;
        for (size_t c = 0; c < n; ++c) d[c] = r[c] + beta * d[c];
        rel = sqrt(rr) / bn;
        ++it;
    }
    const double pm = mean_of(p, n);
    for (size_t c = 0; c < n; ++c) p[c] -= pm;
    if (iters_out) *iters_out = it;
    if (rel_out) *rel_out = rel;
    free(r); free(d); free(Ad);
    return rc;
}

int oracle_cg(int nx, int ny, int nz, double hx, double hy, double hz, int coef,
              const double* rho, const double* b, double* p, double tol, int max_iter,
              int* iters_out, double* rel_out) {
    return oracle_cg_bc(nx, ny, nz, hx, hy, hz, coef, 0, rho, b, p, tol, max_iter, iters_out, rel_out);
}

/* Brute force for tiny grids: assemble the n x n matrix of A column by column
 * from oracle_apply, border it with the constraint sum(p) = 0,
 *      [ A   1 ] [p]   [b - mean b]
 *      [ 1^T 0 ] [c] = [    0     ]
 * and solve by Gaussian elimination with partial pivoting. */
int oracle_dense_bc(int nx, int ny, int nz, double hx, double hy, double hz, int coef, int bcx,
                    const double* rho, const double* b, double* p) {
    if (check_grid(nx, ny, nz, hx, hy, hz) != OR_OK || (coef != 0 && coef != 1) || (bcx != 0 && bcx != 1))
        return OR_EINVAL;
    if (!rho || !b || !p) return OR_EINVAL;
    const size_t n = (size_t)nx * ny * nz;
    if (n > 4096) return OR_EINVAL;
    const size_t m = n + 1;
    double* M = (double*)calloc(m * m, sizeof(double));
    double* e = (double*)calloc(n, sizeof(double));
    double* col = (double*)malloc(n * sizeof(double));
    double* rhs = (double*)malloc(m * sizeof(double));
    if (!M || !e || !col || !rhs) {
        free(M); free(e); free(col); free(rhs);
        return OR_ENOMEM;
    }
    for (size_t jc = 0; jc < n; ++jc) {
        e[jc] = 1.0;
        oracle_apply_bc(nx, ny, nz, hx, hy, hz, coef, bcx, rho, e, col);
        e[jc] = 0.0;
        for (size_t ir = 0; ir < n; ++ir) M[ir * m + jc] = col[ir];
    }
    for (size_t t = 0; t < n; ++t) {
        M[t * m + n] = 1.0;
        M[n * m + t] = 1.0;
    }
    const double bm = mean_of(b, n);
    for (size_t t = 0; t < n; ++t) rhs[t] = b[t] - bm;
    rhs[n] = 0.0;
    int rc = OR_OK;
    for (size_t piv = 0; piv < m; ++piv) {
        size_t best = piv;
        for (size_t ir = piv + 1; ir < m; ++ir)
            if (fabs(M[ir * m + piv]) > fabs(M[best * m + piv])) best = ir;
        if (M[best * m + piv] == 0.0) {
            rc = OR_EDOMAIN;
            break;
        }
        if (best != piv) {
            for (size_t jc = 0; jc < m; ++jc) {
                const double tmp = M[piv * m + jc];
                M[piv * m + jc] = M[best * m + jc];
                M[best * m + jc] = tmp;
            }
            const double tmp = rhs[piv];
            rhs[piv] = rhs[best];
            rhs[best] = tmp;
        }
        for (size_t ir = piv + 1; ir < m; ++ir) {
            const double f = M[ir * m + piv] / M[piv * m + piv];
            if (f == 0.0) continue;
            for (size_t jc = piv; jc < m; ++jc) M[ir * m + jc] -= f * M[piv * m + jc];
            rhs[ir] -= f * rhs[piv];
        }
    }
    if (rc == OR_OK) {
        for (size_t ir = m; ir-- > 0;) {
            double s = rhs[ir];
            for (size_t jc = ir + 1; jc < m; ++jc) s -= M[ir * m + jc] * rhs[jc];
            rhs[ir] = s / M[ir * m + ir];
        }
        for (size_t t = 0; t < n; ++t) p[t] = rhs[t];
    }
    free(M); free(e); free(col); free(rhs);
    return rc;
}

int oracle_dense(int nx, int ny, int nz, double hx, double hy, double hz, int coef,
                 const double* rho, const double* b, double* p) {
    return oracle_dense_bc(nx, ny, nz, hx, hy, hz, coef, 0, rho, b, p);
}

/* A-posteriori error bound.  Every face coefficient is >= 1/rho_max in both
 * coefficient modes (wall faces are 0 in A and in L alike), so -A >= (-L)/rho_max
 * on zero-mean fields and ||p - p*||_2 <= rho_max ||r||_2 / lambda_min(-L), with
 * lambda_min = min_d 4 sin^2(pi/N_d) / h_d^2 (4 sin^2(pi/(2 N_x)) / h_x^2 along x
 * between walls).
 * Returns the bound on the absolute 2-norm error given ||r||_2. */
double oracle_error_bound_bc(int nx, int ny, int nz, double hx, double hy, double hz, int bcx,
                             double rho_max, double r_norm) {
    /* smallest nonzero eigenvalue of -L: the lowest mode of one direction */
    double lmin = bcx ? -symbol_wall_1d(1, nx, hx) : -symbol_1d(1, nx, hx);
    const double ly = -symbol_1d(1, ny, hy), lz = -symbol_1d(1, nz, hz);
    if (ly < lmin) lmin = ly;
    if (lz < lmin) lmin = lz;
    return rho_max * r_norm / lmin;
}

double oracle_error_bound(int nx, int ny, int nz, double hx, double hy, double hz,
                          double rho_max, double r_norm) {
    return oracle_error_bound_bc(nx, ny, nz, hx, hy, hz, 0, rho_max, r_norm);
}

/* ------------------------------------------------------------------------ */
/* the projection step around the solve (appendix A)                        */
/* ------------------------------------------------------------------------ */

/* Face momentum m_d lives on the staggered faces (section "Spatial
 * discretization"): m_d[c] is the normal momentum on the face between cell c
 * and its neighbour c + e_d.  The face velocity is u = m / rho_face with
 * 1 / rho_face = beta, the face coefficient of the operator, so that the
 * divergence of beta times the face gradient of p is exactly A p.
 *
 * out = div(u):  out_c = sum_d ( beta_{c+1/2} m_d[c] - beta_{c-1/2} m_d[c-e_d] ) / h_d,
 * periodic, or with walls in x (bcx = 1): the two end faces of every x row are
 * closed, their beta is 0 (face_coef), so the momentum stored for the face
 * between the last and the first cell takes no part. */
int oracle_divergence_bc(int nx, int ny, int nz, double hx, double hy, double hz, int coef, int bcx,
                         const double* rho, const double* mx, const double* my, const double* mz, double* out) {
    if (check_grid(nx, ny, nz, hx, hy, hz) != OR_OK || (coef != 0 && coef != 1) || (bcx != 0 && bcx != 1) || !rho ||
        !mx || !my || !mz || !out)
        return OR_EINVAL;
    const double h[3] = {hx, hy, hz};
    const double* m[3] = {mx, my, mz};
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t c = cell(nx, ny, i, j, k);
                double acc = 0.0;
                for (int d = 0; d < 3; ++d) {
                    size_t cp, cm;
                    const double bp = face_coef(nx, ny, nz, coef, bcx, rho, i, j, k, d, +1, &cp);
                    const double bm = face_coef(nx, ny, nz, coef, bcx, rho, i, j, k, d, -1, &cm);
                    acc += (bp * m[d][c] - bm * m[d][cm]) / h[d];
                }
                out[c] = acc;
            }
    return OR_OK;
}

/* One pressure projection of the time advance (appendix A), periodic box or,
 * with bcx = 1, walls in x (closed end faces, as in oracle_divergence_bc):
 *   1. RHS^Pois = ( div(m~ / rho_face) - RHS^div ) / (C dt)
 *   2. chi' = -mean(RHS^Pois), reported as chi = C dt chi' (the paper's chi)
 *   3. solve div(beta grad p) = RHS^Pois + chi' with the paper's iteration
 *      (oracle_solve_bc; p in/out, the previous pressure as the estimate p_g)
 *   4. m_d <- m~_d - C dt (p_{c+e_d} - p_c) / h_d on every face
 * Afterwards div(m / rho_face) = RHS^div - chi up to C dt times the residual
 * of the solve.  c_dt is the product C_RK4^pre[k] dt.  mx, my, mz are in/out;
 * with walls the momentum of the closed end faces is left as given (the face
 * gradient across them is not defined).  Returns the solve's status (OR_OK,
 * OR_ENOCONV, ...). */
int oracle_project_bc(int nx, int ny, int nz, double hx, double hy, double hz, int coef, int bcx, int weight,
                      const double* rho, double* mx, double* my, double* mz, const double* rhs_div, double c_dt,
                      double* p, double tol, int max_iter, int* iters_out, double* rel_out, double* chi_out) {
    if (check_grid(nx, ny, nz, hx, hy, hz) != OR_OK || (bcx != 0 && bcx != 1) || !rho || !mx || !my || !mz ||
        !rhs_div || !p || !(c_dt > 0.0) || !isfinite(c_dt))
        return OR_EINVAL;
    const size_t n = (size_t)nx * ny * nz;
    double* b = malloc(n * sizeof(double));
    if (!b) return OR_ENOMEM;
    int rc = oracle_divergence_bc(nx, ny, nz, hx, hy, hz, coef, bcx, rho, mx, my, mz, b);
    if (rc != OR_OK) {
        free(b);
        return rc;
    }
    for (size_t c = 0; c < n; ++c) b[c] = (b[c] - rhs_div[c]) / c_dt;
    if (chi_out) *chi_out = -c_dt * mean_of(b, n);
    double bm;
    rc = oracle_solve_bc(nx, ny, nz, hx, hy, hz, coef, bcx, weight, rho, b, p, tol, max_iter, iters_out, rel_out,
                         &bm, NULL);
    free(b);
    if (rc != OR_OK && rc != OR_ENOCONV) return rc;
    const double h[3] = {hx, hy, hz};
    double* m[3] = {mx, my, mz};
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t c = cell(nx, ny, i, j, k);
                for (int d = 0; d < 3; ++d) {
                    size_t cp;  /* a closed face gives cp = c: no correction */
                    (void)face_coef(nx, ny, nz, coef, bcx, NULL, i, j, k, d, +1, &cp);
                    m[d][c] -= c_dt * (p[cp] - p[c]) / h[d];
                }
            }
    return rc;
}

/* ------------------------------------------------------------------------ */
/* particles and the grid: the linear projection P and interpolation I       */
/* ------------------------------------------------------------------------ */

/* The 1-D linear weights of a point x on a periodic line of n cells of width
 * h, cell centres at (i + 1/2) h: with s = x/h - 1/2, i0 = floor(s), f = s - i0,
 * the point gives weight 1 - f to cell i0 and f to cell i0 + 1 (both wrapped). */
static void linear_weights(double x, int n, double h, int* i0, int* i1, double* w0, double* w1) {
    const double s = x / h - 0.5;
    const double fl = floor(s);
    const double f = s - fl;
    long long a = (long long)fl % n;
    if (a < 0) a += n;
    *i0 = (int)a;
    *i1 = (int)((a + 1) % n);
    *w0 = 1.0 - f;
    *w1 = f;
}

/* out = P(q): the particles' values projected to the grid per unit volume
 * (section "Physical model": P takes data from particle locations to the
 * fluid grid, by a linear approximation; here the trilinear, cloud-in-cell,
 * weights of the eight cells around each particle), periodic:
 *     out_c = sum_p q_p W_x W_y W_z / (hx hy hz).
 * pos: n_p rows (x, y, z) in physical units, any real value (wrapped);
 * q: n_p values, or NULL for q = 1.  Particles are added in index order. */
int oracle_deposit(int nx, int ny, int nz, double hx, double hy, double hz, int np, const double* pos,
                   const double* q, double* out) {
    if (check_grid(nx, ny, nz, hx, hy, hz) != OR_OK || np < 0 || (np > 0 && !pos) || !out) return OR_EINVAL;
    const size_t n = (size_t)nx * ny * nz;
    memset(out, 0, n * sizeof(double));
    const double inv_v = 1.0 / (hx * hy * hz);
    for (int p = 0; p < np; ++p) {
        int ix[2], iy[2], iz[2];
        double wx[2], wy[2], wz[2];
        linear_weights(pos[3 * (size_t)p + 0], nx, hx, &ix[0], &ix[1], &wx[0], &wx[1]);
        linear_weights(pos[3 * (size_t)p + 1], ny, hy, &iy[0], &iy[1], &wy[0], &wy[1]);
        linear_weights(pos[3 * (size_t)p + 2], nz, hz, &iz[0], &iz[1], &wz[0], &wz[1]);
        const double qp = q ? q[p] : 1.0;
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a)
                    out[cell(nx, ny, ix[a], iy[b], iz[c])] += qp * wx[a] * wy[b] * wz[c] * inv_v;
    }
    return OR_OK;
}

/* out_p = I(field)(x_p): trilinear interpolation of a cell-centred field at the
 * particle positions (section "Physical model", the linear interpolation I),
 * periodic, with the same weights as P. */
int oracle_interpolate(int nx, int ny, int nz, double hx, double hy, double hz, int np, const double* pos,
                       const double* field, double* out) {
    if (check_grid(nx, ny, nz, hx, hy, hz) != OR_OK || np < 0 || (np > 0 && (!pos || !out)) || !field)
        return OR_EINVAL;
    for (int p = 0; p < np; ++p) {
        int ix[2], iy[2], iz[2];
        double wx[2], wy[2], wz[2];
        linear_weights(pos[3 * (size_t)p + 0], nx, hx, &ix[0], &ix[1], &wx[0], &wx[1]);
        linear_weights(pos[3 * (size_t)p + 1], ny, hy, &iy[0], &iy[1], &wy[0], &wy[1]);
        linear_weights(pos[3 * (size_t)p + 2], nz, hz, &iz[0], &iz[1], &wz[0], &wz[1]);
        double acc = 0.0;
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int a = 0; a < 2; ++a) acc += wx[a] * wy[b] * wz[c] * field[cell(nx, ny, ix[a], iy[b], iz[c])];
        out[p] = acc;
    }
    return OR_OK;
}

int oracle_abi_version(void) { return 5; }
