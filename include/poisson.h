/*
 * poisson.h -- C ABI of libpoisson, an MI355X (gfx950) solver for the
 * variable-coefficient pressure Poisson equation
 *
 *        div( (1/rho) grad p ) = b
 *
 * on a uniform staggered grid, periodic in y and z and either periodic or
 * closed by zero-flux walls in x (bc_x below), by the iteration of
 * Pouransari, Mortazavi & Mani, "Parallel variable-density particle-laden
 * turbulence simulation" (arXiv:1601.05448), section "Poisson equation",
 * eq. (Pois): write p = p_g + dp, drop the term rho grad(1/rho).grad dp, solve
 * the remaining constant-coefficient Poisson equation by Fourier transform in
 * the periodic directions (a transform that diagonalises the same operator
 * along a walled x), set p_g <- p_g + dp and repeat until convergence.
 *
 * Discretisation (section "Spatial discretization"; staggered-grid figure):
 * rho, b and p live at cell centres, fluxes on faces, second order:
 *     (A p)_c = sum_d [ beta_{c+1/2}(p_{c+e_d} - p_c) - beta_{c-1/2}(p_c - p_{c-e_d}) ] / h_d^2
 * with h_d = L_d / N_d and the face coefficient chosen by `coef` below.
 * Compatibility (Appendix A, the constant chi): the mean of b is removed
 * before solving, and p is returned with zero mean.
 *
 * Fields: contiguous arrays of n = nx*ny*nz values laid out [nz][ny][nx]
 * (x fastest), index (k*ny + j)*nx + i, cell centre ((i+1/2)hx, (j+1/2)hy,
 * (k+1/2)hz).  Every field pointer is a DEVICE pointer (hipMalloc'd memory,
 * e.g. torch.Tensor.data_ptr()) on the current HIP device.  Callers own rho,
 * b and p; the library owns its workspace.  rho, b and p must not overlap.
 *
 * Grid sizes: each of nx, ny, nz must be 2^a or 3*2^a with 4 <= N <= 1024
 * (lengths with a factor 9 or more of 3 are rejected with POISSON_EINVAL: the
 * transforms are compiled per length, and the paper fixes no grid sizes).
 *
 * Threading: a handle is used by one host thread at a time.  Calls enqueue
 * work on the handle's stream and, unless stated otherwise, block until that
 * work has finished.  No C++ exception crosses this interface.
 */
#ifndef PAPER_1601_05448_AMD_POISSON_H
#define PAPER_1601_05448_AMD_POISSON_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define POISSON_OK 0
#define POISSON_EINVAL (-1)    /* bad size, NULL or overlapping pointer, tol <= 0, bad enum */
#define POISSON_ENOMEM (-2)    /* device or host allocation failed                         */
#define POISSON_EDOMAIN (-3)   /* rho <= 0, non-finite rho or b, or max/min rho above the   */
                               /* supported ratio (1e20 FP64, 1e8 FP32_REFINE); p untouched */
#define POISSON_ENOCONV (-4)   /* max_iter reached; p holds the last iterate               */
#define POISSON_EDIVERGED (-5) /* residual grew above 1e8 x ||b~|| or became non-finite    */
#define POISSON_EHIP (-6)      /* HIP runtime error                                        */
#define POISSON_ETOOBIG (-7)   /* serving: request larger than the memory budget           */
#define POISSON_EBUSY (-8)     /* serving: no free slot or memory right now, retry later   */
#define POISSON_ENOTFOUND (-9) /* serving: unknown request id                              */

/* ---- options ------------------------------------------------------------ */
/* Arithmetic of the solve. */
#define POISSON_FP64 0        /* every sweep in FP64                                       */
#define POISSON_FP32_REFINE 1 /* FP32 sweeps, FP64 residual, mean removal and update       */

/* Face coefficient beta between cells a and b (the paper does not write the
 * discrete operator out; both readings are second order and symmetric). */
#define POISSON_COEF_RHO_FACE_MEAN 0    /* beta = 2 / (rho_a + rho_b): 1/rho of the face rho */
#define POISSON_COEF_INVRHO_FACE_MEAN 1 /* beta = (1/rho_a + 1/rho_b) / 2                      */

/* Multiplier of the residual before the constant-coefficient solve.  It
 * changes the iteration count, never the converged answer. */
#define POISSON_W_RHO 0  /* w = rho, the multiplier of eq. (Pois)                */
#define POISSON_W_DIAG 1 /* w = 1 / (mean of the six face coefficients of a cell) */

/* Boundary condition along x (y and z are always periodic).  Section
 * "Boundary and initial conditions": a triply periodic box, or an
 * inflow-outflow duct, periodic in y-z and bounded in x; for the pressure solve
 * the duct's x ends are read as walls through which the pressure flux is zero
 * (homogeneous Neumann).  The paper solves that direction with a tridiagonal
 * solver; this library uses the cosine transform that diagonalises the same
 * discrete operator (cos(pi k (i + 1/2)/Nx), symbol -4 sin^2(pi k/(2 Nx))/hx^2). */
#define POISSON_BC_PERIODIC 0
#define POISSON_BC_WALLS_X 1

typedef struct poisson_s* poisson_t;

typedef struct {
    int nx, ny, nz;       /* cells per direction                                   */
    double lx, ly, lz;    /* box lengths; h_d = l_d / n_d                           */
    int precision;        /* POISSON_FP64 or POISSON_FP32_REFINE                   */
    int coef;             /* POISSON_COEF_*                                         */
    int weight;           /* POISSON_W_*                                            */
    int max_iter;         /* cap on (inner) iterations; <= 0 selects 1000           */
    void* stream;         /* the caller's hipStream_t (NULL = the null stream): a
                             solve is ordered after the work enqueued on it before
                             the call and runs on a stream of the handle's own      */
    double inner_tol;     /* FP32_REFINE: relative residual at which the FP32 inner
                             sweeps of a refinement step stop; <= 0 selects 5e-4   */
    int use_graphs;       /* nonzero: chunks of iterations are captured once into
                             HIP graphs and replayed; 0: every kernel is launched
                             directly (same kernels, same results)                 */
    int bc_x;             /* POISSON_BC_PERIODIC or POISSON_BC_WALLS_X             */
} poisson_opts;

typedef struct {
    int status;             /* POISSON_* code of the last solve                           */
    int iters;              /* FP64: iterations; FP32_REFINE: inner iterations in total   */
    int outer_iters;        /* FP32_REFINE: FP64 refinement steps; FP64: 0                */
    double rel_resid;       /* ||b~ - A p||_2 / ||b~||_2 at exit, evaluated in FP64        */
    double b_mean_removed;  /* mean(b), removed for compatibility                         */
    double b_norm;          /* ||b - mean(b)||_2                                          */
    double rho_min, rho_max;
    double err_bound_rel;   /* bound on ||p - p*||_2 / ||p||_2 from the final residual:   */
                            /* rho_max ||r||_2 / min_d(4 sin^2(pi/N_d)/h_d^2) / ||p||_2   */
    double ms;              /* device time of the solve (HIP events on the stream)        */
    int p1_sweeps;          /* launches of the residual sweep P1 that did work: FP64, one
                               per residual evaluation; FP32_REFINE, one per inner
                               evaluation except the first of a refinement step where
                               the outer residual sweep produced it (a step whose end
                               is predicted from the contraction skips the evaluation
                               that would only confirm it)                           */
    double queue_ms;        /* served requests: host time from submit to admission; else 0 */
} poisson_stats;

/* Create a solver for one grid: validates the options, builds the transform
 * tables (twiddles and the discrete Laplacian symbol -4 sin^2(pi k/N)/h^2 per
 * direction) and allocates the workspace (about 8 B/cell for FP64, 24 B/cell
 * for FP32_REFINE).  Returns POISSON_OK and *out, or an error and *out = NULL. */
int poisson_create(const poisson_opts* opts, poisson_t* out);

/* Solve A p = b - mean(b) for the zero-mean p.  p is in/out: on entry the
 * estimate p_g (warm start; zeros are fine), on exit the solution with
 * ||b~ - A p||_2 <= tol * ||b~||_2.  If b is constant, p is set to 0 with no
 * iteration.  On POISSON_EDOMAIN p is untouched; on POISSON_ENOCONV and
 * POISSON_EDIVERGED p holds the last iterate.  Blocks until done. */
int poisson_solve(poisson_t h, const double* rho, const double* b, double* p, double tol);

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops that must not call the allocator, harnesses that forbid it):
 * the solve of poisson_solve without a handle and without any allocation.
 * opts as for poisson_create (use_graphs is ignored; stream: the caller's
 * hipStream_t or NULL, on which the solve runs); rho, b, p and tol as for
 * poisson_solve, with the same result bits.  The tables, the workspace and the
 * state live in one device array of 64 MiB inside the library (each device
 * holds its own copy from the library's load until the process ends); a grid
 * whose tables plus workspace exceed it returns POISSON_ETOOBIG with p
 * untouched (e.g. 128^3 fits in either precision, 192^3 only in POISSON_FP64).
 * The array keeps the last call's contents; every call rewrites what it reads.
 * Calls are serialised by a process-wide lock (a call waits for the one
 * before it, on any device), so calls that would overlap do not race on the
 * array.  *stats (may be NULL) receives the solve's statistics; stats->ms is
 * the host time of the call.  Blocks until done. */
int poisson_solve_noalloc(const poisson_opts* opts, const double* rho, const double* b, double* p, double tol,
                          poisson_stats* stats);

/* Statistics of the last poisson_solve on this handle. */
int poisson_get_stats(poisson_t h, poisson_stats* stats);

/* Residual history of the last solve: hist[k] = ||r_k|| / ||b~|| for
 * k = 0..count-1 (FP64 path: one entry per iteration; FP32_REFINE: one per
 * outer FP64 step).  Writes at most cap entries; returns the count or < 0. */
int poisson_get_history(poisson_t h, double* hist, int cap);

/* Release the handle and its workspace.  NULL is allowed. */
void poisson_destroy(poisson_t h);

/* Text for a status code.  Never NULL. */
const char* poisson_strerror(int code);

/* ---- single sweeps of the hot path, for parity checks and profiling ------
 * Each uses the handle's grid, coef and stream and blocks until done. */

/* out = A p (the operator above).  rho, p, out: device FP64 fields. */
int poisson_apply(poisson_t h, const double* rho, const double* p, double* out);

/* r = (b - mean(b)) - A p, with ||r||_2 and ||b - mean(b)||_2 returned through
 * r_norm and b_norm (host pointers, may be NULL).  r may be NULL. */
int poisson_residual(poisson_t h, const double* rho, const double* b, const double* p, double* r,
                     double* r_norm, double* b_norm);

/* Device time of one sweep kind inside the solves of this handle.  After
 * poisson_kernel_timer(h, sweep, fp32) with sweep 1, 2, 3 or 5 (as in
 * poisson_time_sweep; fp32 != 0 selects the FP32 sweeps of a
 * POISSON_FP32_REFINE handle), every launch of that sweep by poisson_solve is
 * bracketed by two HIP events on the handle's stream (up to 256 launches per
 * solve) and the elapsed times are summed when the solve returns; launches
 * that find their solve finished or out of stage are counted too (compare
 * poisson_stats.p1_sweeps).  sweep 0 stops the timer.  Every call resets the
 * sums. */
int poisson_kernel_timer(poisson_t h, int sweep, int fp32);
/* Summed bracketed time (ms) and bracketed launches since the timer was set. */
int poisson_kernel_timer_read(poisson_t h, double* total_ms, long long* launches);

/* delta = L^+ q: zero-mean solution of L delta = q - mean(q) with L the
 * constant-coefficient 7-point Laplacian, by separable real (Hartley)
 * transforms, which diagonalise it with the discrete symbol above.  This is
 * the inner solve of eq. (Pois).  q and delta are device FP64 fields and may
 * be the same pointer. */
int poisson_lap_pinv(poisson_t h, const double* q, double* delta);

/* The same L^+ q through the FP32 sweeps that a POISSON_FP32_REFINE handle
 * runs inside its refinement steps (q rounded to FP32 as it is loaded, every
 * transform and the symbol division in FP32 with the FP32 tables, delta
 * widened to FP64 at the end), to check those sweeps on their own.  The handle
 * must be POISSON_FP32_REFINE (else POISSON_EINVAL); its FP32 workspace is used
 * as scratch.  q and delta are device FP64 fields and may be the same pointer. */
int poisson_lap_pinv_fp32(poisson_t h, const double* q, double* delta);

/* Average device time of one sweep of the iteration, launched `reps` times
 * back to back between two HIP events on the handle's stream (after one
 * warm-up launch), written to *avg_ms.  sweep: 1 residual + weight + Hartley
 * along x; 2 Hartley along y; 3 Hartley along z, symbol division, Hartley
 * along z; 5 Hartley along x + update; 6 (POISSON_FP32_REFINE handles only)
 * the FP64 outer residual of a refinement step with its FP32 outputs (where
 * the rows allow it, fused with the first inner sweep's residual and its
 * transform along x).
 * fp32 != 0 times the FP32 sweeps of a POISSON_FP32_REFINE handle.  p is used
 * as scratch: its contents are lost. */
int poisson_time_sweep(poisson_t h, int sweep, int fp32, const double* rho, const double* b, double* p, int reps,
                       double* avg_ms);

/* ---- the projection step around the solve ---------------------------------
 * Appendix A, time advance: the momentum predicted without the pressure
 * gradient is divided by the new density, its divergence gives the right-hand
 * side of the variable-coefficient Poisson equation (with the consistency
 * constant chi from its mean), and after the solve the momentum is corrected
 * by the pressure gradient.  Periodic box, or walls in x (POISSON_BC_WALLS_X):
 * then the two x end faces of every row are closed, the momentum stored for
 * the face between the last and the first cell takes no part in the
 * divergence and is not corrected, and p solves the walls problem.
 *
 * Face momentum: mx, my, mz are device FP64 arrays [nz][ny][nx] like the
 * cell fields; m_d[c] is the normal momentum on the face between cell c and
 * its neighbour c + e_d (wrapped).  The face velocity is u = beta m, with
 * beta the handle's face coefficient (the 1/rho_face of the operator), so
 * that the divergence of beta times the face gradient of p is A p. */

/* out_c = sum_d ( beta_{c+1/2} m_d[c] - beta_{c-1/2} m_d[c - e_d] ) / h_d:
 * the divergence of the face velocity.  All pointers device FP64 fields;
 * out must not alias the inputs.  Blocks until done. */
int poisson_divergence(poisson_t h, const double* rho, const double* mx, const double* my, const double* mz,
                       double* out);

/* One pressure projection.  c_dt = C_RK4^pre[k] * dt > 0 of the substep;
 * rhs_div = RHS^div, the divergence the new velocity must have (cell field).
 *   RHS^Pois = ( div(beta m) - RHS^div ) / c_dt
 *   solve A p = RHS^Pois - mean(RHS^Pois) as poisson_solve does (p in/out:
 *     the previous pressure is the estimate p_g; tol as in poisson_solve)
 *   m_d <- m_d - c_dt (p_{c+e_d} - p_c) / h_d     (mx, my, mz in/out)
 * *chi (host pointer, may be NULL) receives chi = -c_dt mean(RHS^Pois), so
 * that afterwards div(beta m) = RHS^div - chi up to c_dt times the solve's
 * residual.  Returns the solve's status; on POISSON_OK and POISSON_ENOCONV the
 * momentum is corrected, on any other status it is untouched (and p is as
 * poisson_solve leaves it for that status).
 * poisson_get_stats describes the solve.  The six fields must not overlap.
 * The first call allocates one cell field of workspace in the handle. */
int poisson_project(poisson_t h, const double* rho, double* mx, double* my, double* mz, const double* rhs_div,
                    double c_dt, double* p, double tol, double* chi);

/* ---- particles and the grid -----------------------------------------------
 * Section "Physical model": the operator P projects particle data to the
 * fluid grid per unit volume, and I interpolates grid data to the particle
 * positions, both by a linear approximation.  Here: trilinear (cloud-in-cell)
 * weights on the cell centres, periodic.  For a particle at x, per direction
 * s = x/h - 1/2, i0 = floor(s), f = s - i0: weight 1 - f to cell i0 and f to
 * cell i0 + 1 (wrapped); the eight cells around it get the products.
 * pos: device FP64 array of n_particles rows (x, y, z) in the box's physical
 * units, any value within 2^30 cells of the box (wrapped).  Periodic handles
 * only (POISSON_BC_WALLS_X gives POISSON_EINVAL); POISSON_EDOMAIN for a
 * position that is not finite or too far out (outputs then undefined). */

/* out = P(q): out_c = sum_p q_p W_p(c) / (hx hy hz).  q: n_particles device
 * values, or NULL for q = 1 (then out is the particle number density).
 * Deterministic (no floating-point atomics: the particles are sorted by cell,
 * and every cell adds its contributions in a fixed order, so repeated calls
 * give the same bits).  Keeps particle buffers in the handle, grown as needed
 * (about 80 B per particle); out must not overlap pos or q.  Blocks until
 * done. */
int poisson_deposit(poisson_t h, int n_particles, const double* pos, const double* q, double* out);

/* out_p = I(field)(x_p): trilinear interpolation of a device FP64 cell field at
 * the particle positions (the adjoint of P up to the factor 1/(hx hy hz)).
 * out: n_particles device values, not overlapping pos or field.  Blocks until
 * done. */
int poisson_interpolate(poisson_t h, int n_particles, const double* pos, const double* field, double* out);

/* ---- serving: many independent solves of different sizes -----------------
 * A server keeps each admitted request's rho, b, p and iteration state on the
 * device, groups requests of equal grid size into batches that advance
 * together (one chunk of batched launches per size class at a time, blockIdx.y
 * selecting the request, each class on a stream of its own, optionally
 * replayed from captured graphs: poisson_server_use_graphs), and admits new
 * requests between ticks as slots and memory free up.  Requests are
 * independent: each result is the same as a solve of that request alone. */
typedef struct poisson_server_s* poisson_server_t;

/* budget_bytes: device memory the server may hold for admitted requests
 * (fields and workspace); max_slots: most requests resident at once;
 * stream: hipStream_t or NULL.  precision/coef/weight/max_iter as above, for
 * every request. */
int poisson_server_create(size_t budget_bytes, int max_slots, int precision, int coef, int weight,
                          int max_iter, void* stream, poisson_server_t* out);

/* Queue a request on grid (nx, ny, nz), box (lx, ly, lz), boundary condition
 * bc_x (POISSON_BC_PERIODIC or POISSON_BC_WALLS_X; requests batch together only
 * with equal grid, box and condition).  rho, b, p: device FP64 fields of the request's grid that
 * the server uses in place: rho and b must stay valid and unchanged, and p
 * must not be touched, until poisson_server_poll reports the request done.  p
 * is in/out like in poisson_solve.  The request's resident footprint (its
 * three fields plus the solver workspace) counts against the budget while it
 * is admitted.  Does not block.  Returns the id through *id.
 * POISSON_ETOOBIG if the request could never fit the budget. */
int poisson_server_submit(poisson_server_t s, int nx, int ny, int nz, double lx, double ly, double lz, int bc_x,
                          const double* rho, const double* b, double* p, double tol, long long* id);

/* Run one scheduling tick: retire the finished requests of every batch whose
 * last chunk of iterations has completed, admit queued requests that fit, and
 * enqueue the next chunk of every idle batch.  Batches of different grid sizes
 * progress independently on their own streams; the tick does not wait for
 * running chunks, so a caller drives the server by calling it in a loop.
 * Returns the number of requests still queued or resident. */
int poisson_server_tick(poisson_server_t s);

/* 0 and *stats filled if the request is done, 1 if still queued or running,
 * < 0 on error.  For a served request stats->ms is the latency from submit to
 * completion (host clock).  A done request's stats stay readable until the
 * server is destroyed.  A server is driven by one host thread. */
int poisson_server_poll(poisson_server_t s, long long id, poisson_stats* stats);

/* on != 0: each size class's chunk of batched launches is captured once per
 * (batch size, chunk length, share of the chip) into a HIP graph and replayed
 * on later ticks (the slot table it reads is rewritten before each replay);
 * 0 (the default): the same kernels are launched directly.  Same results. */
int poisson_server_use_graphs(poisson_server_t s, int on);

/* *bytes = the footprint a request on grid (nx, ny, nz) with boundary
 * condition bc_x holds against this server's budget while it is admitted: its
 * three caller fields (24 B per cell) plus the solver workspace of the server's
 * precision.  A pooled idle workspace of that grid keeps holding the workspace
 * part until a request reuses it or admission releases it.  POISSON_EINVAL for
 * an unsupported size. */
int poisson_server_footprint(poisson_server_t s, int nx, int ny, int nz, int bc_x, size_t* bytes);

void poisson_server_destroy(poisson_server_t s);

#ifdef __cplusplus
}
#endif

#endif /* PAPER_1601_05448_AMD_POISSON_H */
