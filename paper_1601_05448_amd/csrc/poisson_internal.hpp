// Internal structures shared by the kernels and the host engine of libpoisson.
// Nothing here is part of the C ABI (include/poisson.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pois {

constexpr int kHistCap = 256;      // residual-history entries kept per solve
constexpr int kPartialStride = 8;  // doubles per set of partial sums (one set per block or per unit of work)
constexpr int kMaxSetupBlocks = 4096;
constexpr int kStageTail = 3;  // see SolveState::stage
constexpr int kMaxInnerPerStep = 1 << 20;  // FP32 inner sweeps per refinement step: bounded by max_iter

// Grid description passed by value to every kernel.  Uniform over a batch:
// all solves of one launch share the grid.
struct GridArgs {
    int nx, ny, nz;
    int nxh;           // nx / 2 (complex columns of a row pair view)
    long long n;       // cells
    double ihx2, ihy2, ihz2;  // 1 / h_d^2
    int coef;          // face-coefficient mode
    int weight;        // residual multiplier mode
    int bcx;           // 0 periodic in x; 1 zero-flux walls at both ends of x
};

// Per-solve state, resident in device memory.  Written only by the one-block
// finalize kernels (and zeroed by the init kernel); every sweep kernel reads
// `done` first and returns at once when the solve is over, so that unrolled
// iteration sequences stop doing work after convergence.
struct SolveState {
    // parameters (init kernel)
    double tol;
    double inner_tol;
    double inner_goal;  // inner stop of the current refinement step (decide_outer)
    int max_iter;
    int max_outer;
    int precision;
    int pad0;
    // setup results
    double b_mean;
    double b_sumsq;     // sum b^2 (for the FP32 scale only)
    double rho_min, rho_max;
    int bad;            // non-finite or non-positive input seen
    // outer (FP64) iteration
    int iter;           // FP64 path: current iteration; FP32 path: current outer step
    int done;           // solve finished (any status)
    int status;         // POISSON_* code
    double b_norm;      // ||b - mean b||
    double r_norm;      // last FP64 residual norm
    double rel;         // last relative residual
    double rel0;        // relative residual of the first FP64 evaluation
    double p_shift;     // mean of the incoming p, removed by the first update
    double p_sum;       // sum p and sum p^2 of the last iterate whose residual was taken
    double p_sumsq;
    int p_fixed;        // p_shift already removed
    // FP32 inner iteration.  stage: 0 the next FP64 outer residual is due, 1 inner
    // FP32 sweeps run, 2 the FP64 update is due, 3 (kStageTail) the rest of the
    // first inner sweep is due after an outer residual that also produced that
    // sweep's transformed weighted residual; each kernel acts only on the solves
    // in its stage, so solves at different stages share one launch sequence
    int stage;
    int inner_iter;     // inner iteration within the current outer step
    int inner_done;
    int inner_total;
    int inner_last;     // inner-sweep launches the last finished outer step used
    int p1_work;        // launches of the residual sweep P1 that did their work
    int since_best;
    int stop_next;      // the inner phase ends after the update of the iteration in progress:
                        // the next inner residual sweep idles and its decision closes the phase
    int upd_due;        // the last inner evaluation went on with the phase and its update (the
                        // y, z, y and x sweeps) has not run yet: the next inner residual sweep
                        // and its decision idle until it has (the x sweep clears it)
    int checked;        // the last outer residual was a check (sums alone) that did not end the
                        // solve: `rel` is the residual of the current p, no update is pending
    double inv_s;       // r32 = r * inv_s (a power of two)
    double rhs_mean32;  // mean of r32, removed inside the inner sweeps
    double rhs_norm32;  // ||r32 - mean||
    double rel_in;
    double best_in;
    double hist[kHistCap];
};

// Per-solve device pointers (a batch launch indexes these by blockIdx.y).
struct Slot {
    double tol;       // relative-residual target of this solve
    const double* rho;
    const double* b;
    double* p;
    double* W;        // FP64 spectral workspace, n values
    float* rho32;     // FP32 copies / workspace (FP32_REFINE only)
    float* r32;
    float* d32;
    float* W32;
    double* partial;  // partial sums: kPartialStride doubles per block or per tile / line group
    SolveState* st;
};

// Device tables for one grid, shared by every solve of that grid.
struct Tables {
    const double2* twx; const double2* twy; const double2* twz;  // exp(-2 pi i t/N), FP64
    const float2* twx32; const float2* twy32; const float2* twz32;
    // symbols: -4 sin^2(pi k/N)/h^2; along x between walls -4 sin^2(pi k/(2N))/h^2
    const double* lamx; const double* lamy; const double* lamz;
    const float* lamx32; const float* lamy32; const float* lamz32;
    // walls in x: exp(-i pi k/(2 Nx)), the twiddles of the cosine transform
    const double2* twcx; const float2* twcx32;
};

// Launch geometry of the sweeps of one grid (host side).
struct Geometry {
    int blocks_x;      // row-pair line groups of the x sweep (most blocks P1 can use)
    int blocks_pt;     // pointwise kernels
    int blocks_outer;  // FP64 outer residual
    int max_blocks;    // capacity of the partial-sum array, in sets
    float share;       // fraction of the chip's resident blocks the persistent sweeps take
};

// ---- launchers (poisson_kernels.hip) ----------------------------------------
// Every launcher enqueues on `stream` for `nslots` solves described by the
// device array `slots`.  They return hipSuccess or the launch error.
Geometry make_geometry(const GridArgs& g);
bool length_supported(int n);

// Initialises the state of each slot (tolerance from Slot::tol).
hipError_t launch_init(const GridArgs& g, const Slot* slots, int nslots, double inner_tol, int max_iter,
                       int max_outer, int precision, hipStream_t s);
hipError_t launch_setup(const GridArgs& g, const Geometry& geo, const Slot* slots, int nslots,
                        bool write_rho32, hipStream_t s);
hipError_t launch_setup_finalize(const GridArgs& g, const Geometry& geo, const Slot* slots, int nslots,
                                 hipStream_t s);
// One iteration of the paper's method on all slots (FP64 fields) or one inner
// iteration (FP32 fields).
// HIP events around the launches of one sweep kind inside solves (sweep 0: off);
// the host reads the `used` pairs after the solve and resets `used`.
struct SweepTimer {
    static constexpr int kCap = 256;
    int sweep = 0;
    bool fp32 = false;
    int used = 0;
    hipEvent_t ev[2 * kCap] = {};
};
hipError_t launch_iteration(const GridArgs& g, const Geometry& geo, const Tables& t, const Slot* slots,
                            int nslots, bool fp32, hipStream_t s, SweepTimer* tm = nullptr);
// FP32_REFINE inner iterations in halves: the residual sweep and its decision
// (an evaluation), and the four transform sweeps that apply its update; a
// launch sequence may end on an evaluation and the next start with its update
// (SolveState::upd_due keeps the order).
hipError_t launch_evaluation(const GridArgs& g, const Geometry& geo, const Tables& t, const Slot* slots,
                             int nslots, hipStream_t s, SweepTimer* tm = nullptr);
hipError_t launch_inner_update(const GridArgs& g, const Geometry& geo, const Tables& t, const Slot* slots,
                               int nslots, hipStream_t s, SweepTimer* tm = nullptr);
// One sweep alone (1: P1, 2: P2 and P4, 3: P3, 5: P5), for timing.
hipError_t launch_sweep(const GridArgs& g, const Tables& t, const Slot* slots, int nslots, bool fp32, int which,
                        hipStream_t s);
// poisson_sweeps.hip: one sweep; mode 0 iteration, mode 1 the stand-alone L^+ q
// sweep (FP64).  *nunits (may be NULL) receives the number of partial sums P1
// wrote.  `share`: fraction of the resident blocks the persistent sweeps take.
hipError_t launch_sweep_mode(const GridArgs& g, const Tables& t, const Slot* slots, int nslots, bool fp32, int which,
                             int mode, hipStream_t s, int* nunits, float share = 1.0f, int stage = 1);
unsigned sweep_groups_x(const GridArgs& g);
// FP32_REFINE: whether rows of this length take the outer residual fused with
// the first inner sweep's residual (one marching column per thread), and that
// sweep alone (no decision); *nunits receives the number of partial sums.
// write = false: the partial sums alone (no r32, no transformed residual).
bool outer_fusable(const GridArgs& g);
hipError_t launch_outer_fused(const GridArgs& g, const Tables& t, const Slot* slots, int nslots, hipStream_t s,
                              int* nunits, float share = 1.0f, bool write = true);
// FP32_REFINE outer step pieces.
// the FP64 outer residual sweep alone (no decision); *nunits (may be NULL)
// receives the number of partial sums it wrote
hipError_t launch_outer_resid_sweep(const GridArgs& g, const Slot* slots, int nslots, hipStream_t s, int* nunits);
// The FP64 outer residual of a refinement step and its decision; where the
// rows allow (*fused), fused with the first inner sweep's residual and, with
// `tail`, followed by the rest of that sweep.  Without `tail` (the final check
// of a solve) fused rows take the residual's sums alone: a solve it does not
// end stays in stage 0, and its next outer residual starts the step.
hipError_t launch_outer_residual(const GridArgs& g, const Geometry& geo, const Tables& t, const Slot* slots,
                                 int nslots, hipStream_t s, bool* fused, bool tail = true);
hipError_t launch_outer_tail(const GridArgs& g, const Geometry& geo, const Tables& t, const Slot* slots,
                             int nslots, hipStream_t s);
hipError_t launch_outer_update(const GridArgs& g, const Geometry& geo, const Slot* slots, int nslots,
                               hipStream_t s);
hipError_t launch_fixup(const GridArgs& g, const Geometry& geo, const Slot* slots, int nslots, hipStream_t s);
// Marks every slot whose solve is not done as done with POISSON_ENOCONV.
hipError_t launch_stop_unfinished(const Slot* slots, int nslots, hipStream_t s);

// Single sweeps for parity checks (one slot).
hipError_t launch_apply(const GridArgs& g, const Geometry& geo, const double* rho, const double* p, double* out,
                        hipStream_t s);
hipError_t launch_residual(const GridArgs& g, const Geometry& geo, const Slot* slot, double* r,
                           hipStream_t s);
// delta (slot.p) = L^+ q (slot.b); fp32: through the FP32 sweeps (q rounded
// to FP32 on load, the result widened from d32 at the end).
hipError_t launch_lap_pinv(const GridArgs& g, const Geometry& geo, const Tables& t, const Slot* slot,
                           hipStream_t s, bool fp32 = false);

// The projection step around the solve (poisson_project.hip): out = div(beta m)
// (rhs == nullptr) or (div(beta m) - rhs) / c_dt; m_d -= c_dt grad_d p.
hipError_t launch_divergence(const GridArgs& g, const double* rho, const double* mx, const double* my,
                             const double* mz, const double* rhs, double c_dt, double* out, hipStream_t s);
hipError_t launch_correct(const GridArgs& g, const double* p, double* mx, double* my, double* mz, double c_dt,
                          hipStream_t s);

// Particles and the grid (poisson_particles.hip): out = P(q) per unit volume
// (ws: particle_workspace_bytes(g, np) bytes of device scratch; the grid is
// zeroed on s_aux between the two events while the sort runs on s), out_p =
// I(field)(x_p).  *bad_host = 1 when a position is not finite or too far out
// (then nothing else is written).
size_t particle_workspace_bytes(const GridArgs& g, int np);
hipError_t launch_deposit(const GridArgs& g, int np, const double* pos, const double* q, double* out, void* ws,
                          size_t ws_bytes, int* bad_host, hipStream_t s, hipStream_t s_aux, hipEvent_t ev_fork,
                          hipEvent_t ev_join);
hipError_t launch_interpolate(const GridArgs& g, int np, const double* pos, const double* field, double* out,
                              int* bad_dev, int* bad_host, hipStream_t s);

}  // namespace pois
