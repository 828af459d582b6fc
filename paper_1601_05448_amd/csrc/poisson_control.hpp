// Convergence control of the iteration: the decisions taken on the device
// after each residual evaluation, and the fused hand-off that runs them.
//
// A sweep that evaluates a residual writes one set of partial sums per unit of
// work (a z-marching tile or a line group), in the unit's own slot of the
// solve's partial array, so that the sums do not depend on how many blocks the
// launch had (a solve gives the same bits alone and in a batch, whatever share
// of the chip its launches get).  A one-block kernel per solve then adds the
// units' sums in a fixed order and takes the decision.  (Taking it in the
// sweep's last block instead needs a device-scope fence in every block, which
// on this chip writes back the XCD's L2 and costs far more than the launch.)
#pragma once

#include "poisson_device.hpp"

namespace pois {

// FP64 path, after P1 of iteration st->iter.  sums: r^2, bt^2, p, p^2.
__device__ inline void decide_fp64(const GridArgs& g, SolveState* st, const double* sums) {
    st->p1_work += 1;  // runs exactly when P1 did its work
    const int k = st->iter;
    st->p_sum = sums[2];
    st->p_sumsq = sums[3];
    // the update of this iteration also removes the mean of p (the zero-mean
    // gauge), so rounding in dp never accumulates a constant
    st->p_shift = sums[2] / (double)g.n;
    if (k == 0) {
        st->b_norm = sqrt(sums[1]);
        if (st->b_norm == 0.0) {
            st->rel = 0.0;
            st->r_norm = 0.0;
            st->hist[0] = 0.0;
            st->done = 1;
            st->status = POISSON_OK;
            return;
        }
    }
    const double rn = sqrt(sums[0]);
    const double rel = rn / st->b_norm;
    st->r_norm = rn;
    st->rel = rel;
    if (k == 0) st->rel0 = rel;
    if (k < kHistCap) st->hist[k] = rel;
    if (rel <= st->tol) {
        st->done = 1;
        st->status = POISSON_OK;
    } else if (!(rel < 1e8)) {
        st->done = 1;
        st->status = POISSON_EDIVERGED;
    } else if (k >= st->max_iter) {
        st->done = 1;
        st->status = POISSON_ENOCONV;
    } else {
        st->iter = k + 1;
    }
}

// FP32_REFINE, after the FP64 outer residual of outer step st->iter.  sums: r^2,
// bt^2, p, p^2, r.  fused: the sweep also produced the first inner sweep's
// transformed residual, whose evaluation (rel 1 against the step's own right-
// hand side) is taken here; the rest of that sweep is due next (kStageTail).
// check: the sweep wrote nothing but its sums; a solve it does not end stays in
// stage 0 for an outer residual that starts the step (the same sums again).
__device__ inline void decide_outer(const GridArgs& g, SolveState* st, const double* sums, bool fused,
                                    bool check = false) {
    const int m = st->iter;
    st->checked = check ? 1 : 0;
    st->p_sum = sums[2];
    st->p_sumsq = sums[3];
    if (m == 0) {
        // the mean of the incoming p, removed by the update of step 0
        st->p_shift = sums[2] / (double)g.n;
        st->b_norm = sqrt(sums[1]);
        if (st->b_norm == 0.0) {
            st->rel = 0.0;
            st->r_norm = 0.0;
            st->hist[0] = 0.0;
            st->done = 1;
            st->status = POISSON_OK;
            return;
        }
    }
    const double rn = sqrt(sums[0]);
    const double rel = rn / st->b_norm;
    st->r_norm = rn;
    st->rel = rel;
    if (m < kHistCap) st->hist[m] = rel;
    if (rel <= st->tol) {
        st->done = 1;
        st->status = POISSON_OK;
    } else if (!(rel < 1e8)) {
        st->done = 1;
        st->status = POISSON_EDIVERGED;
    } else if (m >= st->max_outer || st->inner_total >= st->max_iter) {
        st->done = 1;
        st->status = POISSON_ENOCONV;
    } else if (!check) {
        st->rhs_mean32 = sums[4] * st->inv_s / (double)g.n;
        // The update leaves an outer residual of rel times the inner relative
        // residual (up to the FP32 operator's rounding, about 1e-6 of it), so
        // a step needs no more than tol / rel from its inner sweeps; with a
        // margin of 20% the last step of a solve, and a step that starts close
        // to the tolerance as after a warm start, stops as soon as that is
        // reached instead of running to the inner tolerance.
        st->inner_goal = fmax(st->inner_tol, 0.8 * st->tol / rel);
        st->stage = 1;
        st->inner_iter = 0;
        st->inner_done = 0;
        st->stop_next = 0;
        st->upd_due = 0;
        st->since_best = 0;
        st->best_in = INFINITY;
        st->rel_in = 1.0;
        if (fused) {
            // inner evaluation 0: ||r32 - mean|| from the FP64 sums, rel 1; not
            // a stop (inner_total < max_iter here), so its update follows
            const double n = (double)g.n;
            st->rhs_norm32 = st->inv_s * sqrt(fmax(sums[0] - sums[4] * sums[4] / n, 0.0));
            st->best_in = 1.0;
            st->inner_iter = 1;
            st->inner_total += 1;
            st->stage = kStageTail;
        }
    }
}

// FP32_REFINE, after the FP32 P1 of an inner iteration.  sums: r^2, bt^2.
__device__ inline void decide_inner(SolveState* st, const double* sums, int max_inner) {
    const int t = st->inner_iter;
    if (st->stop_next) {
        // the previous iteration was predicted to be the phase's last: its
        // update has been applied and this iteration's P1 idled
        st->stop_next = 0;
        st->inner_done = 1;
        st->inner_last = t + 1;
        st->stage = 2;
        return;
    }
    st->p1_work += 1;  // P1 did its work
    if (t == 0) st->rhs_norm32 = sqrt(sums[1]);
    const double rel = (st->rhs_norm32 > 0.0) ? sqrt(sums[0]) / st->rhs_norm32 : 0.0;
    const double prev = st->rel_in;  // the previous evaluation of this phase (1 before any)
    st->rel_in = rel;
    bool stop = false;
    if (!(rel < 1e8)) stop = true;  // non-finite or blown up: let the FP64 step judge
    if (rel <= st->inner_goal) stop = true;
    if (rel < 0.9 * st->best_in) {
        st->best_in = rel;
        st->since_best = 0;
    } else {
        ++st->since_best;
    }
    // Stagnation at the FP32 rounding floor: no 10% gain in 8 sweeps after the
    // residual has come down.  The iteration can first grow by orders of
    // magnitude on rough density before it contracts, so no stop counts before
    // the best residual is below half its start.
    if (st->best_in < 0.5 && st->since_best >= 8) stop = true;
    if (t >= max_inner || st->inner_total >= st->max_iter) stop = true;
    if (stop) {
        st->inner_done = 1;
        st->inner_last = t + 1;
        st->stage = 2;
    } else {
        st->inner_iter = t + 1;
        st->inner_total += 1;
        st->upd_due = 1;  // this evaluation's update comes next
        // Predicted stop: the sweeps contract the inner residual at a steady
        // rate, so when the contraction since the previous evaluation brings
        // the residual after this iteration's update below half the goal, the
        // phase ends after that update and the residual sweep that would only
        // confirm it is not run (the FP64 outer residual that follows measures
        // the step anyway; a step that falls short costs another step).
        if (t >= 1 && prev > 0.0 && rel < prev && t + 1 < max_inner && st->inner_total < st->max_iter) {
            const double next = rel * (rel / prev);
            if (next <= 0.5 * st->inner_goal) {
                st->stop_next = 1;
                st->rel_in = next;  // what the step is expected to reach (the host's estimate of its reduction)
            }
        }
    }
}

}  // namespace pois
