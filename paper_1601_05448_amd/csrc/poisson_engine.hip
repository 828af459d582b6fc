// Host engine and C ABI of libpoisson (declarations and semantics in
// include/poisson.h).
//
// poisson_create builds, per grid, the tables of the separable Hartley
// transforms (twiddles exp(-2 pi i t/N) and the discrete symbol of the 1-D
// periodic second difference, -4 sin^2(pi k/N)/h^2, both in FP64 from host
// libm) and the workspace.  poisson_solve drives the iteration of the paper
// (section "Poisson equation", eq. (Pois)) on the device; the host only waits
// for chunks of iterations and reads back a small state record.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/poisson.h"
#include "poisson_engine.hpp"
#include "poisson_internal.hpp"

using namespace pois;

namespace pois {

static const double kPi = 3.14159265358979323846264338327950288;

int hip_status(hipError_t e) { return e == hipSuccess ? POISSON_OK : POISSON_EHIP; }

bool valid_lengths(double lx, double ly, double lz) {
    return std::isfinite(lx) && std::isfinite(ly) && std::isfinite(lz) && lx > 0 && ly > 0 && lz > 0;
}

GridArgs make_grid(int nx, int ny, int nz, double lx, double ly, double lz, int coef, int weight, int bcx) {
    GridArgs g{};
    g.nx = nx; g.ny = ny; g.nz = nz;
    g.nxh = nx / 2;
    g.n = (long long)nx * ny * nz;
    const double hx = lx / nx, hy = ly / ny, hz = lz / nz;
    g.ihx2 = 1.0 / (hx * hx);
    g.ihy2 = 1.0 / (hy * hy);
    g.ihz2 = 1.0 / (hz * hz);
    g.coef = coef;
    g.weight = weight;
    g.bcx = bcx;
    return g;
}

// Smallest nonzero eigenvalue magnitude of -L: min_d 4 sin^2(pi/N_d)/h_d^2, with
// 4 sin^2(pi/(2 Nx))/hx^2 along x between walls.
double min_symbol(const GridArgs& g) {
    auto one = [](double arg, double ih2) {
        const double s = std::sin(arg);
        return 4.0 * s * s * ih2;
    };
    const double ax = g.bcx ? kPi / (2.0 * g.nx) : kPi / g.nx;
    return std::min(one(ax, g.ihx2), std::min(one(kPi / g.ny, g.ihy2), one(kPi / g.nz, g.ihz2)));
}

// ---- per-grid tables ---------------------------------------------------------------

// Layout of one grid's tables in one buffer: four 256-byte aligned arrays per
// direction and the cosine transform's twiddles along x.
struct TableLayout {
    size_t at[3][4];
    size_t at_c, at_c32;
    size_t total;
};

static TableLayout table_layout(const GridArgs& g) {
    const int ns[3] = {g.nx, g.ny, g.nz};
    TableLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        const size_t at = off;
        off += bytes;
        return at;
    };
    for (int d = 0; d < 3; ++d) {
        L.at[d][0] = take((size_t)ns[d] * 16);  // FP64 twiddles
        L.at[d][1] = take((size_t)ns[d] * 8);   // FP32 twiddles
        L.at[d][2] = take((size_t)ns[d] * 8);   // FP64 symbol
        L.at[d][3] = take((size_t)ns[d] * 4);   // FP32 symbol
    }
    L.at_c = take((size_t)g.nx * 16);
    L.at_c32 = take((size_t)g.nx * 8);
    L.total = (off + 255) & ~(size_t)255;
    return L;
}

size_t tables_bytes(const GridArgs& g) { return table_layout(g).total; }

void fill_tables(const GridArgs& g, unsigned char* host) {
    const TableLayout L = table_layout(g);
    const int ns[3] = {g.nx, g.ny, g.nz};
    const double ih2[3] = {g.ihx2, g.ihy2, g.ihz2};
    std::memset(host, 0, L.total);
    for (int d = 0; d < 3; ++d) {
        const int n = ns[d];
        double* tw = reinterpret_cast<double*>(host + L.at[d][0]);
        float* tw32 = reinterpret_cast<float*>(host + L.at[d][1]);
        double* lam = reinterpret_cast<double*>(host + L.at[d][2]);
        float* lam32 = reinterpret_cast<float*>(host + L.at[d][3]);
        const bool wall = d == 0 && g.bcx == 1;
        for (int t = 0; t < n; ++t) {
            const double ang = 2.0 * kPi * (double)t / (double)n;
            tw[2 * t] = std::cos(ang);
            tw[2 * t + 1] = -std::sin(ang);
            tw32[2 * t] = (float)tw[2 * t];
            tw32[2 * t + 1] = (float)tw[2 * t + 1];
            const double s = std::sin(kPi * (double)t / (wall ? 2.0 * n : (double)n));
            lam[t] = -4.0 * s * s * ih2[d];
            lam32[t] = (float)lam[t];
        }
    }
    double* c = reinterpret_cast<double*>(host + L.at_c);
    float* c32 = reinterpret_cast<float*>(host + L.at_c32);
    for (int t = 0; t < g.nx; ++t) {
        const double ang = kPi * (double)t / (2.0 * g.nx);
        c[2 * t] = std::cos(ang);
        c[2 * t + 1] = -std::sin(ang);
        c32[2 * t] = (float)c[2 * t];
        c32[2 * t + 1] = (float)c[2 * t + 1];
    }
}

Tables bind_tables(const GridArgs& g, const void* dev) {
    const TableLayout L = table_layout(g);
    const unsigned char* base = static_cast<const unsigned char*>(dev);
    auto ptr = [&](int d, int k) { return static_cast<const void*>(base + L.at[d][k]); };
    Tables t{};
    t.twx = static_cast<const double2*>(ptr(0, 0)); t.twy = static_cast<const double2*>(ptr(1, 0));
    t.twz = static_cast<const double2*>(ptr(2, 0));
    t.twx32 = static_cast<const float2*>(ptr(0, 1)); t.twy32 = static_cast<const float2*>(ptr(1, 1));
    t.twz32 = static_cast<const float2*>(ptr(2, 1));
    t.lamx = static_cast<const double*>(ptr(0, 2)); t.lamy = static_cast<const double*>(ptr(1, 2));
    t.lamz = static_cast<const double*>(ptr(2, 2));
    t.lamx32 = static_cast<const float*>(ptr(0, 3)); t.lamy32 = static_cast<const float*>(ptr(1, 3));
    t.lamz32 = static_cast<const float*>(ptr(2, 3));
    t.twcx = reinterpret_cast<const double2*>(base + L.at_c);
    t.twcx32 = reinterpret_cast<const float2*>(base + L.at_c32);
    return t;
}

int GridTables::build(const GridArgs& g) {
    const size_t total = tables_bytes(g);
    if (hipMalloc(&mem, total) != hipSuccess) {
        mem = nullptr;
        return POISSON_ENOMEM;
    }
    std::vector<unsigned char> host(total, 0);
    fill_tables(g, host.data());
    if (hipMemcpy(mem, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) return POISSON_EHIP;
    t = bind_tables(g, mem);
    return POISSON_OK;
}

void GridTables::release() {
    if (mem) (void)hipFree(mem);
    mem = nullptr;
}

// ---- per-solve workspace -------------------------------------------------------------

size_t workspace_bytes(const GridArgs& g, const Geometry& geo, int precision) {
    size_t b = (size_t)g.n * 8 + 256;                        // W
    if (precision == POISSON_FP32_REFINE) b += 4 * ((size_t)g.n * 4 + 256);
    b += (size_t)geo.max_blocks * kPartialStride * 8 + 256;  // partial sums
    b += sizeof(SolveState) + 256;
    return b;
}

int Workspace::allocate(const GridArgs& g, const Geometry& geo, int precision) {
    bytes = workspace_bytes(g, geo, precision);
    if (hipMalloc(&mem, bytes) != hipSuccess) {
        mem = nullptr;
        return POISSON_ENOMEM;
    }
    carve(g, geo, precision, mem);
    return POISSON_OK;
}

void Workspace::carve(const GridArgs& g, const Geometry& geo, int precision, void* at_mem) {
    unsigned char* base = static_cast<unsigned char*>(at_mem);
    size_t off = 0;
    auto take = [&](size_t n) {
        off = (off + 255) & ~(size_t)255;
        unsigned char* at = base + off;
        off += n;
        return at;
    };
    W = reinterpret_cast<double*>(take((size_t)g.n * 8));
    rho32 = r32 = d32 = W32 = nullptr;
    if (precision == POISSON_FP32_REFINE) {
        rho32 = reinterpret_cast<float*>(take((size_t)g.n * 4));
        r32 = reinterpret_cast<float*>(take((size_t)g.n * 4));
        d32 = reinterpret_cast<float*>(take((size_t)g.n * 4));
        W32 = reinterpret_cast<float*>(take((size_t)g.n * 4));
    }
    partial = reinterpret_cast<double*>(take((size_t)geo.max_blocks * kPartialStride * 8));
    st = reinterpret_cast<SolveState*>(take(sizeof(SolveState)));
}

void Workspace::release() {
    if (mem) (void)hipFree(mem);
    mem = nullptr;
}

Slot Workspace::slot(const double* rho, const double* b, double* p, double tol) const {
    Slot s{};
    s.tol = tol;
    s.rho = rho; s.b = b; s.p = p;
    s.W = W; s.rho32 = rho32; s.r32 = r32; s.d32 = d32; s.W32 = W32;
    s.partial = partial; s.st = st;
    return s;
}

// ---- the solve driver -----------------------------------------------------------------

// n values of T, on the stack for small batches (a single solve allocates
// nothing on the host), on the heap for large ones.
template <class T>
struct SmallArray {
    static constexpr int kLocal = 64;
    T local[kLocal];
    std::vector<T> heap;
    T* v;
    SmallArray(int n, T init) : v(local) {
        if (n > kLocal) {
            heap.assign((size_t)n, init);
            v = heap.data();
        } else {
            for (int q = 0; q < n; ++q) local[q] = init;
        }
    }
    T& operator[](int q) { return v[q]; }
};

// Enqueue the whole solve for the slots on the stream, reading back the state
// header of slot 0..nslots-1 between chunks.  `hdr` is pinned host memory for
// nslots state headers.
int drive_solve(const GridArgs& g, const Geometry& geo, const Tables& t, const Slot* d_slots, int nslots,
                SolveState* const* d_states, SolveState* hdr, const SolveParams& prm, hipStream_t s,
                SweepTimer* tm, GraphCache* gc) {
    hipError_t e;
    // n iterations: replayed graphs of 16, 8, 4, 2, 1 iterations when a graph
    // cache is given (and no timer brackets single launches), else direct launches
    auto iterations = [&](int n, bool f32) -> hipError_t {
        if (!gc || tm) {
            for (int c = 0; c < n; ++c) {
                const hipError_t le = launch_iteration(g, geo, t, d_slots, nslots, f32, s, tm);
                if (le != hipSuccess) return le;
            }
            return hipSuccess;
        }
        for (int b = 4; b >= 0; --b) {
            for (; n >= (1 << b); n -= (1 << b)) {
                const hipError_t le = gc->run((f32 ? 16 : 0) + b, s, [&]() -> hipError_t {
                    for (int c = 0; c < (1 << b); ++c) {
                        const hipError_t ie = launch_iteration(g, geo, t, d_slots, nslots, f32, s, nullptr);
                        if (ie != hipSuccess) return ie;
                    }
                    return hipSuccess;
                });
                if (le != hipSuccess) return le;
            }
        }
        return hipSuccess;
    };
    const bool fp32 = prm.precision == POISSON_FP32_REFINE;
    if ((e = launch_init(g, d_slots, nslots, prm.inner_tol, prm.max_iter, prm.max_outer, prm.precision, s)) !=
        hipSuccess)
        return hip_status(e);
    if ((e = launch_setup(g, geo, d_slots, nslots, fp32, s)) != hipSuccess) return hip_status(e);
    if ((e = launch_setup_finalize(g, geo, d_slots, nslots, s)) != hipSuccess) return hip_status(e);
    const size_t hb = offsetof(SolveState, hist);
    bool all_done = false;
    auto poll = [&]() -> int {  // 1: all done, 0: not yet, <0 error
        for (int q = 0; q < nslots; ++q)
            if ((e = hipMemcpyAsync(&hdr[q], d_states[q], hb, hipMemcpyDeviceToHost, s)) != hipSuccess)
                return hip_status(e);
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_status(e);
        for (int q = 0; q < nslots; ++q) {
            if (!hdr[q].done) return 0;
        }
        all_done = true;
        return 1;
    };
    if (!fp32) {
        // Chunks of iterations between polls.  After the first chunk the next
        // one is sized from the contraction observed so far: the iterations
        // that bring the last residual below the tolerance at that rate, plus a
        // quarter of one (an idle launch costs less than another poll).
        int launched = 0, chunk = prm.first_chunk;
        const int cap = prm.max_iter + 1;
        SmallArray<int> k_prev(nslots, -1);
        SmallArray<double> r_prev(nslots, 0.0);
        while (true) {
            const int now = std::min(chunk, cap - launched);
            if ((e = iterations(now, false)) != hipSuccess) return hip_status(e);
            launched += now;
            const int r = poll();
            if (r < 0) return r;
            if (r == 1 || launched >= cap) break;
            int need = 0;
            for (int q = 0; q < nslots; ++q) {
                const SolveState& h = hdr[q];
                if (h.done) continue;
                const int k = h.iter - 1;  // index of the last residual evaluated
                double rate = 1.0;
                if (k_prev[q] >= 0 && k > k_prev[q] && r_prev[q] > 0.0)
                    rate = std::pow(h.rel / r_prev[q], 1.0 / (k - k_prev[q]));
                else if (k >= 1 && h.rel0 > 0.0)
                    rate = std::pow(h.rel / h.rel0, 1.0 / k);
                k_prev[q] = k;
                r_prev[q] = h.rel;
                int m = 2 * chunk;
                if (rate > 0.0 && rate < 0.95 && h.rel > 0.0)
                    m = (int)std::ceil(std::log(h.tol / h.rel) / std::log(rate) + 0.25);
                need = std::max(need, m);
            }
            chunk = std::clamp(need, 1, prm.max_chunk);
        }
    } else {
        // Speculative rounds of refinement steps between host polls.  Every
        // kernel runs only in its stage of the device state, so inner sweeps
        // launched after the inner phase stopped idle, and an update or outer
        // residual launched before the phase stopped idles until a later round.
        // Each round moves every unfinished solve on by at least one stage, so
        // the count of rounds is bounded.  Where the outer residual is fused
        // with the first inner sweep (and followed by the rest of it), a step
        // needs one full sweep less.
        const int first = outer_fusable(g) ? 1 : 0;
        // sweeps of the first step: a contraction of 0.1 per sweep (the method
        // on smooth densities: 0.05 on the 256^3 lognormal density of ratio 4),
        // plus the one whose residual evaluation stops the sweeps; rougher
        // densities take another round
        const int guess = (int)std::ceil(std::log(prm.inner_tol) / std::log(0.1)) + 1;
        int full = std::clamp(guess - first, 0, prm.max_chunk);
        // n inner sweeps that end on an evaluation: n - 1 full sweeps, then the
        // residual sweep and decision of the n-th.  The sweep whose evaluation
        // stops the phase needs no update, so when the guess is right no
        // transform sweep idles; when the phase goes on, the update of that
        // evaluation opens the next round (SolveState::upd_due holds the
        // residual sweeps back until it has run).
        auto sweeps_to_evaluation = [&](int n) -> hipError_t {
            if (n <= 0) return hipSuccess;
            hipError_t le = iterations(n - 1, true);
            if (le == hipSuccess) le = launch_evaluation(g, geo, t, d_slots, nslots, s, tm);
            return le;
        };
        // A refinement step: outer residual (with the tail of its first inner
        // sweep where fused), `nfull` inner sweeps ending on an evaluation, update.
        auto step = [&](int nfull) -> hipError_t {
            hipError_t le = launch_outer_residual(g, geo, t, d_slots, nslots, s, nullptr);
            if (le == hipSuccess) le = sweeps_to_evaluation(nfull);
            if (le == hipSuccess) le = launch_outer_update(g, geo, d_slots, nslots, s);
            return le;
        };
        int open_full = 0;  // evaluations that finish an open inner phase (then its update)
        bool open_tail = false;    // an open phase's first sweep still needs its transforms
        bool open_update = false;  // an open phase's last evaluation still needs its update
        int steps = 1;      // whole steps after that, then one outer residual to check
        int full_last = full;  // inner sweeps of the last of those steps
        bool check = false;
        const int max_rounds = prm.max_outer + prm.max_iter + 2;
        for (int round = 0; round < max_rounds; ++round) {
            if (open_tail && (e = launch_outer_tail(g, geo, t, d_slots, nslots, s)) != hipSuccess)
                return hip_status(e);
            if (open_update && (e = launch_inner_update(g, geo, t, d_slots, nslots, s, tm)) != hipSuccess)
                return hip_status(e);
            if (open_full > 0) {
                if ((e = sweeps_to_evaluation(open_full)) != hipSuccess) return hip_status(e);
                if ((e = launch_outer_update(g, geo, d_slots, nslots, s)) != hipSuccess) return hip_status(e);
            }
            for (int k = 0; k < steps; ++k)
                if ((e = step(k + 1 == steps ? full_last : full)) != hipSuccess) return hip_status(e);
            // the check: the outer residual's sums alone (on rows that take the
            // fused sweep); a solve it does not end starts its next step with
            // a full outer residual in the next round
            if (check && (e = launch_outer_residual(g, geo, t, d_slots, nslots, s, nullptr, false)) != hipSuccess)
                return hip_status(e);
            const int r = poll();
            if (r < 0) return r;
            if (r == 1) break;
            // What the next round enqueues, from the state now:
            //  * a solve inside its inner sweeps: the full sweeps that bring its
            //    inner residual to the inner tolerance at the contraction it has
            //    shown (twice the last count when it has shown none), then its
            //    update;
            //  * then as many whole steps as the outer residual needs to pass the
            //    tolerance if every step reduces it as the last one did (the
            //    inner tolerance for a step still open), each with as many full
            //    sweeps as the last finished step used (the last of them as many
            //    as its smaller inner goal, max(inner tol, 0.8 tol / rel), needs
            //    at the contraction per sweep of the last finished step), and the
            //    outer residual that checks the result.
            // Kernels out of their stage idle, so a short guess costs another
            // round and a long one a few idle launches.
            int need_open = 0, need_full = 0, need_steps = 0, need_last = 0;
            bool need_tail = false, need_update = false;
            for (int q = 0; q < nslots; ++q) {
                const SolveState& h = hdr[q];
                if (h.done) continue;
                double red = h.rel_in;  // outer reduction per step
                double rel = h.rel;     // outer residual before the next outer evaluation
                if (h.stage == kStageTail) {
                    // a step's first sweep still open (not left by the launch
                    // sequences above, which follow every fused outer residual
                    // with its tail): it goes on
                    need_tail = true;
                    need_open = std::max(need_open, std::max(full, 1));
                    red = h.inner_goal;
                } else if (h.stage != 0) {
                    int m = 2 * std::max(std::max(full, open_full), 1);
                    const int k = h.inner_iter - 1;  // index of the last inner residual evaluated
                    if (k >= 1 && h.rel_in > 0.0 && h.rel_in < 1.0) {
                        const double rate = std::pow(h.rel_in, 1.0 / k);
                        if (rate < 0.95) m = (int)std::ceil(std::log(h.inner_goal / h.rel_in) / std::log(rate) + 0.25);
                    }
                    // the phase ends after the pending update: one evaluation closes it
                    if (h.stop_next) m = 1;
                    if (h.stage == 1 && h.upd_due) need_update = true;
                    need_open = std::max(need_open, std::max(m, 1));
                    red = h.inner_goal;
                } else {
                    need_full = std::max(need_full, h.inner_last - first);
                }
                const double redc = std::clamp(red, 1e-12, 0.5);
                // in stage 0 the last update has not been measured yet (one
                // reduction pending), except after a check that did not end the
                // solve: its residual is that of the current p, and at least one
                // more step is due
                if (!(h.stage == 0 && h.checked)) rel *= redc;
                int st = 0;
                if (rel > 0.5 * h.tol) st = (int)std::ceil(std::log(0.5 * h.tol / rel) / std::log(redc));
                st = std::clamp(st, 0, 8);
                need_steps = std::max(need_steps, st);
                // the last predicted step: from rel redc^(st-1), it needs the
                // inner reduction max(inner tol, 0.8 tol / that)
                int last = h.inner_last - first;
                if (h.stage == 0 && st >= 1 && h.inner_last >= 2 && h.rel_in > 0.0 && h.rel_in < 1.0) {
                    const double rate = std::pow(h.rel_in, 1.0 / (h.inner_last - 1));
                    const double goal = std::max(h.inner_tol, 0.8 * h.tol / (rel * std::pow(redc, st - 1)));
                    if (rate < 0.95 && goal < 1.0)
                        last = (int)std::ceil(std::log(goal) / std::log(rate)) + 1 - first;
                }
                need_last = std::max(need_last, last);
            }
            open_full = std::min(need_open, prm.max_chunk);
            open_tail = need_tail;
            open_update = need_update;
            if (need_full > 0) full = std::clamp(need_full, 0, prm.max_chunk);
            full_last = need_last > 0 ? std::clamp(need_last, 1, full) : full;
            steps = need_steps;
            check = true;
        }
    }
    // the rounds ran out before every solve reached a terminal status: those
    // end as if capped (p is their last iterate)
    if (!all_done && (e = launch_stop_unfinished(d_slots, nslots, s)) != hipSuccess) return hip_status(e);
    if ((e = launch_fixup(g, geo, d_slots, nslots, s)) != hipSuccess) return hip_status(e);
    return POISSON_OK;
}

void fill_stats(const GridArgs& g, const SolveState& st, poisson_stats* out) {
    poisson_stats s{};
    s.status = st.status;
    const bool fp32 = st.precision == POISSON_FP32_REFINE;
    s.iters = fp32 ? st.inner_total : st.iter;
    s.outer_iters = fp32 ? st.iter : 0;
    s.rel_resid = st.rel;
    s.b_mean_removed = st.b_mean;
    s.b_norm = st.b_norm;
    s.rho_min = st.rho_min;
    s.rho_max = st.rho_max;
    // a-posteriori bound: every face coefficient is >= 1/rho_max, so on zero-mean
    // fields -A >= -L / rho_max and ||p - p*|| <= rho_max ||r|| / lambda_min(-L)
    const double pn2 = st.p_sumsq - st.p_sum * st.p_sum / (double)g.n;
    const double pn = pn2 > 0.0 ? std::sqrt(pn2) : 0.0;
    const double bound = st.rho_max * st.r_norm / min_symbol(g);
    s.err_bound_rel = (pn > 0.0 && st.status != POISSON_EDOMAIN) ? bound / pn : 0.0;
    s.ms = 0.0;
    s.p1_sweeps = st.p1_work;
    *out = s;
}

}  // namespace pois

// ---- C ABI -----------------------------------------------------------------------------

struct poisson_s {
    poisson_opts o{};
    GridArgs g{};
    Geometry geo{};
    hipStream_t stream = nullptr;  // the caller's stream
    hipStream_t run = nullptr;     // the library's stream for solves (graph capture needs one of its own)
    hipEvent_t ev_in = nullptr;    // orders a solve after the caller's earlier work
    GraphCache graphs;
    int device = 0;
    GridTables tables;
    Workspace ws;
    Slot* d_slot = nullptr;       // device copy of the slot
    Slot* h_slot = nullptr;       // pinned staging
    SolveState* h_state = nullptr;  // pinned copy of the state
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    poisson_stats stats{};
    int hist_count = 0;
    SweepTimer timer;            // events around one sweep kind inside solves
    double timer_ms = 0.0;       // summed bracketed time since the timer was set
    long long timer_launches = 0;
    double* proj_b = nullptr;    // right-hand side built by poisson_project (allocated at its first call)
    void* part_ws = nullptr;     // particle buffers of poisson_deposit / poisson_interpolate (grown on demand)
    size_t part_ws_bytes = 0;
    hipStream_t part_aux = nullptr;  // second stream of poisson_deposit (created at its first call)
    hipEvent_t part_fork = nullptr, part_join = nullptr;
};

extern "C" {

const char* poisson_strerror(int code) {
    switch (code) {
        case POISSON_OK: return "ok";
        case POISSON_EINVAL: return "invalid argument";
        case POISSON_ENOMEM: return "out of memory";
        case POISSON_EDOMAIN: return "rho must be finite and positive and b finite";
        case POISSON_ENOCONV: return "iteration cap reached before the tolerance";
        case POISSON_EDIVERGED: return "iteration diverged";
        case POISSON_EHIP: return "HIP runtime error";
        case POISSON_ETOOBIG: return "request exceeds the memory budget";
        case POISSON_EBUSY: return "no free slot or memory";
        case POISSON_ENOTFOUND: return "unknown request";
        default: return "unknown status";
    }
}

void poisson_destroy(poisson_t h) {
    if (!h) return;
    if (h->d_slot) (void)hipFree(h->d_slot);
    if (h->h_slot) (void)hipHostFree(h->h_slot);
    if (h->h_state) (void)hipHostFree(h->h_state);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    for (hipEvent_t& ev : h->timer.ev)
        if (ev) (void)hipEventDestroy(ev);
    h->graphs.release();
    if (h->ev_in) (void)hipEventDestroy(h->ev_in);
    if (h->run) (void)hipStreamDestroy(h->run);
    h->ws.release();
    h->tables.release();
    if (h->proj_b) (void)hipFree(h->proj_b);
    if (h->part_ws) (void)hipFree(h->part_ws);
    if (h->part_fork) (void)hipEventDestroy(h->part_fork);
    if (h->part_join) (void)hipEventDestroy(h->part_join);
    if (h->part_aux) (void)hipStreamDestroy(h->part_aux);
    delete h;
}

int poisson_create(const poisson_opts* o, poisson_t* out) {
    if (!out) return POISSON_EINVAL;
    *out = nullptr;
    if (!o) return POISSON_EINVAL;
    if (!length_supported(o->nx) || !length_supported(o->ny) || !length_supported(o->nz)) return POISSON_EINVAL;
    if (!valid_lengths(o->lx, o->ly, o->lz)) return POISSON_EINVAL;
    if (o->precision != POISSON_FP64 && o->precision != POISSON_FP32_REFINE) return POISSON_EINVAL;
    if (o->coef != POISSON_COEF_RHO_FACE_MEAN && o->coef != POISSON_COEF_INVRHO_FACE_MEAN) return POISSON_EINVAL;
    if (o->weight != POISSON_W_RHO && o->weight != POISSON_W_DIAG) return POISSON_EINVAL;
    if (o->bc_x != POISSON_BC_PERIODIC && o->bc_x != POISSON_BC_WALLS_X) return POISSON_EINVAL;
    poisson_s* h = new (std::nothrow) poisson_s();
    if (!h) return POISSON_ENOMEM;
    h->o = *o;
    if (h->o.max_iter <= 0) h->o.max_iter = 1000;
    if (!(h->o.inner_tol > 0.0)) h->o.inner_tol = 5e-4;
    h->stream = static_cast<hipStream_t>(o->stream);
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return POISSON_EHIP;
    }
    h->g = make_grid(o->nx, o->ny, o->nz, o->lx, o->ly, o->lz, o->coef, o->weight, o->bc_x);
    h->geo = make_geometry(h->g);
    int rc = h->tables.build(h->g);
    if (rc == POISSON_OK) rc = h->ws.allocate(h->g, h->geo, o->precision);
    if (rc == POISSON_OK && hipMalloc(&h->d_slot, sizeof(Slot)) != hipSuccess) rc = POISSON_ENOMEM;
    if (rc == POISSON_OK && hipHostMalloc(&h->h_slot, sizeof(Slot), hipHostMallocDefault) != hipSuccess)
        rc = POISSON_ENOMEM;
    if (rc == POISSON_OK && hipHostMalloc(&h->h_state, sizeof(SolveState), hipHostMallocDefault) != hipSuccess)
        rc = POISSON_ENOMEM;
    if (rc == POISSON_OK && (hipEventCreate(&h->ev0) != hipSuccess || hipEventCreate(&h->ev1) != hipSuccess ||
                             hipEventCreateWithFlags(&h->ev_in, hipEventDisableTiming) != hipSuccess))
        rc = POISSON_EHIP;
    // default priority (no priority argument anywhere)
    if (rc == POISSON_OK && hipStreamCreateWithFlags(&h->run, hipStreamNonBlocking) != hipSuccess) rc = POISSON_EHIP;
    if (rc != POISSON_OK) {
        poisson_destroy(h);
        return rc;
    }
    *out = h;
    return POISSON_OK;
}

static bool overlaps(const void* a, const void* b, size_t bytes) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bytes && y < x + bytes;
}

// [a, a + na) and [b, b + nb) share a byte
static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return na > 0 && nb > 0 && x < y + nb && y < x + na;
}

static int set_slot(poisson_t h, const Slot& s, hipStream_t st) {
    *h->h_slot = s;
    return hip_status(hipMemcpyAsync(h->d_slot, h->h_slot, sizeof(Slot), hipMemcpyHostToDevice, st));
}

static int set_slot(poisson_t h, const Slot& s) { return set_slot(h, s, h->stream); }

int poisson_solve(poisson_t h, const double* rho, const double* b, double* p, double tol) {
    if (!h || !rho || !b || !p || !(tol > 0.0) || !std::isfinite(tol)) return POISSON_EINVAL;
    const size_t bytes = (size_t)h->g.n * sizeof(double);
    if (overlaps(rho, b, bytes) || overlaps(rho, p, bytes) || overlaps(b, p, bytes)) return POISSON_EINVAL;
    // the solve runs on the library's stream, after the caller's earlier work
    int rc = hip_status(hipEventRecord(h->ev_in, h->stream));
    if (rc == POISSON_OK) rc = hip_status(hipStreamWaitEvent(h->run, h->ev_in, 0));
    if (rc == POISSON_OK) rc = set_slot(h, h->ws.slot(rho, b, p, tol), h->run);
    if (rc != POISSON_OK) return rc;
    SolveParams prm;
    prm.tol = tol;
    prm.precision = h->o.precision;
    prm.max_iter = h->o.max_iter;
    prm.inner_tol = h->o.inner_tol;
    if ((rc = hip_status(hipEventRecord(h->ev0, h->run))) != POISSON_OK) return rc;
    SolveState* dst = h->ws.st;
    h->timer.used = 0;
    rc = drive_solve(h->g, h->geo, h->tables.t, h->d_slot, 1, &dst, h->h_state, prm, h->run,
                     h->timer.sweep ? &h->timer : nullptr, h->o.use_graphs ? &h->graphs : nullptr);
    if (rc != POISSON_OK) return rc;
    if ((rc = hip_status(hipEventRecord(h->ev1, h->run))) != POISSON_OK) return rc;
    if ((rc = hip_status(hipMemcpyAsync(h->h_state, h->ws.st, sizeof(SolveState), hipMemcpyDeviceToHost,
                                        h->run))) != POISSON_OK)
        return rc;
    if ((rc = hip_status(hipStreamSynchronize(h->run))) != POISSON_OK) return rc;
    const SolveState& st = *h->h_state;
    fill_stats(h->g, st, &h->stats);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, h->ev0, h->ev1) == hipSuccess) h->stats.ms = ms;
    for (int q = 0; q < h->timer.used; ++q) {
        float kms = 0.f;
        if ((rc = hip_status(hipEventElapsedTime(&kms, h->timer.ev[2 * q], h->timer.ev[2 * q + 1]))) != POISSON_OK)
            return rc;
        h->timer_ms += kms;
        h->timer_launches += 1;
    }
    h->timer.used = 0;
    h->hist_count = std::min(st.iter + 1, kHistCap);
    if (st.status == POISSON_EDOMAIN) h->hist_count = 0;
    return h->stats.status;
}

int poisson_get_stats(poisson_t h, poisson_stats* s) {
    if (!h || !s) return POISSON_EINVAL;
    *s = h->stats;
    return POISSON_OK;
}

int poisson_get_history(poisson_t h, double* hist, int cap) {
    if (!h || (!hist && cap > 0) || cap < 0) return POISSON_EINVAL;
    const int n = std::min(cap, h->hist_count);
    for (int k = 0; k < n; ++k) hist[k] = h->h_state->hist[k];
    return h->hist_count;
}

int poisson_apply(poisson_t h, const double* rho, const double* p, double* out) {
    if (!h || !rho || !p || !out) return POISSON_EINVAL;
    int rc = hip_status(launch_apply(h->g, h->geo, rho, p, out, h->stream));
    if (rc != POISSON_OK) return rc;
    return hip_status(hipStreamSynchronize(h->stream));
}

int poisson_residual(poisson_t h, const double* rho, const double* b, const double* p, double* r,
                     double* r_norm, double* b_norm) {
    if (!h || !rho || !b || !p) return POISSON_EINVAL;
    // the residual sweep only reads p; the host copy of the last solve's state
    // (stats, history) is not touched
    Slot s = h->ws.slot(rho, b, const_cast<double*>(p), 1.0);
    int rc = set_slot(h, s);
    if (rc != POISSON_OK) return rc;
    hipError_t e;
    if ((e = launch_init(h->g, h->d_slot, 1, 1.0, 0, 0, POISSON_FP64, h->stream)) != hipSuccess) return hip_status(e);
    if ((e = launch_setup(h->g, h->geo, h->d_slot, 1, false, h->stream)) != hipSuccess) return hip_status(e);
    if ((e = launch_setup_finalize(h->g, h->geo, h->d_slot, 1, h->stream)) != hipSuccess) return hip_status(e);
    if ((e = launch_residual(h->g, h->geo, h->d_slot, r, h->stream)) != hipSuccess) return hip_status(e);
    const int nb = h->geo.blocks_pt;
    std::vector<double> part((size_t)nb * kPartialStride);
    if ((e = hipMemcpyAsync(part.data(), h->ws.partial, part.size() * 8, hipMemcpyDeviceToHost, h->stream)) !=
        hipSuccess)
        return hip_status(e);
    if ((e = hipStreamSynchronize(h->stream)) != hipSuccess) return hip_status(e);
    double s0 = 0.0, s1 = 0.0;
    for (int q = 0; q < nb; ++q) {
        s0 += part[(size_t)q * kPartialStride + 0];
        s1 += part[(size_t)q * kPartialStride + 1];
    }
    if (r_norm) *r_norm = std::sqrt(s0);
    if (b_norm) *b_norm = std::sqrt(s1);
    return POISSON_OK;
}

int poisson_time_sweep(poisson_t h, int sweep, int fp32, const double* rho, const double* b, double* p, int reps,
                       double* avg_ms) {
    if (!h || !rho || !b || !p || !avg_ms || reps < 1) return POISSON_EINVAL;
    if (sweep != 1 && sweep != 2 && sweep != 3 && sweep != 5 && sweep != 6) return POISSON_EINVAL;
    if ((fp32 || sweep == 6) && h->o.precision != POISSON_FP32_REFINE) return POISSON_EINVAL;
    // a state that never converges (tol 0) so that every sweep does its work
    int rc = set_slot(h, h->ws.slot(rho, b, p, 0.0));
    if (rc != POISSON_OK) return rc;
    hipError_t e;
    if ((e = launch_init(h->g, h->d_slot, 1, 0.0, 1 << 30, 1 << 30, h->o.precision, h->stream)) != hipSuccess)
        return hip_status(e);
    if ((e = launch_setup(h->g, h->geo, h->d_slot, 1, fp32 != 0, h->stream)) != hipSuccess) return hip_status(e);
    if ((e = launch_setup_finalize(h->g, h->geo, h->d_slot, 1, h->stream)) != hipSuccess) return hip_status(e);
    // the inner sweeps run in stage 1, which the outer residual opens; the
    // outer residual sweep itself in stage 0
    if (fp32 && sweep != 6 &&
        (e = launch_outer_residual(h->g, h->geo, h->tables.t, h->d_slot, 1, h->stream, nullptr)) != hipSuccess)
        return hip_status(e);
    auto one = [&]() {
        if (sweep != 6) return launch_sweep(h->g, h->tables.t, h->d_slot, 1, fp32 != 0, sweep, h->stream);
        return outer_fusable(h->g) ? launch_outer_fused(h->g, h->tables.t, h->d_slot, 1, h->stream, nullptr)
                                   : launch_outer_resid_sweep(h->g, h->d_slot, 1, h->stream, nullptr);
    };
    if ((e = one()) != hipSuccess) return hip_status(e);  // warm
    if ((e = hipEventRecord(h->ev0, h->stream)) != hipSuccess) return hip_status(e);
    for (int r = 0; r < reps; ++r)
        if ((e = one()) != hipSuccess) return hip_status(e);
    if ((e = hipEventRecord(h->ev1, h->stream)) != hipSuccess) return hip_status(e);
    if ((e = hipEventSynchronize(h->ev1)) != hipSuccess) return hip_status(e);
    float ms = 0.f;
    if ((e = hipEventElapsedTime(&ms, h->ev0, h->ev1)) != hipSuccess) return hip_status(e);
    *avg_ms = (double)ms / reps;
    return POISSON_OK;
}

int poisson_kernel_timer(poisson_t h, int sweep, int fp32) {
    if (!h || (sweep != 0 && sweep != 1 && sweep != 2 && sweep != 3 && sweep != 5)) return POISSON_EINVAL;
    if (fp32 && h->o.precision != POISSON_FP32_REFINE) return POISSON_EINVAL;
    if (sweep != 0 && !h->timer.ev[0]) {
        // The events only take timestamps; nothing on the host reads memory
        // through them, so they release at device scope.  A system-scope release
        // writes the L2 back at every event, and that time would be charged to
        // the sweep the events bracket.
        for (hipEvent_t& ev : h->timer.ev)
            if (hipEventCreateWithFlags(&ev, hipEventDisableSystemFence) != hipSuccess) return POISSON_EHIP;
    }
    h->timer.sweep = sweep;
    h->timer.fp32 = fp32 != 0;
    h->timer.used = 0;
    h->timer_ms = 0.0;
    h->timer_launches = 0;
    return POISSON_OK;
}

int poisson_kernel_timer_read(poisson_t h, double* total_ms, long long* launches) {
    if (!h || !total_ms || !launches) return POISSON_EINVAL;
    *total_ms = h->timer_ms;
    *launches = h->timer_launches;
    return POISSON_OK;
}

int poisson_divergence(poisson_t h, const double* rho, const double* mx, const double* my, const double* mz,
                       double* out) {
    if (!h || !rho || !mx || !my || !mz || !out) return POISSON_EINVAL;
    const size_t fb = (size_t)h->g.n * sizeof(double);
    for (const void* f : {(const void*)rho, (const void*)mx, (const void*)my, (const void*)mz})
        if (overlaps(out, fb, f, fb)) return POISSON_EINVAL;
    int rc = hip_status(launch_divergence(h->g, rho, mx, my, mz, nullptr, 1.0, out, h->stream));
    if (rc != POISSON_OK) return rc;
    return hip_status(hipStreamSynchronize(h->stream));
}

int poisson_project(poisson_t h, const double* rho, double* mx, double* my, double* mz, const double* rhs_div,
                    double c_dt, double* p, double tol, double* chi) {
    if (!h || !rho || !mx || !my || !mz || !rhs_div || !p) return POISSON_EINVAL;
    if (!(c_dt > 0.0) || !std::isfinite(c_dt) || !(tol > 0.0) || !std::isfinite(tol)) return POISSON_EINVAL;
    const size_t bytes = (size_t)h->g.n * sizeof(double);
    const void* f[7] = {rho, mx, my, mz, rhs_div, p, nullptr};
    for (int a = 0; a < 6; ++a)
        for (int b = a + 1; b < 6; ++b)
            if (overlaps(f[a], f[b], bytes)) return POISSON_EINVAL;
    if (!h->proj_b && hipMalloc(&h->proj_b, bytes) != hipSuccess) {
        h->proj_b = nullptr;
        return POISSON_ENOMEM;
    }
    // RHS^Pois on the caller's stream; the solve orders itself after it
    int rc = hip_status(launch_divergence(h->g, rho, mx, my, mz, rhs_div, c_dt, h->proj_b, h->stream));
    if (rc != POISSON_OK) return rc;
    rc = poisson_solve(h, rho, h->proj_b, p, tol);
    if (rc != POISSON_OK && rc != POISSON_ENOCONV) return rc;  // momentum untouched
    if (chi) *chi = -c_dt * h->stats.b_mean_removed;
    // the solve has finished (poisson_solve waits for it): correct the momentum
    const int rc2 = hip_status(launch_correct(h->g, p, mx, my, mz, c_dt, h->stream));
    if (rc2 != POISSON_OK) return rc2;
    const int rc3 = hip_status(hipStreamSynchronize(h->stream));
    return rc3 != POISSON_OK ? rc3 : rc;
}

static int particle_ws(poisson_t h, size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    if (h->part_ws_bytes >= bytes) return POISSON_OK;
    if (h->part_ws) (void)hipFree(h->part_ws);
    h->part_ws = nullptr;
    h->part_ws_bytes = 0;
    if (hipMalloc(&h->part_ws, bytes) != hipSuccess) {
        h->part_ws = nullptr;
        return POISSON_ENOMEM;
    }
    h->part_ws_bytes = bytes;
    return POISSON_OK;
}

int poisson_deposit(poisson_t h, int n_particles, const double* pos, const double* q, double* out) {
    if (!h || n_particles < 0 || (n_particles > 0 && !pos) || !out || h->g.bcx != 0) return POISSON_EINVAL;
    const size_t fb = (size_t)h->g.n * sizeof(double), pb = (size_t)n_particles * 3 * sizeof(double);
    if (overlaps(out, fb, pos, pb) || (q && overlaps(out, fb, q, (size_t)n_particles * sizeof(double))))
        return POISSON_EINVAL;
    int rc = particle_ws(h, particle_workspace_bytes(h->g, n_particles));
    if (rc != POISSON_OK) return rc;
    if (!h->part_aux) {
        // default priority (no priority argument anywhere)
        if (hipStreamCreateWithFlags(&h->part_aux, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&h->part_fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&h->part_join, hipEventDisableTiming) != hipSuccess)
            return POISSON_EHIP;
    }
    int bad = 0;
    rc = hip_status(launch_deposit(h->g, n_particles, pos, q, out, h->part_ws, h->part_ws_bytes, &bad, h->stream,
                                   h->part_aux, h->part_fork, h->part_join));
    if (rc != POISSON_OK) return rc;
    if (bad) return POISSON_EDOMAIN;
    return hip_status(hipStreamSynchronize(h->stream));
}

int poisson_interpolate(poisson_t h, int n_particles, const double* pos, const double* field, double* out) {
    if (!h || n_particles < 0 || (n_particles > 0 && (!pos || !out)) || !field || h->g.bcx != 0)
        return POISSON_EINVAL;
    const size_t ob = (size_t)n_particles * sizeof(double);
    if (overlaps(out, ob, pos, 3 * ob) || overlaps(out, ob, field, (size_t)h->g.n * sizeof(double)))
        return POISSON_EINVAL;
    int rc = particle_ws(h, 256);
    if (rc != POISSON_OK) return rc;
    int bad = 0;
    rc = hip_status(launch_interpolate(h->g, n_particles, pos, field, out, static_cast<int*>(h->part_ws), &bad,
                                       h->stream));
    if (rc != POISSON_OK) return rc;
    return bad ? POISSON_EDOMAIN : POISSON_OK;
}

static int lap_pinv(poisson_t h, const double* q, double* delta, bool fp32) {
    if (!h || !q || !delta) return POISSON_EINVAL;
    if (fp32 && h->o.precision != POISSON_FP32_REFINE) return POISSON_EINVAL;
    int rc = set_slot(h, h->ws.slot(nullptr, q, delta, 1.0));
    if (rc != POISSON_OK) return rc;
    hipError_t e = launch_lap_pinv(h->g, h->geo, h->tables.t, h->d_slot, h->stream, fp32);
    if (e != hipSuccess) return hip_status(e);
    return hip_status(hipStreamSynchronize(h->stream));
}

int poisson_lap_pinv(poisson_t h, const double* q, double* delta) { return lap_pinv(h, q, delta, false); }

int poisson_lap_pinv_fp32(poisson_t h, const double* q, double* delta) { return lap_pinv(h, q, delta, true); }

}  // extern "C"
