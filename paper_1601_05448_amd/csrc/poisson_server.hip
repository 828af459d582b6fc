// Serving engine of libpoisson: many independent variable-density Poisson
// solves of different grid sizes on one GPU, with continuous batching.
//
// Requests are queued in arrival order.  Each tick
//   1. admits queued requests, first come first served, while a slot is free
//      and the request's resident footprint (its rho, b and p plus the solver
//      workspace) fits the memory budget; workspaces are recycled per grid size;
//   2. advances every size class (all resident requests of one grid) by a chunk
//      of iterations with batched launches: blockIdx.y of every kernel selects
//      the request, each request keeps its own state, norms and stopping
//      decision on the device, and the classes run on their own streams so that
//      their work overlaps on the device.  A class's chunk is as long as its
//      request closest to done needs at the contraction it has shown, so that
//      requests retire as soon as they finish; with graphs on, each chunk's
//      launches are captured once per (batch size, chunk, share of the chip)
//      and replayed, the slot table being rewritten between replays;
//   3. retires finished requests (their p is final) and frees their slots.
// A request's arithmetic is exactly that of a solve of it alone: the kernels of
// one request read only that request's fields and workspace, and every
// reduction runs in a fixed order within the request.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/poisson.h"
#include "poisson_engine.hpp"
#include "poisson_internal.hpp"

using namespace pois;

namespace {

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    long long id;
    int nx, ny, nz;
    double lx, ly, lz;
    int bc_x;
    const double* rho;
    const double* b;
    double* p;
    double tol;
    double t_submit;
    double t_admit;
};

using ClassKey = std::tuple<int, int, int, double, double, double, int>;

struct Resident {
    Request req;
    Workspace* ws;
    bool fresh;
    int k_prev = -1;     // index of the residual evaluated at the previous chunk's end
    double r_prev = 0.0;  // and its relative residual
};

struct SizeClass {
    GridArgs g{};
    Geometry geo{};
    GridTables tables;
    hipStream_t stream = nullptr;
    hipEvent_t done_ev = nullptr;
    std::vector<Resident> active;
    std::vector<Workspace*> pool;  // idle workspaces of this grid
    Slot* d_slots = nullptr;       // device slot array, capacity max_slots
    Slot* h_slots = nullptr;       // pinned staging
    SolveState* h_hdr = nullptr;   // pinned state headers
    size_t ws_bytes = 0;
    long long cells = 0;
    bool in_flight = false;  // a chunk of this class is enqueued and not yet retired
    int n_launched = 0;      // active[0, n_launched) are the solves of that chunk
    int chunk = 4;           // iterations (FP32: inner sweeps) of the next chunk
    GraphCache graphs;       // captured chunks, keyed by batch size, chunk and share

    ~SizeClass() {
        for (Workspace* w : pool) {
            w->release();
            delete w;
        }
        for (Resident& r : active) {
            r.ws->release();
            delete r.ws;
        }
        if (d_slots) (void)hipFree(d_slots);
        if (h_slots) (void)hipHostFree(h_slots);
        if (h_hdr) (void)hipHostFree(h_hdr);
        graphs.release();
        if (done_ev) (void)hipEventDestroy(done_ev);
        if (stream) (void)hipStreamDestroy(stream);
        tables.release();
    }
};

}  // namespace

struct poisson_server_s {
    size_t budget = 0;
    size_t used = 0;  // bytes held: resident footprints plus pooled workspaces
    int max_slots = 0;
    SolveParams prm;
    int coef = 0, weight = 0;
    hipStream_t stream = nullptr;  // caller's stream: ticks are ordered after its prior work
    hipEvent_t fork_ev = nullptr;
    long long next_id = 1;
    std::deque<Request> queue;
    std::map<ClassKey, std::unique_ptr<SizeClass>> classes;
    std::map<long long, poisson_stats> finished;
    int resident = 0;
    bool use_graphs = false;
};

static size_t field_bytes(long long cells) { return (size_t)cells * 3 * sizeof(double); }

static int class_for(poisson_server_s* s, const Request& r, SizeClass** out) {
    const ClassKey key{r.nx, r.ny, r.nz, r.lx, r.ly, r.lz, r.bc_x};
    auto it = s->classes.find(key);
    if (it != s->classes.end()) {
        *out = it->second.get();
        return POISSON_OK;
    }
    auto c = std::make_unique<SizeClass>();
    c->g = make_grid(r.nx, r.ny, r.nz, r.lx, r.ly, r.lz, s->coef, s->weight, r.bc_x);
    c->geo = make_geometry(c->g);
    c->cells = c->g.n;
    c->ws_bytes = workspace_bytes(c->g, c->geo, s->prm.precision);
    int rc = c->tables.build(c->g);
    if (rc != POISSON_OK) return rc;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) return POISSON_EHIP;
    if (hipEventCreateWithFlags(&c->done_ev, hipEventDisableTiming) != hipSuccess) return POISSON_EHIP;
    if (hipMalloc(&c->d_slots, sizeof(Slot) * s->max_slots) != hipSuccess) return POISSON_ENOMEM;
    if (hipHostMalloc(&c->h_slots, sizeof(Slot) * s->max_slots, hipHostMallocDefault) != hipSuccess)
        return POISSON_ENOMEM;
    if (hipHostMalloc(&c->h_hdr, sizeof(SolveState) * s->max_slots, hipHostMallocDefault) != hipSuccess)
        return POISSON_ENOMEM;
    *out = c.get();
    s->classes.emplace(key, std::move(c));
    return POISSON_OK;
}

static size_t request_footprint(poisson_server_s* s, const Request& r) {
    const GridArgs g = make_grid(r.nx, r.ny, r.nz, r.lx, r.ly, r.lz, s->coef, s->weight, r.bc_x);
    return workspace_bytes(g, make_geometry(g), s->prm.precision) + field_bytes(g.n);
}

// Release idle pooled workspaces (largest first) until `need` more bytes fit.
// `keep` (may be NULL) is the class being admitted into when it is about to
// take one of its own pooled workspaces: its last pooled workspace stays.
static void trim_pools(poisson_server_s* s, size_t need, const SizeClass* keep) {
    while (s->used + need > s->budget) {
        SizeClass* best = nullptr;
        for (auto& kv : s->classes) {
            const SizeClass* c = kv.second.get();
            const size_t spare = c->pool.size() - (c == keep && !c->pool.empty() ? 1 : 0);
            if (spare > 0 && (!best || c->ws_bytes > best->ws_bytes)) best = kv.second.get();
        }
        if (!best) return;
        Workspace* w = best->pool.back();
        best->pool.pop_back();
        w->release();
        delete w;
        s->used -= best->ws_bytes;
    }
}

// Admit queued requests in arrival order while they fit.
static int admit(poisson_server_s* s) {
    while (!s->queue.empty() && s->resident < s->max_slots) {
        const Request& r = s->queue.front();
        SizeClass* c = nullptr;
        int rc = class_for(s, r, &c);
        if (rc != POISSON_OK) return rc;
        const size_t fields = field_bytes(c->cells);
        Workspace* w = nullptr;
        if (!c->pool.empty()) {
            // reuse one of the class's pooled workspaces (already counted in
            // `used`): only the fields are new
            if (s->used + fields > s->budget) trim_pools(s, fields, c);
            if (s->used + fields > s->budget) break;
            w = c->pool.back();
            c->pool.pop_back();
            s->used += fields;
        } else {
            const size_t need = c->ws_bytes + fields;
            if (s->used + need > s->budget) trim_pools(s, need, nullptr);
            if (s->used + need > s->budget) break;
            w = new (std::nothrow) Workspace();
            if (!w) return POISSON_ENOMEM;
            if (w->allocate(c->g, c->geo, s->prm.precision) != POISSON_OK) {
                delete w;
                break;  // the device is fuller than the budget says: wait for retirements
            }
            s->used += need;
        }
        Resident res{r, w, true};
        res.req.t_admit = now_ms();
        c->active.push_back(res);
        ++s->resident;
        s->queue.pop_front();
    }
    return POISSON_OK;
}

// Enqueue this tick's work of one class on its stream.
static int launch_class(poisson_server_s* s, SizeClass* c) {
    // fresh requests first, so that their set-up launches cover a prefix
    std::stable_partition(c->active.begin(), c->active.end(), [](const Resident& r) { return r.fresh; });
    int nfresh = 0;
    const int n = (int)c->active.size();
    for (int q = 0; q < n; ++q) {
        const Resident& r = c->active[q];
        c->h_slots[q] = r.ws->slot(r.req.rho, r.req.b, r.req.p, r.req.tol);
        if (r.fresh) ++nfresh;
    }
    hipError_t e;
    if ((e = hipMemcpyAsync(c->d_slots, c->h_slots, sizeof(Slot) * n, hipMemcpyHostToDevice, c->stream)) !=
        hipSuccess)
        return hip_status(e);
    const SolveParams& prm = s->prm;
    const bool fp32 = prm.precision == POISSON_FP32_REFINE;
    if (nfresh > 0) {
        if ((e = launch_init(c->g, c->d_slots, nfresh, prm.inner_tol, prm.max_iter, prm.max_outer, prm.precision,
                             c->stream)) != hipSuccess)
            return hip_status(e);
        if ((e = launch_setup(c->g, c->geo, c->d_slots, nfresh, fp32, c->stream)) != hipSuccess) return hip_status(e);
        if ((e = launch_setup_finalize(c->g, c->geo, c->d_slots, nfresh, c->stream)) != hipSuccess)
            return hip_status(e);
        for (Resident& r : c->active) r.fresh = false;
    }
    // FP64: `chunk` iterations.  FP32: one fixed sequence for solves at any
    // stage (each kernel acts only on the solves whose stage it serves): the
    // outer residual, `chunk` inner sweeps, the update.
    const int chunk = c->chunk;
    auto body = [&]() -> hipError_t {
        hipError_t le = hipSuccess;
        if (fp32) le = launch_outer_residual(c->g, c->geo, c->tables.t, c->d_slots, n, c->stream, nullptr);
        for (int k = 0; k < chunk && le == hipSuccess; ++k)
            le = launch_iteration(c->g, c->geo, c->tables.t, c->d_slots, n, fp32, c->stream);
        if (fp32 && le == hipSuccess) le = launch_outer_update(c->g, c->geo, c->d_slots, n, c->stream);
        return le;
    };
    if (s->use_graphs) {
        // the launch grids depend on the batch size and the share of the chip
        const int share = c->geo.share < 0.6f ? 0 : c->geo.share < 0.9f ? 1 : 2;
        const long long key = ((long long)n << 8) | ((long long)chunk << 2) | share;
        if (c->graphs.exec.size() >= 256) c->graphs.release();
        e = c->graphs.run(key, c->stream, body);
    } else {
        e = body();
    }
    if (e != hipSuccess) return hip_status(e);
    const size_t hb = offsetof(SolveState, hist);
    for (int q = 0; q < n; ++q)
        if ((e = hipMemcpyAsync(&c->h_hdr[q], c->active[q].ws->st, hb, hipMemcpyDeviceToHost, c->stream)) !=
            hipSuccess)
            return hip_status(e);
    if ((e = hipEventRecord(c->done_ev, c->stream)) != hipSuccess) return hip_status(e);
    c->n_launched = n;
    c->in_flight = true;
    return POISSON_OK;
}

// After a class's chunk has completed: finish and retire the solves that are
// done.  Requests admitted while the chunk ran sit after active[n_launched).
static int retire_class(poisson_server_s* s, SizeClass* c) {
    hipError_t e;
    if ((e = hipEventSynchronize(c->done_ev)) != hipSuccess) return hip_status(e);
    c->in_flight = false;
    std::vector<int> done;
    // The next chunk: as many iterations as the request closest to done needs
    // to pass its tolerance at the contraction it has shown since the previous
    // chunk (or since its first residual), plus a quarter; 4 while no request
    // has shown one.  FP32: inner sweeps of the refinement step in progress.
    int need = 1 << 30;
    for (int q = 0; q < c->n_launched; ++q) {
        const SolveState& h = c->h_hdr[q];
        if (h.done) {
            done.push_back(q);
            continue;
        }
        Resident& r = c->active[q];
        if (s->prm.precision == POISSON_FP32_REFINE) {
            const int k = h.inner_iter - 1;
            if (h.stage == 1 && k >= 1 && h.rel_in > 0.0 && h.rel_in < 1.0) {
                const double rate = std::pow(h.rel_in, 1.0 / k);
                if (rate < 0.95)
                    need = std::min(need, (int)std::ceil(std::log(h.inner_goal / h.rel_in) / std::log(rate) + 0.25));
            }
            continue;
        }
        const int k = h.iter - 1;
        double rate = 1.0;
        if (r.k_prev >= 0 && k > r.k_prev && r.r_prev > 0.0)
            rate = std::pow(h.rel / r.r_prev, 1.0 / (k - r.k_prev));
        else if (k >= 1 && h.rel0 > 0.0)
            rate = std::pow(h.rel / h.rel0, 1.0 / k);
        r.k_prev = k;
        r.r_prev = h.rel;
        if (rate > 0.0 && rate < 0.95 && h.rel > 0.0)
            need = std::min(need, (int)std::ceil(std::log(h.tol / h.rel) / std::log(rate) + 0.25));
    }
    c->chunk = need == (1 << 30) ? 4 : std::clamp(need, 1, 16);
    c->n_launched = 0;
    if (done.empty()) return POISSON_OK;
    // end-of-solve fix-up (mean of p, b~ = 0) for the finished ones
    for (int u = 0; u < (int)done.size(); ++u) {
        const Resident& r = c->active[done[u]];
        c->h_slots[u] = r.ws->slot(r.req.rho, r.req.b, r.req.p, r.req.tol);
    }
    if ((e = hipMemcpyAsync(c->d_slots, c->h_slots, sizeof(Slot) * done.size(), hipMemcpyHostToDevice, c->stream)) !=
        hipSuccess)
        return hip_status(e);
    if ((e = launch_fixup(c->g, c->geo, c->d_slots, (int)done.size(), c->stream)) != hipSuccess) return hip_status(e);
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) return hip_status(e);
    const double t = now_ms();
    std::vector<Resident> keep;
    keep.reserve(c->active.size());
    size_t di = 0;
    for (int q = 0; q < (int)c->active.size(); ++q) {
        Resident& r = c->active[q];
        if (di < done.size() && done[di] == q) {
            ++di;
            poisson_stats st{};
            fill_stats(c->g, c->h_hdr[q], &st);
            st.ms = t - r.req.t_submit;
            st.queue_ms = r.req.t_admit - r.req.t_submit;
            s->finished[r.req.id] = st;
            c->pool.push_back(r.ws);
            s->used -= field_bytes(c->cells);
            --s->resident;
        } else {
            keep.push_back(r);
        }
    }
    c->active.swap(keep);
    return POISSON_OK;
}

extern "C" {

int poisson_server_create(size_t budget_bytes, int max_slots, int precision, int coef, int weight, int max_iter,
                          void* stream, poisson_server_t* out) {
    if (!out) return POISSON_EINVAL;
    *out = nullptr;
    if (budget_bytes == 0 || max_slots < 1 || max_slots > 4096) return POISSON_EINVAL;
    if (precision != POISSON_FP64 && precision != POISSON_FP32_REFINE) return POISSON_EINVAL;
    if (coef != POISSON_COEF_RHO_FACE_MEAN && coef != POISSON_COEF_INVRHO_FACE_MEAN) return POISSON_EINVAL;
    if (weight != POISSON_W_RHO && weight != POISSON_W_DIAG) return POISSON_EINVAL;
    poisson_server_s* s = new (std::nothrow) poisson_server_s();
    if (!s) return POISSON_ENOMEM;
    s->budget = budget_bytes;
    s->max_slots = max_slots;
    s->prm.precision = precision;
    s->prm.max_iter = max_iter > 0 ? max_iter : 1000;
    s->coef = coef;
    s->weight = weight;
    s->stream = static_cast<hipStream_t>(stream);
    if (hipEventCreateWithFlags(&s->fork_ev, hipEventDisableTiming) != hipSuccess) {
        delete s;
        return POISSON_EHIP;
    }
    *out = s;
    return POISSON_OK;
}

void poisson_server_destroy(poisson_server_t s) {
    if (!s) return;
    for (auto& kv : s->classes)
        if (kv.second->stream) (void)hipStreamSynchronize(kv.second->stream);
    s->classes.clear();
    if (s->fork_ev) (void)hipEventDestroy(s->fork_ev);
    delete s;
}

int poisson_server_submit(poisson_server_t s, int nx, int ny, int nz, double lx, double ly, double lz, int bc_x,
                          const double* rho, const double* b, double* p, double tol, long long* id) {
    if (!s || !id || !rho || !b || !p || !(tol > 0.0) || !std::isfinite(tol)) return POISSON_EINVAL;
    if (bc_x != POISSON_BC_PERIODIC && bc_x != POISSON_BC_WALLS_X) return POISSON_EINVAL;
    if (!length_supported(nx) || !length_supported(ny) || !length_supported(nz)) return POISSON_EINVAL;
    if (!valid_lengths(lx, ly, lz)) return POISSON_EINVAL;
    const size_t bytes = (size_t)nx * ny * nz * sizeof(double);
    auto overlaps = [bytes](const void* x, const void* y) {
        const uintptr_t a = reinterpret_cast<uintptr_t>(x), c = reinterpret_cast<uintptr_t>(y);
        return a < c + bytes && c < a + bytes;
    };
    if (overlaps(rho, b) || overlaps(rho, p) || overlaps(b, p)) return POISSON_EINVAL;
    Request r{s->next_id, nx, ny, nz, lx, ly, lz, bc_x, rho, b, p, tol, now_ms()};
    if (request_footprint(s, r) > s->budget) return POISSON_ETOOBIG;
    s->queue.push_back(r);
    *id = s->next_id++;
    return POISSON_OK;
}

int poisson_server_use_graphs(poisson_server_t s, int on) {
    if (!s) return POISSON_EINVAL;
    s->use_graphs = on != 0;
    return POISSON_OK;
}

int poisson_server_footprint(poisson_server_t s, int nx, int ny, int nz, int bc_x, size_t* bytes) {
    if (!s || !bytes) return POISSON_EINVAL;
    if (bc_x != POISSON_BC_PERIODIC && bc_x != POISSON_BC_WALLS_X) return POISSON_EINVAL;
    if (!length_supported(nx) || !length_supported(ny) || !length_supported(nz)) return POISSON_EINVAL;
    Request r{};
    r.nx = nx; r.ny = ny; r.nz = nz;
    r.lx = r.ly = r.lz = 1.0;  // the footprint does not depend on the box
    r.bc_x = bc_x;
    *bytes = request_footprint(s, r);
    return POISSON_OK;
}

int poisson_server_tick(poisson_server_t s) {
    if (!s) return POISSON_EINVAL;
    int rc;
    // retire the classes whose chunk has completed; the others keep running
    for (auto& kv : s->classes) {
        SizeClass* c = kv.second.get();
        if (!c->in_flight) continue;
        const hipError_t q = hipEventQuery(c->done_ev);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) return POISSON_EHIP;
        if ((rc = retire_class(s, c)) != POISSON_OK) return rc;
    }
    if ((rc = admit(s)) != POISSON_OK) return rc;
    // A class at least four times larger than the smallest active one takes
    // three quarters of the chip's resident blocks in its persistent sweeps,
    // so that the small classes' blocks find room beside it instead of waiting
    // for each of its sweeps to end; one at least 64 times larger takes half of
    // the CUs, one block on each that reserves the CU's LDS, so that the small
    // classes' blocks run on the other half and never share a CU with one of
    // its long sweeps (see persistent_grid in the sweeps).
    long long smallest = 0;
    for (auto& kv : s->classes)
        if (!kv.second->active.empty() && (smallest == 0 || kv.second->cells < smallest)) smallest = kv.second->cells;
    // idle classes start their next chunk, after the caller's earlier work on its stream
    bool forked = false;
    for (auto& kv : s->classes) {
        SizeClass* c = kv.second.get();
        if (c->in_flight || c->active.empty()) continue;
        c->geo.share = (c->cells >= 64 * smallest) ? 0.5f : (c->cells >= 4 * smallest) ? 0.75f : 1.0f;
        if (!forked) {
            if (hipEventRecord(s->fork_ev, s->stream) != hipSuccess) return POISSON_EHIP;
            forked = true;
        }
        if (hipStreamWaitEvent(c->stream, s->fork_ev, 0) != hipSuccess) return POISSON_EHIP;
        if ((rc = launch_class(s, c)) != POISSON_OK) return rc;
    }
    return (int)s->queue.size() + s->resident;
}

int poisson_server_poll(poisson_server_t s, long long id, poisson_stats* stats) {
    if (!s || !stats) return POISSON_EINVAL;
    auto it = s->finished.find(id);
    if (it != s->finished.end()) {
        *stats = it->second;
        return 0;
    }
    if (id >= 1 && id < s->next_id) return 1;
    return POISSON_ENOTFOUND;
}

}  // extern "C"
