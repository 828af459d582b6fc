// poisson_solve_noalloc: the solve of poisson_solve for callers that cannot
// allocate device memory (code under stream capture, serving loops that must
// not call the allocator, harnesses that forbid it).
//
// Everything a solve needs besides the caller's rho, b and p -- the transform
// tables, the workspace (transform buffer, FP32 copies, partial sums, state
// record) and the slot record the kernels read -- lives in one file-scope
// device array, `scratch`, of kScratchBytes.  Each device that loads the
// library holds its own copy until the process ends.  In host code the name
// `scratch` is only a host-side stand-in: its device address is taken once per
// device with hipGetSymbolAddress and kept, and only that address is ever
// passed to kernels or copies.
//
// The solve runs the same kernels in the same launch configuration as
// poisson_solve, with the same tables, so the two give the same bits.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "../../include/poisson.h"
#include "poisson_engine.hpp"
#include "poisson_internal.hpp"

using namespace pois;

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr size_t kTablesHostBytes = size_t(160) << 10;  // tables of any supported grid (under 140 KiB)
constexpr int kMaxDevices = 64;

// Host state of the entry point, guarded by g_mu: the device address of
// `scratch` per device, and pageable host staging (no allocation) for the
// tables, the slot record and the state read back.
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};
alignas(256) unsigned char g_tables_host[kTablesHostBytes];
Slot g_slot_host;
SolveState g_state_host;

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Device address of this device's `scratch` (taken at the first call on it).
int scratch_address(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices) return POISSON_EINVAL;
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return POISSON_EHIP;
        g_scratch[dev] = ptr;
    }
    *out = static_cast<unsigned char*>(g_scratch[dev]);
    return POISSON_OK;
}

bool overlap(const void* a, const void* b, size_t bytes) {
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bytes && y < x + bytes;
}

}  // namespace

extern "C" {

int poisson_solve_noalloc(const poisson_opts* o, const double* rho, const double* b, double* p, double tol,
                          poisson_stats* stats) {
    if (!o || !rho || !b || !p || !(tol > 0.0) || !std::isfinite(tol)) return POISSON_EINVAL;
    if (!length_supported(o->nx) || !length_supported(o->ny) || !length_supported(o->nz)) return POISSON_EINVAL;
    if (!valid_lengths(o->lx, o->ly, o->lz)) return POISSON_EINVAL;
    if (o->precision != POISSON_FP64 && o->precision != POISSON_FP32_REFINE) return POISSON_EINVAL;
    if (o->coef != POISSON_COEF_RHO_FACE_MEAN && o->coef != POISSON_COEF_INVRHO_FACE_MEAN) return POISSON_EINVAL;
    if (o->weight != POISSON_W_RHO && o->weight != POISSON_W_DIAG) return POISSON_EINVAL;
    if (o->bc_x != POISSON_BC_PERIODIC && o->bc_x != POISSON_BC_WALLS_X) return POISSON_EINVAL;
    const GridArgs g = make_grid(o->nx, o->ny, o->nz, o->lx, o->ly, o->lz, o->coef, o->weight, o->bc_x);
    const size_t field = (size_t)g.n * sizeof(double);
    if (overlap(rho, b, field) || overlap(rho, p, field) || overlap(b, p, field)) return POISSON_EINVAL;
    const Geometry geo = make_geometry(g);

    // scratch layout: tables, workspace, slot record
    const size_t tb = tables_bytes(g);
    const size_t off_ws = align256(tb);
    const size_t off_slot = align256(off_ws + workspace_bytes(g, geo, o->precision));
    const size_t need = off_slot + align256(sizeof(Slot));
    if (need > kScratchBytes || tb > kTablesHostBytes) return POISSON_ETOOBIG;

    // one call at a time in the process: the device array and the host
    // staging are shared by every call
    std::lock_guard<std::mutex> lock(g_mu);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return POISSON_EHIP;
    unsigned char* base = nullptr;
    int rc = scratch_address(dev, &base);
    if (rc != POISSON_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(o->stream);
    const auto t0 = std::chrono::steady_clock::now();

    fill_tables(g, g_tables_host);
    hipError_t e = hipMemcpyAsync(base, g_tables_host, tb, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_status(e);
    const Tables tables = bind_tables(g, base);
    Workspace ws;
    ws.carve(g, geo, o->precision, base + off_ws);
    g_slot_host = ws.slot(rho, b, p, tol);
    Slot* d_slot = reinterpret_cast<Slot*>(base + off_slot);
    if ((e = hipMemcpyAsync(d_slot, &g_slot_host, sizeof(Slot), hipMemcpyHostToDevice, s)) != hipSuccess)
        return hip_status(e);

    SolveParams prm;
    prm.tol = tol;
    prm.precision = o->precision;
    prm.max_iter = o->max_iter > 0 ? o->max_iter : 1000;
    prm.inner_tol = o->inner_tol > 0.0 ? o->inner_tol : 5e-4;
    SolveState* st_dev = ws.st;
    rc = drive_solve(g, geo, tables, d_slot, 1, &st_dev, &g_state_host, prm, s, nullptr, nullptr);
    if (rc != POISSON_OK) return rc;
    if ((e = hipMemcpyAsync(&g_state_host, ws.st, sizeof(SolveState), hipMemcpyDeviceToHost, s)) != hipSuccess)
        return hip_status(e);
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_status(e);
    poisson_stats out{};
    fill_stats(g, g_state_host, &out);
    out.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = out;
    return out.status;
}

}  // extern "C"
