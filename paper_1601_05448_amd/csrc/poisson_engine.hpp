// Host-side pieces of the solve driver shared by the single-solve C ABI and
// the serving engine.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <map>

#include "../../include/poisson.h"
#include "poisson_internal.hpp"

namespace pois {

struct SolveParams {
    double tol = 1e-10;
    double inner_tol = 5e-4;  // FP32 inner sweeps stop at this relative residual ...
    int precision = POISSON_FP64;
    int max_iter = 1000;      // ... or after this many inner (or FP64) iterations in total
    int max_outer = 30;
    int first_chunk = 4;      // iterations enqueued before the first poll
    int max_chunk = 16;
};

// Transform tables of one grid: their size in one buffer, their values written
// into a host buffer of that size, and the device pointers into a copy of it.
size_t tables_bytes(const GridArgs& g);
void fill_tables(const GridArgs& g, unsigned char* host);
Tables bind_tables(const GridArgs& g, const void* dev);

// Transform tables of one grid in device memory.
struct GridTables {
    void* mem = nullptr;
    Tables t{};
    int build(const GridArgs& g);
    void release();
};

// Workspace of one solve in one device allocation.
struct Workspace {
    void* mem = nullptr;
    size_t bytes = 0;
    double* W = nullptr;
    float *rho32 = nullptr, *r32 = nullptr, *d32 = nullptr, *W32 = nullptr;
    double* partial = nullptr;
    SolveState* st = nullptr;
    int allocate(const GridArgs& g, const Geometry& geo, int precision);
    // lay the workspace out in workspace_bytes(g, geo, precision) bytes at at_mem
    // (256-byte aligned) without allocating; release() then frees nothing
    void carve(const GridArgs& g, const Geometry& geo, int precision, void* at_mem);
    void release();
    Slot slot(const double* rho, const double* b, double* p, double tol) const;
};

// Captured HIP graphs of fixed launch sequences, keyed by an integer: the first
// run of a key captures what `enqueue` launches on the stream and instantiates
// it; every run replays the instantiated graph on the stream.  The sequences
// hold kernel launches only (no memsets, no host work), and their arguments
// point at device records (slots, states) whose contents may change between
// replays.
struct GraphCache {
    std::map<long long, hipGraphExec_t> exec;

    template <class F>
    hipError_t run(long long key, hipStream_t s, F&& enqueue) {
        auto it = exec.find(key);
        if (it == exec.end()) {
            hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return e;
            const hipError_t le = enqueue();
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(s, &g);
            if (le != hipSuccess || e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                return le != hipSuccess ? le : e;
            }
            hipGraphExec_t x = nullptr;
            e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return e;
            it = exec.emplace(key, x).first;
        }
        return hipGraphLaunch(it->second, s);
    }
    void release() {
        for (auto& kv : exec) (void)hipGraphExecDestroy(kv.second);
        exec.clear();
    }
};

int hip_status(hipError_t e);
bool valid_lengths(double lx, double ly, double lz);
GridArgs make_grid(int nx, int ny, int nz, double lx, double ly, double lz, int coef, int weight, int bcx = 0);
double min_symbol(const GridArgs& g);
size_t workspace_bytes(const GridArgs& g, const Geometry& geo, int precision);
int drive_solve(const GridArgs& g, const Geometry& geo, const Tables& t, const Slot* d_slots, int nslots,
                SolveState* const* d_states, SolveState* hdr, const SolveParams& prm, hipStream_t s,
                SweepTimer* tm = nullptr, GraphCache* gc = nullptr);
void fill_stats(const GridArgs& g, const SolveState& st, poisson_stats* out);

}  // namespace pois
