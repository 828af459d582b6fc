// Host-side pieces of the solve driver shared by the single-solve C ABI and
// the serving engine.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

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
    void release();
    Slot slot(const double* rho, const double* b, double* p, double tol) const;
};

int hip_status(hipError_t e);
bool valid_lengths(double lx, double ly, double lz);
GridArgs make_grid(int nx, int ny, int nz, double lx, double ly, double lz, int coef, int weight);
double min_symbol(const GridArgs& g);
size_t workspace_bytes(const GridArgs& g, const Geometry& geo, int precision);
int drive_solve(const GridArgs& g, const Geometry& geo, const Tables& t, const Slot* d_slots, int nslots,
                SolveState* const* d_states, SolveState* hdr, const SolveParams& prm, hipStream_t s,
                SweepTimer* tm = nullptr);
void fill_stats(const GridArgs& g, const SolveState& st, poisson_stats* out);

}  // namespace pois
