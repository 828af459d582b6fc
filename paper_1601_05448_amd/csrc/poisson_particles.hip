// Particles and the grid (section "Physical model" of the paper): the linear
// projection P of particle values to the grid, per unit volume, and the linear
// interpolation I of a grid field at the particle positions, periodic.  A
// particle at x has, per direction, s = x/h - 1/2, i0 = floor(s), f = s - i0 and
// gives weight 1 - f to cell i0 and f to cell i0 + 1; its eight cells get the
// products of the three directions' weights.
//
// P without atomics, deterministic: every particle gets the key of its lower
// corner cell (i0, j0, k0); a stable radix sort (rocPRIM) orders the particles by
// key and, within a key, by index; for every occupied cell the thread at the
// start of its run of sorted particles records that start and adds, over the
// run in order, the eight corner sums sum_p q_p W_a W_b W_e (a, b, e the offsets
// 0/1 of the corner cell in x, y, z); then every grid cell adds the matching
// corner sums of its eight lower neighbours (itself included), in a fixed
// order, by one thread that marches along z (four run starts loaded per cell,
// the next plane's while the current cell adds).  Every cell is written once,
// by one thread, with the same sum order in every run.  I is a plain gather,
// one thread per particle.
#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>

#include "poisson_device.hpp"

namespace pois {

constexpr int kPartThreads = 256;
constexpr unsigned kNoParticle = 0xffffffffu;

// lower cell index and fraction of a coordinate along one direction; false if
// the position is not finite or more than 2^30 cells away
__device__ __forceinline__ bool cell_frac(double x, double inv_h, int n, int& i0, double& f) {
    const double s = x * inv_h - 0.5;
    if (!(fabs(s) < 1073741824.0)) return false;
    const double fl = floor(s);
    f = s - fl;
    long long a = (long long)fl % n;
    if (a < 0) a += n;
    i0 = (int)a;
    return true;
}

struct PartGeom {
    int nx, ny, nz;
    double inv_hx, inv_hy, inv_hz, inv_v;
};

__global__ void __launch_bounds__(kPartThreads)
k_part_keys(PartGeom pg, int np, const double* __restrict__ pos, unsigned* __restrict__ key,
            unsigned* __restrict__ idx, int* __restrict__ bad) {
    const int p = blockIdx.x * kPartThreads + threadIdx.x;
    if (p >= np) return;
    int i, j, k;
    double fx, fy, fz;
    const bool ok = cell_frac(pos[3 * (size_t)p], pg.inv_hx, pg.nx, i, fx) &&
                    cell_frac(pos[3 * (size_t)p + 1], pg.inv_hy, pg.ny, j, fy) &&
                    cell_frac(pos[3 * (size_t)p + 2], pg.inv_hz, pg.nz, k, fz);
    if (!ok) {
        bad[0] = 1;  // plain vector store: every writer writes the same value
        i = j = k = 0;
    }
    key[p] = ((unsigned)k * (unsigned)pg.ny + (unsigned)j) * (unsigned)pg.nx + (unsigned)i;
    idx[p] = (unsigned)p;
}

__global__ void __launch_bounds__(kPartThreads) k_part_fill(unsigned* __restrict__ a, unsigned long long n, unsigned v) {
    for (unsigned long long c = (unsigned long long)blockIdx.x * kPartThreads + threadIdx.x; c < n;
         c += (unsigned long long)gridDim.x * kPartThreads)
        a[c] = v;
}

__global__ void __launch_bounds__(kPartThreads) k_part_flag_clear(int* __restrict__ bad) {
    if (threadIdx.x == 0) bad[0] = 0;
}

// The thread at the start s of each run of equal keys (one occupied lower
// corner cell c): first[c] = s, and corner[8 s + q] = the run's sum, in sorted
// order, of q_p W_a W_b W_e for corner q = a + 2 b + 4 e, with W = 1 - f for
// offset 0 and f for offset 1.
__global__ void __launch_bounds__(kPartThreads)
k_part_runs(PartGeom pg, int np, const double* __restrict__ pos, const double* __restrict__ q,
            const unsigned* __restrict__ key_s, const unsigned* __restrict__ idx_s, unsigned* __restrict__ first,
            double* __restrict__ corner) {
    const int s = blockIdx.x * kPartThreads + threadIdx.x;
    if (s >= np) return;
    const unsigned k = key_s[s];
    if (s > 0 && key_s[s - 1] == k) return;
    first[k] = (unsigned)s;
    double acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.0;
    for (int e = s; e < np && key_s[e] == k; ++e) {
        const unsigned p = idx_s[e];
        int i;
        double fx = 0.0, fy = 0.0, fz = 0.0;
        (void)cell_frac(pos[3 * (size_t)p], pg.inv_hx, pg.nx, i, fx);
        (void)cell_frac(pos[3 * (size_t)p + 1], pg.inv_hy, pg.ny, i, fy);
        (void)cell_frac(pos[3 * (size_t)p + 2], pg.inv_hz, pg.nz, i, fz);
        const double qp = q ? q[p] : 1.0;
#pragma unroll
        for (int c = 0; c < 8; ++c)
            acc[c] += qp * ((c & 1) ? fx : 1.0 - fx) * ((c & 2) ? fy : 1.0 - fy) * ((c & 4) ? fz : 1.0 - fz);
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) corner[8 * (size_t)s + c] = acc[c];
}

// out_c = sum over the lower neighbours c - (a, b, e), a, b, e in {0, 1}, of
// their runs' corner sums for corner a + 2 b + 4 e, times 1/V.  A thread owns
// column (i, j) and marches along z through kGatherPlanes cells: the run starts
// of plane k (four columns: (i, j), (i-1, j), (i, j-1), (i-1, j-1)) serve as the
// e = 0 corners of cell k and the e = 1 corners of cell k + 1, and the next
// plane's starts are loaded while the current cell adds its sums.
constexpr int kGatherPlanes = 16;

__global__ void __launch_bounds__(kPartThreads)
k_part_gather(PartGeom pg, const unsigned* __restrict__ first, const double* __restrict__ corner,
              double* __restrict__ out) {
    const unsigned nx = pg.nx, ny = pg.ny, nz = pg.nz;
    const unsigned i = blockIdx.x * kPartThreads + threadIdx.x, j = blockIdx.y;
    if (i >= nx) return;
    const unsigned im = (i == 0) ? nx - 1 : i - 1, jm = (j == 0) ? ny - 1 : j - 1;
    const unsigned col[4] = {j * nx + i, j * nx + im, jm * nx + i, jm * nx + im};  // a + 2 b
    const unsigned sz = nx * ny;
    const unsigned k0 = blockIdx.z * kGatherPlanes;
    const unsigned k1 = (k0 + kGatherPlanes < nz) ? k0 + kGatherPlanes : nz;
    unsigned prev[4], cur[4];
    const unsigned km = (k0 == 0 ? nz - 1 : k0 - 1) * sz;
#pragma unroll
    for (int q = 0; q < 4; ++q) prev[q] = first[km + col[q]];
#pragma unroll
    for (int q = 0; q < 4; ++q) cur[q] = first[k0 * sz + col[q]];
    for (unsigned k = k0; k < k1; ++k) {
        unsigned nxt[4];
        const unsigned kn = (k + 1 < nz ? k + 1 : 0) * sz;
#pragma unroll
        for (int q = 0; q < 4; ++q) nxt[q] = first[kn + col[q]];  // in flight during this cell
        double v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const unsigned f0 = (q & 4) ? prev[q & 3] : cur[q & 3];
            v[q] = (f0 == kNoParticle) ? 0.0 : corner[8 * (size_t)f0 + q];
        }
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) acc += v[q];
        out[(size_t)k * sz + col[0]] = acc * pg.inv_v;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            prev[q] = cur[q];
            cur[q] = nxt[q];
        }
    }
}

__global__ void __launch_bounds__(kPartThreads)
k_part_interp(PartGeom pg, int np, const double* __restrict__ pos, const double* __restrict__ field,
              double* __restrict__ out, int* __restrict__ bad) {
    const int p = blockIdx.x * kPartThreads + threadIdx.x;
    if (p >= np) return;
    int i, j, k;
    double fx, fy, fz;
    const bool ok = cell_frac(pos[3 * (size_t)p], pg.inv_hx, pg.nx, i, fx) &&
                    cell_frac(pos[3 * (size_t)p + 1], pg.inv_hy, pg.ny, j, fy) &&
                    cell_frac(pos[3 * (size_t)p + 2], pg.inv_hz, pg.nz, k, fz);
    if (!ok) {
        bad[0] = 1;
        out[p] = 0.0;
        return;
    }
    const unsigned nx = pg.nx, ny = pg.ny, nz = pg.nz;
    const unsigned ix[2] = {(unsigned)i, ((unsigned)i + 1) % nx};
    const unsigned iy[2] = {(unsigned)j, ((unsigned)j + 1) % ny};
    const unsigned iz[2] = {(unsigned)k, ((unsigned)k + 1) % nz};
    const double wx[2] = {1.0 - fx, fx}, wy[2] = {1.0 - fy, fy}, wz[2] = {1.0 - fz, fz};
    double acc = 0.0;
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a)
                acc += wx[a] * wy[b] * wz[e] * field[((size_t)iz[e] * ny + iy[b]) * nx + ix[a]];
    out[p] = acc;
}

static PartGeom part_geom(const GridArgs& g) {
    PartGeom pg;
    pg.nx = g.nx;
    pg.ny = g.ny;
    pg.nz = g.nz;
    pg.inv_hx = std::sqrt(g.ihx2);
    pg.inv_hy = std::sqrt(g.ihy2);
    pg.inv_hz = std::sqrt(g.ihz2);
    pg.inv_v = pg.inv_hx * pg.inv_hy * pg.inv_hz;
    return pg;
}

static int key_bits(long long n) {
    int b = 1;
    while ((1ll << b) < n) ++b;
    return b;
}

size_t particle_workspace_bytes(const GridArgs& g, int np) {
    size_t temp = 0;
    (void)rocprim::radix_sort_pairs(nullptr, temp, (const unsigned*)nullptr, (unsigned*)nullptr,
                                    (const unsigned*)nullptr, (unsigned*)nullptr, (unsigned)np, 0,
                                    key_bits(g.n), (hipStream_t)0);
    // keys, indices, sorted keys, sorted indices, corner sums, flag, sort temp
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return 4 * up((size_t)np * 4) + up((size_t)np * 64) + 256 + up(temp);
}

hipError_t launch_deposit(const GridArgs& g, int np, const double* pos, const double* q, double* out,
                          unsigned* cells2, void* ws, size_t ws_bytes, int* bad_host, hipStream_t s) {
    const PartGeom pg = part_geom(g);
    auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
    char* w = static_cast<char*>(ws);
    unsigned* key = reinterpret_cast<unsigned*>(w);
    unsigned* idx = reinterpret_cast<unsigned*>(w + up((size_t)np * 4));
    unsigned* key_s = reinterpret_cast<unsigned*>(w + 2 * up((size_t)np * 4));
    unsigned* idx_s = reinterpret_cast<unsigned*>(w + 3 * up((size_t)np * 4));
    double* corner = reinterpret_cast<double*>(w + 4 * up((size_t)np * 4));
    int* bad = reinterpret_cast<int*>(w + 4 * up((size_t)np * 4) + up((size_t)np * 64));
    void* temp = w + 4 * up((size_t)np * 4) + up((size_t)np * 64) + 256;
    size_t temp_bytes = ws_bytes - (4 * up((size_t)np * 4) + up((size_t)np * 64) + 256);
    unsigned* first = cells2;
    const unsigned long long n = (unsigned long long)g.n;
    const int pb = (np + kPartThreads - 1) / kPartThreads;
    hipError_t e;
    k_part_flag_clear<<<1, 64, 0, s>>>(bad);
    if (np > 0) {
        k_part_keys<<<pb, kPartThreads, 0, s>>>(pg, np, pos, key, idx, bad);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        int flag = 0;
        if ((e = hipMemcpyAsync(&flag, bad, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        if (flag) {
            *bad_host = 1;
            return hipSuccess;
        }
        if ((e = rocprim::radix_sort_pairs(temp, temp_bytes, key, key_s, idx, idx_s, (unsigned)np, 0, key_bits(g.n),
                                           s)) != hipSuccess)
            return e;
    }
    const unsigned fb = (unsigned)std::min<unsigned long long>((n + kPartThreads - 1) / kPartThreads, 65536ull);
    k_part_fill<<<fb, kPartThreads, 0, s>>>(first, n, kNoParticle);
    if (np > 0) k_part_runs<<<pb, kPartThreads, 0, s>>>(pg, np, pos, q, key_s, idx_s, first, corner);
    const dim3 gg((unsigned)(g.nx + kPartThreads - 1) / kPartThreads, (unsigned)g.ny,
                  (unsigned)(g.nz + kGatherPlanes - 1) / kGatherPlanes);
    k_part_gather<<<gg, kPartThreads, 0, s>>>(pg, first, corner, out);
    return hipGetLastError();
}

hipError_t launch_interpolate(const GridArgs& g, int np, const double* pos, const double* field, double* out,
                              int* bad_dev, int* bad_host, hipStream_t s) {
    const PartGeom pg = part_geom(g);
    k_part_flag_clear<<<1, 64, 0, s>>>(bad_dev);
    if (np > 0) k_part_interp<<<(np + kPartThreads - 1) / kPartThreads, kPartThreads, 0, s>>>(pg, np, pos, field,
                                                                                               out, bad_dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int flag = 0;
    if ((e = hipMemcpyAsync(&flag, bad_dev, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    *bad_host = flag;
    return hipSuccess;
}

}  // namespace pois
