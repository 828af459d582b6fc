// Particles and the grid (section "Physical model" of the paper): the linear
// projection P of particle values to the grid, per unit volume, and the linear
// interpolation I of a grid field at the particle positions, periodic.  A
// particle at x has, per direction, s = x/h - 1/2, i0 = floor(s), f = s - i0 and
// gives weight 1 - f to cell i0 and f to cell i0 + 1; its eight cells get the
// products of the three directions' weights.
//
// P without floating-point atomics, deterministic: every particle gets the key
// of its lower corner cell (i0, j0, k0); a stable radix sort (least significant
// digit first, 10-bit digits; within a block the rank of a key among equal
// digits comes from wave ballots, so equal keys keep their index order) orders
// the particles by key and, within a key, by index; the run of each occupied
// cell is summed in pieces of at most kPiece sorted particles (so a cell holding
// many particles costs a few piece sums, not a long serial loop), and the
// pieces of a run are added in order into its eight corner sums
// sum_p q_p W_a W_b W_e (a, b, e the offsets 0/1 of the corner cell in x, y, z).
// The grid is zeroed, then eight passes, one per parity class of the run's cell,
// add each run's eight corner sums (over the cell volume) to its 2 x 2 x 2
// cells: within a pass no two runs touch the same cell, so every cell adds its
// contributions in the same order in every run.  I is a plain gather, one
// thread per particle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>

#include "poisson_device.hpp"

namespace pois {

constexpr int kPartThreads = 256;

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

// The key of a particle: its lower corner cell c = (k ny + j) nx + i, below it
// the parity class (i, j, k) mod 2 of that cell, so that the sorted particles
// come in eight contiguous classes (the scatter passes below), each ordered by
// cell.
__global__ void __launch_bounds__(kPartThreads)
k_part_keys(PartGeom pg, int np, const double* __restrict__ pos, unsigned* __restrict__ key,
            unsigned* __restrict__ idx, int* __restrict__ bad, int cell_bits) {
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
    // (grids of more than 2^29 cells leave no room for the class: cell keys alone)
    const unsigned color = (unsigned)(i & 1) | ((unsigned)(j & 1) << 1) | ((unsigned)(k & 1) << 2);
    const unsigned cell = ((unsigned)k * (unsigned)pg.ny + (unsigned)j) * (unsigned)pg.nx + (unsigned)i;
    key[p] = cell_bits <= 29 ? (color << cell_bits) | cell : cell;
    idx[p] = (unsigned)p;
}

__global__ void __launch_bounds__(kPartThreads) k_part_zero(double* __restrict__ a, unsigned long long n) {
    for (unsigned long long c = (unsigned long long)blockIdx.x * kPartThreads + threadIdx.x; c < n;
         c += (unsigned long long)gridDim.x * kPartThreads)
        a[c] = 0.0;
}

__global__ void __launch_bounds__(kPartThreads) k_part_flag_clear(int* __restrict__ bad) {
    if (threadIdx.x == 0) bad[0] = 0;
}

// ---- stable LSD radix sort of (key, index) pairs ----------------------------------
// One pass orders by the digit (key >> shift) & (kDigits - 1), keeping the order
// of equal digits: per tile of kSortTile pairs a block counts its digits
// (k_rs_count), one block turns the counts into each (digit, tile)'s first
// output position (k_rs_scan, digit-major so that lower tiles come first), and
// every block writes its pairs there in tile order (k_rs_scatter).
constexpr int kDigitBits = 10;
constexpr int kDigits = 1 << kDigitBits;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;

__global__ void __launch_bounds__(kSortThreads)
k_rs_count(int np, const unsigned* __restrict__ key, int shift, unsigned* __restrict__ counts) {
    __shared__ unsigned hist[kDigits];
    for (int d = threadIdx.x; d < kDigits; d += kSortThreads) hist[d] = 0u;
    __syncthreads();
    const int base = blockIdx.x * kSortTile;
    for (int it = 0; it < kSortItems; ++it) {
        const int e = base + it * kSortThreads + (int)threadIdx.x;
        if (e < np) atomicAdd(&hist[(key[e] >> shift) & (kDigits - 1)], 1u);  // integer: exact in any order
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kDigits; d += kSortThreads) counts[(size_t)d * gridDim.x + blockIdx.x] = hist[d];
}

// Exclusive prefix sums of the counts, digit-major: one block per digit scans
// that digit's per-tile counts in place (chunks of kSortThreads with a carry)
// and writes the digit's total; then one block turns the totals into each
// digit's first output position (k_rs_digits).  The scatter adds the two.
__global__ void __launch_bounds__(kSortThreads) k_rs_scan_tiles(unsigned* __restrict__ counts, int tiles,
                                                                unsigned* __restrict__ digit_tot) {
    __shared__ unsigned buf[kSortThreads];
    unsigned* c = counts + (size_t)blockIdx.x * tiles;
    unsigned carry = 0u;
    for (int t0 = 0; t0 < tiles; t0 += kSortThreads) {
        const int t = t0 + (int)threadIdx.x;
        const unsigned v = t < tiles ? c[t] : 0u;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kSortThreads; off <<= 1) {  // Hillis-Steele inclusive scan
            const unsigned u = threadIdx.x >= (unsigned)off ? buf[threadIdx.x - off] : 0u;
            __syncthreads();
            buf[threadIdx.x] += u;
            __syncthreads();
        }
        if (t < tiles) c[t] = carry + buf[threadIdx.x] - v;
        carry += buf[kSortThreads - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) digit_tot[blockIdx.x] = carry;
}

__global__ void __launch_bounds__(kDigits) k_rs_digits(unsigned* __restrict__ digit_tot) {
    __shared__ unsigned buf[kDigits];
    const unsigned v = digit_tot[threadIdx.x];
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kDigits; off <<= 1) {
        const unsigned u = threadIdx.x >= (unsigned)off ? buf[threadIdx.x - off] : 0u;
        __syncthreads();
        buf[threadIdx.x] += u;
        __syncthreads();
    }
    digit_tot[threadIdx.x] = buf[threadIdx.x] - v;  // exclusive
}

__global__ void __launch_bounds__(kSortThreads)
k_rs_scatter(int np, const unsigned* __restrict__ key, const unsigned* __restrict__ idx, int shift,
             const unsigned* __restrict__ start, const unsigned* __restrict__ digit_base,
             unsigned* __restrict__ key_out, unsigned* __restrict__ idx_out) {
    constexpr int kWaves = kSortThreads / 64;
    __shared__ unsigned run[kDigits];               // pairs of each digit this block has placed so far
    __shared__ unsigned wcnt[kWaves * kDigits];     // this round's count of each digit per wave
    for (int d = threadIdx.x; d < kDigits; d += kSortThreads)
        run[d] = digit_base[d] + start[(size_t)d * gridDim.x + blockIdx.x];
    for (int q = threadIdx.x; q < kWaves * kDigits; q += kSortThreads) wcnt[q] = 0u;
    __syncthreads();
    const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
    const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int base = blockIdx.x * kSortTile;
    for (int it = 0; it < kSortItems; ++it) {
        const int e = base + it * kSortThreads + (int)threadIdx.x;
        const bool valid = e < np;
        const unsigned k = valid ? key[e] : 0u;
        const unsigned d = (k >> shift) & (kDigits - 1);
        // lanes of this wave with the same digit: the AND over the digit's bits
        unsigned long long same = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < kDigitBits; ++bit) {
            const unsigned long long on = __ballot((d >> bit) & 1u);
            same &= ((d >> bit) & 1u) ? on : ~on;
        }
        const unsigned rank = (unsigned)__popcll(same & below);
        // the lowest lane of each digit group records the group's size
        if (valid && rank == 0u) wcnt[wave * kDigits + d] = (unsigned)__popcll(same);
        __syncthreads();
        if (valid) {
            unsigned pos = run[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w * kDigits + d];
            key_out[pos] = k;
            idx_out[pos] = idx[e];
        }
        __syncthreads();
        for (int dd = threadIdx.x; dd < kDigits; dd += kSortThreads) {
            unsigned add = 0u;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                add += wcnt[w * kDigits + dd];
                wcnt[w * kDigits + dd] = 0u;
            }
            run[dd] += add;
        }
        __syncthreads();
    }
}

// ---- run sums --------------------------------------------------------------------------
// Pieces: runs cut at every multiple of kPiece sorted positions.  The thread of
// positions [kPiece t, kPiece (t + 1)) sums each piece that starts in its range
// (at a run start or at kPiece t) in sorted order and stores the eight sums at
// the piece's first position; then the thread at each run start adds the run's
// pieces in order (its own, then those at the following multiples of kPiece).
constexpr int kPiece = 8;

__device__ __forceinline__ void corner_weights(const PartGeom& pg, const double* __restrict__ pos,
                                               const double* __restrict__ q, unsigned p, double (&w)[8]) {
    int i;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    (void)cell_frac(pos[3 * (size_t)p], pg.inv_hx, pg.nx, i, fx);
    (void)cell_frac(pos[3 * (size_t)p + 1], pg.inv_hy, pg.ny, i, fy);
    (void)cell_frac(pos[3 * (size_t)p + 2], pg.inv_hz, pg.nz, i, fz);
    const double qp = q ? q[p] : 1.0;
#pragma unroll
    for (int c = 0; c < 8; ++c)
        w[c] = qp * ((c & 1) ? fx : 1.0 - fx) * ((c & 2) ? fy : 1.0 - fy) * ((c & 4) ? fz : 1.0 - fz);
}

__global__ void __launch_bounds__(kPartThreads)
k_part_pieces(PartGeom pg, int np, const double* __restrict__ pos, const double* __restrict__ q,
              const unsigned* __restrict__ key_s, const unsigned* __restrict__ idx_s, double* __restrict__ psum) {
    const int t = blockIdx.x * kPartThreads + threadIdx.x;
    const int s0 = t * kPiece;
    if (s0 >= np) return;
    const int s1 = min(np, s0 + kPiece);
    double acc[8];
    int at = s0;
    unsigned kprev = key_s[s0];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.0;
    for (int s = s0; s < s1; ++s) {
        const unsigned k = key_s[s];
        if (k != kprev) {
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                psum[8 * (size_t)at + c] = acc[c];
                acc[c] = 0.0;
            }
            at = s;
            kprev = k;
        }
        double w[8];
        corner_weights(pg, pos, q, idx_s[s], w);
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] += w[c];
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) psum[8 * (size_t)at + c] = acc[c];
}

__global__ void __launch_bounds__(kPartThreads)
k_part_runs(int np, const unsigned* __restrict__ key_s, double* __restrict__ psum) {
    const int s = blockIdx.x * kPartThreads + threadIdx.x;
    if (s >= np) return;
    const unsigned k = key_s[s];
    if (s > 0 && key_s[s - 1] == k) return;
    int nxt = (s / kPiece + 1) * kPiece;
    if (nxt >= np || key_s[nxt] != k) return;  // a single piece: its sums are the run's
    double acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = psum[8 * (size_t)s + c];
    for (; nxt < np && key_s[nxt] == k; nxt += kPiece) {
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] += psum[8 * (size_t)nxt + c];
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) psum[8 * (size_t)s + c] = acc[c];
}

// First sorted position of each parity class (bound[8] = np): a binary search
// of the sorted keys per class.
__global__ void __launch_bounds__(64) k_part_bounds(int np, const unsigned* __restrict__ key_s, int cell_bits,
                                                   int* __restrict__ bound) {
    const int c = threadIdx.x;
    if (c > 8) return;
    const unsigned lo_key = (unsigned)c << cell_bits;
    int lo = 0, hi = np;  // first s with key_s[s] >= lo_key
    if (c == 8) lo = np;
    while (lo < hi) {
        const int mid = lo + (hi - lo) / 2;
        if (key_s[mid] < lo_key) lo = mid + 1;
        else hi = mid;
    }
    bound[c] = lo;
}

// Pass `color` of the eight: the runs of the cells (i, j, k) with parities
// (i, j, k) mod 2 = color, the sorted positions [bound[color], bound[color+1]),
// add their eight corner sums (over the cell volume) to the cells (i + a,
// j + b, k + e), wrapped.  Every length is even, so two runs of one class are
// two or more cells apart in some direction and their 2 x 2 x 2 footprints are
// disjoint: no two threads of a pass touch one cell, and each cell receives its
// contributions in the fixed order of the passes.
// (Keys without the class, on grids above 2^29 cells: every pass walks all the
// runs and takes those of its class.)
__global__ void __launch_bounds__(kPartThreads)
k_part_scatter(PartGeom pg, int np, const unsigned* __restrict__ key_s, const double* __restrict__ psum,
               const int* __restrict__ bound, int color, int cell_bits, double* __restrict__ out) {
    const bool keyed = cell_bits <= 29;
    const int s0 = keyed ? bound[color] : 0, s1 = keyed ? bound[color + 1] : np;
    const unsigned nx = pg.nx, ny = pg.ny, nz = pg.nz;
    const unsigned cmask = keyed ? (1u << cell_bits) - 1u : 0xffffffffu;
    for (int s = s0 + (int)(blockIdx.x * kPartThreads + threadIdx.x); s < s1; s += (int)(gridDim.x * kPartThreads)) {
        const unsigned key = key_s[s];
        if (s > s0 && key_s[s - 1] == key) continue;
        const unsigned cell = key & cmask;
        const unsigned i = cell % nx, j = (cell / nx) % ny, k = cell / (nx * ny);
        if (!keyed && (int)((i & 1u) | ((j & 1u) << 1) | ((k & 1u) << 2)) != color) continue;
        const unsigned i1 = i + 1 == nx ? 0u : i + 1, j1 = j + 1 == ny ? 0u : j + 1, k1 = k + 1 == nz ? 0u : k + 1;
        // the eight cells are distinct (every length is at least 4): all loads
        // are issued before any store, so the thread waits for memory once
        size_t c[8];
        double w[8], o[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            c[q] = ((size_t)((q & 4) ? k1 : k) * ny + ((q & 2) ? j1 : j)) * nx + ((q & 1) ? i1 : i);
            w[q] = psum[8 * (size_t)s + q];
            o[q] = out[c[q]];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) out[c[q]] = o[q] + w[q] * pg.inv_v;
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

static size_t up256(size_t b) { return (b + 255) & ~(size_t)255; }

static int sort_tiles(int np) { return (np + kSortTile - 1) / kSortTile; }

size_t particle_workspace_bytes(const GridArgs& g, int np) {
    (void)g;
    // keys, indices (two of each for the sort passes), piece and run sums, the
    // per-(digit, tile) counts, the digit totals, the bad-position flag
    return 4 * up256((size_t)np * 4) + up256((size_t)np * 64) +
           up256((size_t)kDigits * std::max(1, sort_tiles(np)) * 4) + up256((size_t)kDigits * 4) + 256;
}

hipError_t launch_deposit(const GridArgs& g, int np, const double* pos, const double* q, double* out, void* ws,
                          size_t ws_bytes, int* bad_host, hipStream_t s, hipStream_t s_aux, hipEvent_t ev_fork,
                          hipEvent_t ev_join) {
    if (ws_bytes < particle_workspace_bytes(g, np)) return hipErrorInvalidValue;
    const PartGeom pg = part_geom(g);
    char* w = static_cast<char*>(ws);
    const size_t kb = up256((size_t)np * 4);
    unsigned* key = reinterpret_cast<unsigned*>(w);
    unsigned* idx = reinterpret_cast<unsigned*>(w + kb);
    unsigned* key2 = reinterpret_cast<unsigned*>(w + 2 * kb);
    unsigned* idx2 = reinterpret_cast<unsigned*>(w + 3 * kb);
    double* psum = reinterpret_cast<double*>(w + 4 * kb);
    unsigned* counts = reinterpret_cast<unsigned*>(w + 4 * kb + up256((size_t)np * 64));
    const size_t cb = up256((size_t)kDigits * std::max(1, sort_tiles(np)) * 4);
    unsigned* digit_tot = reinterpret_cast<unsigned*>(w + 4 * kb + up256((size_t)np * 64) + cb);
    int* bad = reinterpret_cast<int*>(w + 4 * kb + up256((size_t)np * 64) + cb + up256((size_t)kDigits * 4));
    int* bound = bad + 16;  // nine class bounds after the flag, in the same 256 bytes
    const unsigned long long n = (unsigned long long)g.n;
    const int pb = (np + kPartThreads - 1) / kPartThreads;
    const int cell_bits = key_bits(g.n);
    hipError_t e;
    k_part_flag_clear<<<1, 64, 0, s>>>(bad);
    if (np > 0) {
        k_part_keys<<<pb, kPartThreads, 0, s>>>(pg, np, pos, key, idx, bad, cell_bits);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        int flag = 0;
        if ((e = hipMemcpyAsync(&flag, bad, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        if (flag) {
            *bad_host = 1;
            return hipSuccess;
        }
    }
    // the zero fill (bandwidth) runs on the second stream while the sort and the
    // run sums (latency) run on the first; the scatter passes wait for both
    const unsigned zb = (unsigned)std::min<unsigned long long>((n + kPartThreads - 1) / kPartThreads, 8192ull);
    if ((e = hipEventRecord(ev_fork, s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s_aux, ev_fork, 0)) != hipSuccess) return e;
    k_part_zero<<<zb, kPartThreads, 0, s_aux>>>(out, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipEventRecord(ev_join, s_aux)) != hipSuccess) return e;
    if (np > 0) {
        const int tiles = sort_tiles(np);
        const int bits = cell_bits <= 29 ? cell_bits + 3 : cell_bits;
        for (int shift = 0; shift < bits; shift += kDigitBits) {
            k_rs_count<<<tiles, kSortThreads, 0, s>>>(np, key, shift, counts);
            k_rs_scan_tiles<<<kDigits, kSortThreads, 0, s>>>(counts, tiles, digit_tot);
            k_rs_digits<<<1, kDigits, 0, s>>>(digit_tot);
            k_rs_scatter<<<tiles, kSortThreads, 0, s>>>(np, key, idx, shift, counts, digit_tot, key2, idx2);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            std::swap(key, key2);
            std::swap(idx, idx2);
        }
        const int nb_pieces = ((np + kPiece - 1) / kPiece + kPartThreads - 1) / kPartThreads;
        k_part_pieces<<<nb_pieces, kPartThreads, 0, s>>>(pg, np, pos, q, key, idx, psum);
        k_part_runs<<<pb, kPartThreads, 0, s>>>(np, key, psum);
        if (cell_bits <= 29) k_part_bounds<<<1, 64, 0, s>>>(np, key, cell_bits, bound);
    }
    if ((e = hipStreamWaitEvent(s, ev_join, 0)) != hipSuccess) return e;
    if (np > 0) {
        // about a class's share of the particles per pass (at least one block)
        const int sb = cell_bits <= 29 ? std::max(1, std::min(pb / 8 + 1, 2048)) : std::max(1, std::min(pb, 8192));
        for (int c = 0; c < 8; ++c)
            k_part_scatter<<<sb, kPartThreads, 0, s>>>(pg, np, key, psum, bound, c, cell_bits, out);
    }
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
