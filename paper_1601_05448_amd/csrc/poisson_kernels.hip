// gfx950 kernels of the variable-density pressure Poisson solve and their
// launchers.
//
// One iteration of the paper's method (section "Poisson equation", eq. (Pois):
// p = p_g + dp, drop rho grad(1/rho).grad dp, solve the constant-coefficient
// equation by transforms in the periodic directions, p_g <- p_g + dp) is, in
// residual form,
//     r = b~ - A p,  q = w r,  dp = L^+ q,  p += dp,
// and runs as five sweeps over the field:
//   P1 k_resid_dhtx   stencil residual, weight, partial norms, Hartley along x -> W;
//                     its last block takes ||r|| / ||b~|| and the decision
//                     (convergence, divergence, iteration cap; poisson_control.hpp)
//   P2 k_dht_cols<Y>  Hartley along y of W
//   P3 k_dht_z_solve  Hartley along z, divide by n * symbol, Hartley along z
//   P4 k_dht_cols<Y>  Hartley along y
//   P5 k_dhtx_update  Hartley along x, p += dp
// Every sweep first reads the solve's `done` flag and returns when the solve is
// over, so a stream or graph may hold more iterations than are needed.
//
// Batching: blockIdx.y selects the solve (slot) of a batch of equal-size grids.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "poisson_control.hpp"
#include "poisson_device.hpp"

namespace pois {

// ---- setup ------------------------------------------------------------------------

constexpr int kPtThreads = 256;

__global__ void __launch_bounds__(256) k_init(const Slot* __restrict__ slots, double inner_tol, int max_iter,
                                             int max_outer, int precision) {
    SolveState* st = slots[blockIdx.x].st;
    // zero the whole record with vector stores, then set the parameters
    unsigned long long* w = reinterpret_cast<unsigned long long*>(st);
    constexpr int words = (int)(sizeof(SolveState) / sizeof(unsigned long long));
    for (int q = threadIdx.x; q < words; q += 256) w[q] = 0ull;
    __syncthreads();
    if (threadIdx.x != 0) return;
    st->tol = slots[blockIdx.x].tol;
    st->inner_tol = inner_tol;
    st->inner_goal = inner_tol;
    st->max_iter = max_iter;
    st->max_outer = max_outer;
    st->precision = precision;
    st->status = POISSON_OK;
    st->inv_s = 1.0;
}

// rho: min, max, validity; b: sum, sum of squares, validity; optional FP32 copy of rho.
__global__ void __launch_bounds__(kPtThreads)
k_setup(GridArgs g, const Slot* __restrict__ slots, int write_rho32) {
    __shared__ double red[(kPtThreads / 64) * 5];
    const Slot& s = slots[blockIdx.y];
    double sb = 0.0, sb2 = 0.0, mn = INFINITY, mx = -INFINITY, bad = 0.0;
    const long long stride = (long long)gridDim.x * kPtThreads;
    auto cell = [&](long long c, double r, double b) {
        if (!(r > 0.0) || !isfinite(r) || !isfinite(b)) bad += 1.0;
        mn = fmin(mn, r);
        mx = fmax(mx, r);
        sb += b;
        sb2 += b * b;
        if (write_rho32) gptr(s.rho32)[c] = (float)r;
    };
    // four cells' loads in flight per thread, the sums taken in the same order
    // as one cell at a time
    constexpr int kU = 4;
    long long c = (long long)blockIdx.x * kPtThreads + threadIdx.x;
    for (; c + (kU - 1) * stride < g.n; c += kU * stride) {
        double r[kU], b[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            r[u] = gptr(s.rho)[c + u * stride];
            b[u] = gptr(s.b)[c + u * stride];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) cell(c + u * stride, r[u], b[u]);
    }
    for (; c < g.n; c += stride) cell(c, gptr(s.rho)[c], gptr(s.b)[c]);
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    sb = wave_sum(sb); sb2 = wave_sum(sb2); bad = wave_sum(bad);
    mn = wave_min(mn); mx = wave_max(mx);
    if (lane == 0) {
        red[w * 5 + 0] = sb; red[w * 5 + 1] = sb2; red[w * 5 + 2] = mn; red[w * 5 + 3] = mx;
        red[w * 5 + 4] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int u = 1; u < kPtThreads / 64; ++u) {
            sb += red[u * 5 + 0]; sb2 += red[u * 5 + 1]; mn = fmin(mn, red[u * 5 + 2]);
            mx = fmax(mx, red[u * 5 + 3]); bad += red[u * 5 + 4];
        }
        double* out = s.partial + (long long)blockIdx.x * 8;
        out[0] = sb; out[1] = sb2; out[2] = mn; out[3] = mx; out[4] = bad;
    }
}

__device__ double pow2_near(double x) {
    // nearest power of two to x (x > 0, finite), else 1
    if (!(x > 0.0) || !isfinite(x)) return 1.0;
    return ldexp(1.0, (int)lrint(log2(x)));
}

__global__ void __launch_bounds__(256) k_setup_finalize(GridArgs g, const Slot* __restrict__ slots, int nblk) {
    __shared__ double red[4 * 5];
    const Slot& s = slots[blockIdx.x];
    SolveState* st = s.st;
    double sb = 0.0, sb2 = 0.0, mn = INFINITY, mx = -INFINITY, bad = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) {
        const double* in = s.partial + (long long)b * 8;
        sb += in[0]; sb2 += in[1]; mn = fmin(mn, in[2]); mx = fmax(mx, in[3]); bad += in[4];
    }
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    sb = wave_sum(sb); sb2 = wave_sum(sb2); bad = wave_sum(bad);
    mn = wave_min(mn); mx = wave_max(mx);
    if (lane == 0) {
        red[w * 5 + 0] = sb; red[w * 5 + 1] = sb2; red[w * 5 + 2] = mn; red[w * 5 + 3] = mx;
        red[w * 5 + 4] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int u = 1; u < 4; ++u) {
            sb += red[u * 5 + 0]; sb2 += red[u * 5 + 1]; mn = fmin(mn, red[u * 5 + 2]);
            mx = fmax(mx, red[u * 5 + 3]); bad += red[u * 5 + 4];
        }
        st->b_mean = sb / (double)g.n;
        st->b_sumsq = sb2;
        st->rho_min = mn;
        st->rho_max = mx;
        st->bad = bad > 0.0;
        // scale of the first FP32 right-hand side: near the RMS of b
        st->inv_s = 1.0 / pow2_near(sqrt(sb2 / (double)g.n));
        // density ratio the scaled batched reciprocals of the sweeps support
        const double max_ratio = (st->precision == POISSON_FP32_REFINE) ? 1e8 : 1e20;
        if (!(mx <= max_ratio * mn)) bad += 1.0;
        if (bad > 0.0) {
            st->done = 1;
            st->status = POISSON_EDOMAIN;
        }
    }
}

// ---- decisions (one block per solve, after the sweep that wrote the sums) -------------

// One block of kDecideThreads per solve: the units' sums of a residual sweep
// (up to one per row pair) are read by many threads at once.
constexpr int kDecideThreads = 1024;

// After P1 of an iteration: FP64 path (fp32 = 0) or an FP32 inner sweep.
__global__ void __launch_bounds__(kDecideThreads) k_decide_iter(GridArgs g, const Slot* __restrict__ slots,
                                                                int nunits, int fp32) {
    __shared__ double red[(kDecideThreads / 64) * 4];
    const Slot& s = slots[blockIdx.x];
    SolveState* st = s.st;
    if (fp32 ? (st->done || st->stage != 1 || st->inner_done || st->upd_due) : st->done) return;
    double sums[4] = {0.0, 0.0, 0.0, 0.0};
    if (!(fp32 && st->stop_next)) sum_units<kDecideThreads, 4>(s.partial, (unsigned)nunits, sums, red);
    if (threadIdx.x != 0) return;
    if (fp32) decide_inner(st, sums, kMaxInnerPerStep);
    else decide_fp64(g, st, sums);
}

// After the FP64 outer residual of a refinement step.  mode 0: the residual
// alone (r32 written), 1: fused with the first inner sweep's residual, 2: its
// sums alone (a check: no step starts from it).
__global__ void __launch_bounds__(kDecideThreads) k_decide_outer(GridArgs g, const Slot* __restrict__ slots,
                                                                 int nunits, int mode) {
    __shared__ double red[(kDecideThreads / 64) * 5];
    const Slot& s = slots[blockIdx.x];
    SolveState* st = s.st;
    if (st->done || st->stage != 0) return;
    double sums[5];
    sum_units<kDecideThreads, 5>(s.partial, (unsigned)nunits, sums, red);
    if (threadIdx.x == 0) decide_outer(g, st, sums, mode == 1, mode == 2);
}

// After the rest of a fused first inner sweep: the inner sweeps go on.
__global__ void __launch_bounds__(64) k_tail_done(const Slot* __restrict__ slots) {
    SolveState* st = slots[blockIdx.x].st;
    if (threadIdx.x == 0 && !st->done && st->stage == kStageTail) st->stage = 1;
}

// ---- pointwise FP64 stencil sweeps -------------------------------------------------
// MODE 0: out = A p (apply).  MODE 1: r = b~ - A p into a FP64 field with partial
// norms (stand-alone residual).  Partials: sum r^2, sum bt^2, sum p, sum p^2, sum r.
template <int MODE>
__global__ void __launch_bounds__(kPtThreads)
k_stencil(GridArgs g, const Slot* __restrict__ slots, const double* __restrict__ rho_in,
          const double* __restrict__ p_in, double* __restrict__ out) {
    __shared__ double red[(kPtThreads / 64) * 5];
    const Slot* sp = slots ? &slots[blockIdx.y] : nullptr;
    const POIS_GLOBAL double* rho = gptr((MODE == 0) ? rho_in : sp->rho);
    const POIS_GLOBAL double* p = gptr((MODE == 0) ? p_in : sp->p);
    const POIS_GLOBAL double* b = (MODE == 0) ? nullptr : gptr(sp->b);
    POIS_GLOBAL double* og = out ? gptr(out) : nullptr;
    const double bm = (MODE == 0) ? 0.0 : sp->st->b_mean;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    // rows of x: a block pass covers rpp rows (several short rows, or one long row
    // that each thread strides over); row -> (j, k) is decoded once per row
    const unsigned nx = g.nx, nrows = (unsigned)(g.ny * g.nz);
    const unsigned rpp = nx >= kPtThreads ? 1u : kPtThreads / nx;
    const unsigned tr = nx >= kPtThreads ? 0u : threadIdx.x / nx;
    const unsigned ti = nx >= kPtThreads ? threadIdx.x : threadIdx.x - tr * nx;
    const unsigned istep = nx >= kPtThreads ? kPtThreads : nx;
    for (unsigned r = blockIdx.x * rpp + tr; tr < rpp && r < nrows; r += gridDim.x * rpp)
    for (unsigned i = ti; i < nx; i += istep) {
        const unsigned c = r * nx + i;
        const int j = (int)(r % (unsigned)g.ny), k = (int)(r / (unsigned)g.ny);
        if (MODE == 0) {
            // with no right-hand side the residual is -A p
            const CellOut<double> o = cell_residual<double>(g, p, rho, nullptr, 0.0, i, j, k);
            og[c] = -o.r;
        } else {
            const CellOut<double> o = cell_residual<double>(g, p, rho, b, bm, i, j, k);
            acc[0] += o.r * o.r;
            acc[1] += o.bt * o.bt;
            acc[2] += o.pc;
            acc[3] += o.pc * o.pc;
            acc[4] += o.r;
            if (og) og[c] = o.r;
        }
    }
    if (MODE != 0) {
        block_sums<kPtThreads, 5>(acc, red);
        if (threadIdx.x == 0) {
            double* o = sp->partial + (long long)blockIdx.x * kPartialStride;
            o[0] = acc[0]; o[1] = acc[1]; o[2] = acc[2]; o[3] = acc[3]; o[4] = acc[4];
        }
    }
}

// FP32_REFINE outer residual in FP64: r = b~ - A p, r32 = r inv_s, d32 = 0, by
// z-marching columns (see ZMarch) over tiles of kOuterPlanes planes x SUB row
// pairs (rows of the lengths OuterCfg accepts; others take k_outer_resid_rows).  Partials:
// sum r^2, sum bt^2, sum p, sum p^2, sum r.
constexpr int kOuterPlanes = 16;

// 256 threads: SUB = 256 / N strips of one column per thread, or CPT = N / 256
// columns per thread; rows whose length divides or is a multiple of 256.
template <int N>
struct OuterCfg {
    static constexpr bool ok = N % 64 == 0 && (N >= 256 ? N % 256 == 0 : 256 % N == 0);
    static constexpr int CPT = N >= 256 ? N / 256 : 1;
    static constexpr int SUB = N >= 256 ? 1 : 256 / N;
};

template <int N, int COEF, int WEIGHT>
__global__ void __launch_bounds__(256) k_outer_resid(GridArgs g, const Slot* __restrict__ slots) {
    using O = OuterCfg<N>;
    constexpr int EDGE = (N / 64) * 2 * 4;
    __shared__ double red[(256 / 64) * 5];
    __shared__ double edge[2 * O::SUB * EDGE];
    const Slot& s = slots[blockIdx.y];
    SolveState* st = s.st;
    if (st->done || st->stage != 0) return;
    const double bm = st->b_mean, inv_s = st->inv_s, rmax = st->rho_max, rinv = recip(st->rho_max);
    const unsigned nyh = (unsigned)g.ny / 2, nz = (unsigned)g.nz;
    const unsigned ngj = (nyh + O::SUB - 1) / O::SUB, ngk = (nz + kOuterPlanes - 1) / kOuterPlanes;
    const unsigned ntiles = ngj * ngk;
    const int sidx = (N >= 256) ? 0 : (int)threadIdx.x / N;
    const unsigned col0 = (N >= 256) ? threadIdx.x : threadIdx.x % N;
    POIS_GLOBAL float* r32 = gptr(s.r32);
    POIS_GLOBAL float* d32 = gptr(s.d32);
    ZMarch<double> zm;
    zm.p = s.p;
    zm.rho = s.rho;
    zm.rhs = s.b;
    zm.nx = (unsigned)g.nx;
    zm.nz = nz;
    zm.sz = (unsigned)g.nx * (unsigned)g.ny;
    zm.lane = (int)(threadIdx.x & 63);
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (unsigned tile = xcd_block(blockIdx.x, gridDim.x); tile < ntiles; tile += gridDim.x) {
        const unsigned tj = tile % ngj, tk = tile / ngj;
        const unsigned jp = tj * O::SUB + sidx;
        const bool jvalid = jp < nyh;
        zm.rows_of(jvalid ? jp : 0u, (unsigned)g.ny);
        const int k0 = (int)(tk * kOuterPlanes);
        PlaneRows<double> pl[O::CPT][3];
        PlaneSide<double> sd[O::CPT];
#pragma unroll
        for (int c = 0; c < O::CPT; ++c) {
            const unsigned i = col0 + c * 256;
            zm.load_rows(zm.plane(k0 - 1), i, pl[c][0]);
            zm.load_rows(zm.plane(k0), i, pl[c][1]);
            zm.load_rows(zm.plane(k0 + 1), i, pl[c][2]);
            zm.load_side(zm.plane(k0), i, sd[c]);
        }
#pragma unroll
        for (int kk = 0; kk < kOuterPlanes; ++kk) {
            const int k = k0 + kk;
            const bool valid = jvalid && k < (int)nz;
            PlaneRows<double> nn[O::CPT];
            PlaneSide<double> ns[O::CPT];
#pragma unroll
            for (int c = 0; c < O::CPT; ++c) {
                const unsigned i = col0 + c * 256;
                zm.load_rows(zm.plane(k + 2), i, nn[c]);
                zm.load_side(zm.plane(k + 1), i, ns[c]);
            }
            double* eb = edge + ((kk & 1) * O::SUB + sidx) * EDGE;
#pragma unroll
            for (int c = 0; c < O::CPT; ++c) zm.edge_put(eb, col0 + c * 256, pl[c][1]);
            __syncthreads();
#pragma unroll
            for (int c = 0; c < O::CPT; ++c) {
                const unsigned i = col0 + c * 256;
                PairIn<double> in;
                zm.pair(pl[c][0], pl[c][1], pl[c][2], sd[c], zm.edge_get(eb, i), in);
                if (valid) {
                    const PairOut<double> pr = pair_eval<double, COEF, WEIGHT>(g, in, bm, rmax, rinv, x_walls(g, i));
                    const unsigned a = (unsigned)k * zm.sz + zm.ra + i, b = a + (unsigned)g.nx;
                    acc[0] += pr.a.r * pr.a.r + pr.b.r * pr.b.r;
                    acc[1] += pr.a.bt * pr.a.bt + pr.b.bt * pr.b.bt;
                    acc[2] += pr.a.pc + pr.b.pc;
                    acc[3] += pr.a.pc * pr.a.pc + pr.b.pc * pr.b.pc;
                    acc[4] += pr.a.r + pr.b.r;
                    r32[a] = (float)(pr.a.r * inv_s);
                    r32[b] = (float)(pr.b.r * inv_s);
                    d32[a] = 0.0f;
                    d32[b] = 0.0f;
                }
            }
#pragma unroll
            for (int c = 0; c < O::CPT; ++c) {
                pl[c][0] = pl[c][1];
                pl[c][1] = pl[c][2];
                pl[c][2] = nn[c];
                sd[c] = ns[c];
            }
        }
        put_unit_sums<256, 5>(acc, red, s.partial + (unsigned long long)tile * kPartialStride);
    }
}

// The same for rows of any length: row pairs gathered with all their neighbours
// (the layout of P1's line groups), one pair evaluated while the next one's
// loads are in flight.
constexpr int kOuterElems = 2048;  // (pair, column) elements per block

template <int N, int COEF, int WEIGHT>
__global__ void __launch_bounds__(kPtThreads) k_outer_resid_rows(GridArgs g, const Slot* __restrict__ slots) {
    constexpr int RPB = N >= kOuterElems ? 1 : kOuterElems / N;  // row pairs per block
    __shared__ double red[(kPtThreads / 64) * 5];
    __shared__ int s_j0[RPB], s_k0[RPB];
    const Slot& s = slots[blockIdx.y];
    SolveState* st = s.st;
    if (st->done || st->stage != 0) return;
    const unsigned npairs = (unsigned)(g.ny * g.nz / 2);
    const unsigned pair0 = blockIdx.x * RPB;
    for (int l = threadIdx.x; l < RPB; l += kPtThreads) {
        const unsigned r0 = 2u * (pair0 + l);
        s_j0[l] = (int)(r0 % (unsigned)g.ny);
        s_k0[l] = (int)(r0 / (unsigned)g.ny);
    }
    __syncthreads();
    const double bm = st->b_mean, inv_s = st->inv_s, rmax = st->rho_max, rinv = recip(st->rho_max);
    const POIS_GLOBAL double* p = gptr(s.p);
    const POIS_GLOBAL double* rho = gptr(s.rho);
    const POIS_GLOBAL double* rhs = gptr(s.b);
    POIS_GLOBAL float* r32 = gptr(s.r32);
    POIS_GLOBAL float* d32 = gptr(s.d32);
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    constexpr int IT = (RPB * N + kPtThreads - 1) / kPtThreads;  // elements per thread
    auto fetch = [&](int it, PairIn<double>& in) {
        const int e = threadIdx.x + it * kPtThreads;
        const int l = e / N;
        if (e < RPB * N && pair0 + l < npairs) {
            pair_fetch<double>(g, p, rho, rhs, e % N, s_j0[l], s_k0[l], in);
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                in.r[k] = 1.0;
                in.q[k] = 0.0;
            }
            in.ba = in.bb = 0.0;
        }
    };
    auto evaluate = [&](int it, const PairIn<double>& in) {
        const int e = threadIdx.x + it * kPtThreads;
        const int l = e / N, i = e % N;
        const unsigned P = pair0 + l;
        if (e >= RPB * N || P >= npairs) return;
        const PairOut<double> pr = pair_eval<double, COEF, WEIGHT>(g, in, bm, rmax, rinv, x_walls(g, i));
        const unsigned a = (2 * P) * N + i, b = a + N;
        acc[0] += pr.a.r * pr.a.r + pr.b.r * pr.b.r;
        acc[1] += pr.a.bt * pr.a.bt + pr.b.bt * pr.b.bt;
        acc[2] += pr.a.pc + pr.b.pc;
        acc[3] += pr.a.pc * pr.a.pc + pr.b.pc * pr.b.pc;
        acc[4] += pr.a.r + pr.b.r;
        r32[a] = (float)(pr.a.r * inv_s);
        r32[b] = (float)(pr.b.r * inv_s);
        d32[a] = 0.0f;
        d32[b] = 0.0f;
    };
    // one row pair evaluated while the next one's loads are in flight
    PairIn<double> A, B;
    fetch(0, A);
    for (int it = 0; it < IT; it += 2) {
        if (it + 1 < IT) fetch(it + 1, B);
        evaluate(it, A);
        if (it + 2 < IT) fetch(it + 2, A);
        if (it + 1 < IT) evaluate(it + 1, B);
    }
    put_unit_sums<kPtThreads, 5>(acc, red, s.partial + (unsigned long long)blockIdx.x * kPartialStride);
}

template <int N>
static int blocks_outer(const GridArgs& g) {
    if constexpr (OuterCfg<N>::ok) {
        using O = OuterCfg<N>;
        const long long ngj = ((long long)g.ny / 2 + O::SUB - 1) / O::SUB;
        const long long ngk = ((long long)g.nz + kOuterPlanes - 1) / kOuterPlanes;
        return (int)std::min<long long>(ngj * ngk, 2048);
    } else {
        constexpr int RPB = N >= kOuterElems ? 1 : kOuterElems / N;
        const long long np = (long long)g.ny * g.nz / 2;
        return (int)((np + RPB - 1) / RPB);
    }
}

// partial sums the outer residual writes: one per tile (z kernel) or per block
template <int N>
static int outer_units(const GridArgs& g) {
    if constexpr (OuterCfg<N>::ok) {
        using O = OuterCfg<N>;
        const long long ngj = ((long long)g.ny / 2 + O::SUB - 1) / O::SUB;
        const long long ngk = ((long long)g.nz + kOuterPlanes - 1) / kOuterPlanes;
        return (int)(ngj * ngk);
    } else {
        return blocks_outer<N>(g);
    }
}


// FP32_REFINE outer update: p += d32 / inv_s - p_shift (FP64), then the next scale.
__global__ void __launch_bounds__(kPtThreads) k_outer_update(GridArgs g, const Slot* __restrict__ slots) {
    const Slot& s = slots[blockIdx.y];
    const SolveState* st = s.st;
    if (st->done || st->stage != 2) return;
    const double scale = 1.0 / st->inv_s;
    // mean of the current p (FP64 sum of the outer residual sweep): removing it
    // here keeps p zero-mean although the FP32 correction is not exactly so
    const double shift = st->p_sum / (double)g.n;
    const unsigned n = (unsigned)g.n, stride = gridDim.x * kPtThreads;
    for (unsigned c = blockIdx.x * kPtThreads + threadIdx.x; c < n; c += stride)
        gptr(s.p)[c] = gptr(s.p)[c] + (double)gptr(s.d32)[c] * scale - shift;
}

// One block per slot: between the outer update and the next outer residual.
__global__ void __launch_bounds__(64) k_outer_advance(GridArgs g, const Slot* __restrict__ slots) {
    SolveState* st = slots[blockIdx.x].st;
    if (st->done || st->stage != 2 || threadIdx.x != 0) return;
    st->stage = 0;
    // predicted size of the next FP64 residual: ||r|| times the inner reduction
    const double est = st->r_norm * fmax(st->rel_in, 1e-30);
    st->inv_s = 1.0 / pow2_near(est / sqrt((double)g.n));
    st->iter += 1;
}

// End of a solve: remove the mean of p if no update did, or zero p when b~ = 0.
__global__ void __launch_bounds__(kPtThreads) k_fixup(GridArgs g, const Slot* __restrict__ slots) {
    const Slot& s = slots[blockIdx.y];
    const SolveState* st = s.st;
    if (st->status == POISSON_EDOMAIN) return;
    const bool zero = st->b_norm == 0.0 && st->done && st->status == POISSON_OK;
    // the first update removes p_shift; a solve that ends before any update
    // (iter == 0 on both paths) still has to
    const bool shift_left = st->iter == 0 && st->p_shift != 0.0;
    if (!zero && !shift_left) return;
    const double sh = st->p_shift;
    const long long stride = (long long)gridDim.x * kPtThreads;
    for (long long c = (long long)blockIdx.x * kPtThreads + threadIdx.x; c < g.n; c += stride)
        gptr(s.p)[c] = zero ? 0.0 : gptr(s.p)[c] - sh;
}

// A solve that the host driver stopped driving before it reached a terminal
// status (its rounds ran out) ends with the status of the iteration cap; p is
// the last iterate its updates left.
__global__ void __launch_bounds__(64) k_stop_unfinished(const Slot* __restrict__ slots) {
    if (threadIdx.x != 0) return;
    SolveState* st = slots[blockIdx.x].st;
    if (!st->done) {
        st->done = 1;
        st->status = POISSON_ENOCONV;
    }
}

// ---- launch helpers ------------------------------------------------------------------

bool length_supported(int n) {
    if (n < 4 || n > 1024) return false;
    int m = n;
    if (m % 3 == 0) m /= 3;
    return (m & (m - 1)) == 0 && m >= 1 && (n % 2 == 0);
}

static int pt_blocks(const GridArgs& g) {
    const long long b = (g.n + kPtThreads - 1) / kPtThreads;
    return (int)(b < 4096 ? b : 4096);
}

Geometry make_geometry(const GridArgs& g) {
    Geometry geo{};
    geo.blocks_x = (int)sweep_groups_x(g);
    geo.blocks_pt = pt_blocks(g);
    int nbo = 0;
    (void)dispatch_len(g.nx, [&]<int N>() {
        nbo = blocks_outer<N>(g);
        return hipSuccess;
    });
    geo.blocks_outer = nbo;
    // partial sums: one set per block of the set-up and pointwise sweeps, per
    // tile or line group of the residual sweeps (at most one per row pair)
    const int row_pairs = (int)((long long)g.ny * g.nz / 2);
    geo.max_blocks = std::max(std::max(std::max(std::max(geo.blocks_x, geo.blocks_pt), nbo), kMaxSetupBlocks),
                              row_pairs);
    geo.share = 1.0f;
    return geo;
}

hipError_t launch_init(const GridArgs& g, const Slot* slots, int nslots, double inner_tol, int max_iter,
                       int max_outer, int precision, hipStream_t s) {
    (void)g;
    k_init<<<nslots, 256, 0, s>>>(slots, inner_tol, max_iter, max_outer, precision);
    return hipGetLastError();
}

hipError_t launch_setup(const GridArgs& g, const Geometry& geo, const Slot* slots, int nslots, bool write_rho32,
                        hipStream_t s) {
    (void)geo;
    const int nb = std::min(pt_blocks(g), kMaxSetupBlocks);
    k_setup<<<dim3(nb, nslots), kPtThreads, 0, s>>>(g, slots, write_rho32 ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_setup_finalize(const GridArgs& g, const Geometry& geo, const Slot* slots, int nslots,
                                 hipStream_t s) {
    (void)geo;
    const int nb = std::min(pt_blocks(g), kMaxSetupBlocks);
    k_setup_finalize<<<nslots, 256, 0, s>>>(g, slots, nb);
    return hipGetLastError();
}

// P1, convergence check, P2, P3, P4 (= P2), P5.  MODE 1 is the stand-alone
// L^+ q sweep (q in slot.b, result in slot.p), which has no check.
// parts: 1 the residual sweep and its decision only (an evaluation), 2 the
// four transform sweeps only (the update of an evaluation), 3 both
static hipError_t five_sweeps(const GridArgs& g, const Tables& t, const Slot* slots, int nslots, bool fp32,
                              int mode, hipStream_t s, SweepTimer* tm, float share = 1.0f, int parts = 3) {
    hipError_t e;
    int nunits = 0;
    // one sweep, bracketed by the timer's events when it times this sweep
    auto sweep = [&](int which) -> hipError_t {
        const bool timed = tm && tm->sweep == which && tm->fp32 == fp32 && tm->used < SweepTimer::kCap;
        if (timed && (e = hipEventRecord(tm->ev[2 * tm->used], s)) != hipSuccess) return e;
        if ((e = launch_sweep_mode(g, t, slots, nslots, fp32, which, mode, s, which == 1 ? &nunits : nullptr,
                                   share)) != hipSuccess)
            return e;
        if (timed) {
            if ((e = hipEventRecord(tm->ev[2 * tm->used + 1], s)) != hipSuccess) return e;
            ++tm->used;
        }
        return hipSuccess;
    };
    if (parts & 1) {
        if ((e = sweep(1)) != hipSuccess) return e;
        if (mode == 0) {
            k_decide_iter<<<nslots, kDecideThreads, 0, s>>>(g, slots, nunits, fp32 ? 1 : 0);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
    }
    if (!(parts & 2)) return hipSuccess;
    if ((e = sweep(2)) != hipSuccess) return e;
    if ((e = sweep(3)) != hipSuccess) return e;
    if ((e = sweep(2)) != hipSuccess) return e;
    return sweep(5);
}

hipError_t launch_sweep(const GridArgs& g, const Tables& t, const Slot* slots, int nslots, bool fp32, int which,
                        hipStream_t s) {
    return launch_sweep_mode(g, t, slots, nslots, fp32, which, 0, s, nullptr);
}

hipError_t launch_iteration(const GridArgs& g, const Geometry& geo, const Tables& t, const Slot* slots,
                            int nslots, bool fp32, hipStream_t s, SweepTimer* tm) {
    return five_sweeps(g, t, slots, nslots, fp32, 0, s, tm, geo.share);
}

hipError_t launch_evaluation(const GridArgs& g, const Geometry& geo, const Tables& t, const Slot* slots,
                             int nslots, hipStream_t s, SweepTimer* tm) {
    return five_sweeps(g, t, slots, nslots, true, 0, s, tm, geo.share, 1);
}

hipError_t launch_inner_update(const GridArgs& g, const Geometry& geo, const Tables& t, const Slot* slots,
                               int nslots, hipStream_t s, SweepTimer* tm) {
    return five_sweeps(g, t, slots, nslots, true, 0, s, tm, geo.share, 2);
}

hipError_t launch_outer_resid_sweep(const GridArgs& g, const Slot* slots, int nslots, hipStream_t s, int* nunits) {
    return dispatch_len(g.nx, [&]<int N>() {
        const int nb = blocks_outer<N>(g);
        if (nunits) *nunits = outer_units<N>(g);
        return dispatch_op(g.coef, g.weight, [&]<int C, int W>() {
            if constexpr (OuterCfg<N>::ok) k_outer_resid<N, C, W><<<dim3(nb, nslots), 256, 0, s>>>(g, slots);
            else k_outer_resid_rows<N, C, W><<<dim3(nb, nslots), kPtThreads, 0, s>>>(g, slots);
            return hipGetLastError();
        });
    });
}

hipError_t launch_outer_tail(const GridArgs& g, const Geometry& geo, const Tables& t, const Slot* slots,
                             int nslots, hipStream_t s) {
    hipError_t e;
    for (int which : {2, 3, 2, 5})
        if ((e = launch_sweep_mode(g, t, slots, nslots, true, which, 0, s, nullptr, geo.share, kStageTail)) !=
            hipSuccess)
            return e;
    k_tail_done<<<nslots, 64, 0, s>>>(slots);
    return hipGetLastError();
}

hipError_t launch_outer_residual(const GridArgs& g, const Geometry& geo, const Tables& t, const Slot* slots,
                                 int nslots, hipStream_t s, bool* fused, bool tail) {
    int nu = 0;
    hipError_t e;
    const bool fu = outer_fusable(g);
    if (fused) *fused = fu;
    if (fu) {
        if ((e = launch_outer_fused(g, t, slots, nslots, s, &nu, geo.share, tail)) != hipSuccess) return e;
    } else if ((e = launch_outer_resid_sweep(g, slots, nslots, s, &nu)) != hipSuccess) {
        return e;
    }
    k_decide_outer<<<nslots, kDecideThreads, 0, s>>>(g, slots, nu, fu ? (tail ? 1 : 2) : 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (!fu || !tail) return hipSuccess;
    // the rest of the first inner sweep: P2, P3, P4, P5 (which stores dp as d32)
    return launch_outer_tail(g, geo, t, slots, nslots, s);
}

hipError_t launch_outer_update(const GridArgs& g, const Geometry& geo, const Slot* slots, int nslots,
                               hipStream_t s) {
    k_outer_update<<<dim3(geo.blocks_pt, nslots), kPtThreads, 0, s>>>(g, slots);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_outer_advance<<<nslots, 64, 0, s>>>(g, slots);
    return hipGetLastError();
}

hipError_t launch_stop_unfinished(const Slot* slots, int nslots, hipStream_t s) {
    k_stop_unfinished<<<dim3(nslots), 64, 0, s>>>(slots);
    return hipGetLastError();
}

hipError_t launch_fixup(const GridArgs& g, const Geometry& geo, const Slot* slots, int nslots, hipStream_t s) {
    k_fixup<<<dim3(geo.blocks_pt, nslots), kPtThreads, 0, s>>>(g, slots);
    return hipGetLastError();
}

hipError_t launch_apply(const GridArgs& g, const Geometry& geo, const double* rho, const double* p, double* out,
                        hipStream_t s) {
    k_stencil<0><<<dim3(geo.blocks_pt, 1), kPtThreads, 0, s>>>(g, nullptr, rho, p, out);
    return hipGetLastError();
}

hipError_t launch_residual(const GridArgs& g, const Geometry& geo, const Slot* slot, double* r, hipStream_t s) {
    k_stencil<1><<<dim3(geo.blocks_pt, 1), kPtThreads, 0, s>>>(g, slot, nullptr, nullptr, r);
    return hipGetLastError();
}

// p = (double) d32: the FP32 stand-alone L^+ sweep leaves its result in d32.
__global__ void __launch_bounds__(kPtThreads) k_widen(GridArgs g, const Slot* __restrict__ slots) {
    const Slot& s = slots[blockIdx.y];
    const long long stride = (long long)gridDim.x * kPtThreads;
    for (long long c = (long long)blockIdx.x * kPtThreads + threadIdx.x; c < g.n; c += stride)
        gptr(s.p)[c] = (double)gptr(s.d32)[c];
}

hipError_t launch_lap_pinv(const GridArgs& g, const Geometry& geo, const Tables& t, const Slot* slot,
                           hipStream_t s, bool fp32) {
    hipError_t e = five_sweeps(g, t, slot, 1, fp32, 1, s, nullptr);
    if (e != hipSuccess || !fp32) return e;
    k_widen<<<dim3(geo.blocks_pt, 1), kPtThreads, 0, s>>>(g, slot);
    return hipGetLastError();
}

}  // namespace pois
