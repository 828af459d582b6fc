// The four field sweeps of one iteration of the paper's method (section
// "Poisson equation", eq. (Pois)), written for gfx950:
//   P1 k_resid_dhtx_z r = b~ - A p, q = w r, partial norms per tile, Hartley
//                     along x -> W (z-marching stencil; k_resid_dhtx, a row-pair
//                     gather, for rows that do not fill whole waves)
//   P2 k_dht_cols     Hartley along y of W (also P4: the transform is self-inverse)
//   P3 k_dht_z_solve  Hartley along z, divide by n * symbol, Hartley along z
//                     (taken as FFT, scaling of the separated spectra, inverse FFT)
//   P5 k_dhtx_update  Hartley along x, p += dp (minus the mean of p)
// With walls in x (GridArgs::bcx) P1 and P5 take the cosine transform along x
// instead of the Hartley transform; P2-P4 are the same.
// and, for the FP32 refinement, k_outer_resid_dhtx: the FP64 outer residual
// fused with the first inner sweep's residual.
//
// Each block holds L whole lines of its transform direction in LDS.  The LDS a
// line group needs limits an FP64 sweep to two blocks per CU, too few waves to
// hide HBM latency by occupancy alone, so the blocks are persistent and
// software-pipelined: a block loops over line groups, and the global loads of
// the next group (and, in the FP32 P5, the loads of the values to update) are
// issued before the FFT of the current group, so that they are in flight while
// the block works in LDS.  The stencil sweeps keep the next plane's loads in
// flight while they evaluate the current one, for the same reason.
//
// blockIdx.y selects the solve (slot) of a batch of equal-size grids; every sweep
// returns at once for solves that are done or, on the FP32 path, not in the
// stage the sweep serves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <cstdint>

#include "poisson_device.hpp"

namespace pois {

// ---- P1: residual, weight, Hartley along x --------------------------------------
// MODE 0: stencil residual of the iteration view; MODE 1: q = b (copy, for the
// stand-alone L^+ sweep).
template <typename T, int N, int MODE, int COEF, int WEIGHT>
__global__ void __launch_bounds__((LineCfg<T, N>::NT))
k_resid_dhtx(GridArgs g, const Slot* __restrict__ slots, Tables tb) {
    using C = LineCfg<T, N>;
    __shared__ cpx<T> lds[C::L * C::LS];
    __shared__ cpx<T> tw[N];
    __shared__ double red[(C::NT / 64) * 4];
    const Slot& s = slots[blockIdx.y];
    if (MODE == 0 && IterView<T>::skip_p1(s.st)) return;
    const cpx<T>* twg = twiddles<T>(tb, 0);
    const cpx<T>* twc = dct_twiddles<T>(tb);
    for (int e = threadIdx.x; e < N; e += C::NT) tw[e] = twg[e];

    const unsigned nlines = (unsigned)(g.ny * g.nz / 2);
    const unsigned ngroups = (nlines + C::L - 1) / C::L;
    const IterView<T> v(s);
    POIS_GLOBAL T* W = (MODE == 0) ? v.W : (POIS_GLOBAL T*)gptr(s.W);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};  // sum r^2, sum bt^2, sum p, sum p^2

    // element `it` of this thread in a group: line (tid + it NT) / N, column (tid + it NT) % N
    auto fetch = [&](unsigned grp, int it, PairIn<T>& in) {
        const int e = threadIdx.x + it * C::NT;
        const unsigned P = grp * C::L + e / N;
        if (P < nlines) {
            const unsigned r0 = 2u * P;  // first row of the pair, k*ny + j
            pair_fetch<T>(g, v.p, v.rho, v.rhs, e % N, (int)(r0 % (unsigned)g.ny), (int)(r0 / (unsigned)g.ny), in);
        } else {
#pragma unroll
            for (int k = 0; k < 12; ++k) {
                in.r[k] = T(1);
                in.q[k] = T(0);
            }
            in.ba = in.bb = T(0);
        }
    };
    auto evaluate = [&](unsigned grp, int it, const PairIn<T>& in) {
        const int e = threadIdx.x + it * C::NT;
        const int l = e / N, i = e % N;
        cpx<T> qv = {T(0), T(0)};
        if (grp * C::L + l < nlines) {
            const PairOut<T> o = pair_eval<T, COEF, WEIGHT>(g, in, v.rhs_mean, v.rmax, v.rinv, x_walls(g, i));
            qv = {o.a.w * o.a.r, o.b.w * o.b.r};
            acc[0] += (double)o.a.r * o.a.r + (double)o.b.r * o.b.r;
            acc[1] += (double)o.a.bt * o.a.bt + (double)o.b.bt * o.b.bt;
            acc[2] += (double)o.a.pc + (double)o.b.pc;
            acc[3] += (double)o.a.pc * o.a.pc + (double)o.b.pc * o.b.pc;
        }
        lds[l * C::LS + C::pos(x_slot(i, N, g.bcx))] = qv;
    };

    unsigned grp = blockIdx.x;
    PairIn<T> A, B;
    if (MODE == 0) fetch(grp, 0, A);
    while (true) {
        if (MODE == 0) {
            // two row pairs per step, each evaluated while the next one's loads fly
            for (int it = 0; it < C::IT; it += 2) {
                fetch(grp, it + 1, B);
                evaluate(grp, it, A);
                const bool last = it + 2 >= C::IT;
                const unsigned ng = last ? grp + gridDim.x : grp;
                if (ng < ngroups) fetch(ng, last ? 0 : it + 2, A);
                evaluate(grp, it + 1, B);
            }
        } else {
#pragma unroll
            for (int it = 0; it < C::IT; ++it) {
                const int e = threadIdx.x + it * C::NT;
                const int l = e / N, i = e % N;
                const unsigned P = grp * C::L + l;
                const POIS_GLOBAL double* q = gptr(s.b);
                lds[l * C::LS + C::pos(x_slot(i, N, g.bcx))] =
                    (P < nlines) ? cpx<T>{T(q[(2 * P) * N + i]), T(q[(2 * P + 1) * N + i])} : cpx<T>{T(0), T(0)};
            }
        }
        __syncthreads();
        fft_block_lines<T, N>(lds, tw);
#pragma unroll
        for (int it = 0; it < C::IT; ++it) {
            const int e = threadIdx.x + it * C::NT;
            const int l = e / N, k = e % N;
            const unsigned P = grp * C::L + l;
            if (P < nlines) {
                const cpx<T> h = x_forward_out<T, N>(lds + l * C::LS, k, g.bcx, twc);
                W[(2 * P) * N + k] = h.x;
                W[(2 * P + 1) * N + k] = h.y;
            }
        }
        if (MODE == 0) put_unit_sums<C::NT, 4>(acc, red, s.partial + (unsigned long long)grp * kPartialStride);
        grp += gridDim.x;
        if (grp >= ngroups) break;
        __syncthreads();  // the next group overwrites the lines
    }
}

// P1 for rows whose length is a multiple of the wave size: the residual of a tile
// of KM planes x SUB row pairs is computed by z-marching columns (see ZMarch);
// every KF planes the tile's L lines are transformed along x and written out.
// Within a flush, line l = s KF + q is row pair jp = tj SUB + s of plane
// k = tk KM + f KF + q.
template <typename T, int N>
constexpr int p1_min_blocks();

template <typename T, int N, int COEF, int WEIGHT, int BCX>
__global__ void __launch_bounds__((LineCfg<T, N>::NT), (p1_min_blocks<T, N>()))
k_resid_dhtx_z(GridArgs g, const Slot* __restrict__ slots, Tables tb) {
    using C = LineCfg<T, N>;
    using Z = P1Tile<T, N>;
    __shared__ cpx<T> lds[C::L * C::LS];
    __shared__ cpx<T> tw[N];
    __shared__ double red[(C::NT / 64) * 4];
    __shared__ T edge[2 * Z::SUB * Z::EDGE];  // wave-edge columns, double-buffered by step parity
    const Slot& s = slots[blockIdx.y];
    if (IterView<T>::skip_p1(s.st)) return;
    const cpx<T>* twg = twiddles<T>(tb, 0);
    const cpx<T>* twc = dct_twiddles<T>(tb);
    for (int e = threadIdx.x; e < N; e += C::NT) tw[e] = twg[e];
    const IterView<T> v(s);

    const unsigned nyh = (unsigned)g.ny / 2, nz = (unsigned)g.nz;
    const unsigned ngj = (nyh + Z::SUB - 1) / Z::SUB, ngk = (nz + Z::KM - 1) / Z::KM;
    const unsigned ntiles = ngj * ngk;
    const int sidx = (N >= C::NT) ? 0 : (int)threadIdx.x / N;
    const unsigned col0 = (N >= C::NT) ? threadIdx.x : threadIdx.x % N;
    ZMarch<T> zm;
    zm.p = (const T*)v.p;
    zm.rho = (const T*)v.rho;
    zm.rhs = (const T*)v.rhs;
    zm.nx = (unsigned)g.nx;
    zm.nz = nz;
    zm.sz = (unsigned)g.nx * (unsigned)g.ny;
    zm.lane = (int)(threadIdx.x & 63);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};  // sum r^2, sum bt^2, sum p, sum p^2

    for (unsigned tile = xcd_block(blockIdx.x, gridDim.x); tile < ntiles; tile += gridDim.x) {
        const unsigned tj = tile % ngj, tk = tile / ngj;
        const unsigned jp = tj * Z::SUB + sidx;
        const bool jvalid = jp < nyh;
        zm.rows_of(jvalid ? jp : 0u, (unsigned)g.ny);
        const int k0 = (int)(tk * Z::KM);
        PlaneRows<T> pl[Z::CPT][3];
        PlaneSide<T> sd[Z::CPT];
#pragma unroll
        for (int c = 0; c < Z::CPT; ++c) {
            const unsigned i = col0 + c * C::NT;
            zm.load_rows(zm.plane(k0 - 1), i, pl[c][0]);
            zm.load_rows(zm.plane(k0), i, pl[c][1]);
            zm.load_rows(zm.plane(k0 + 1), i, pl[c][2]);
            zm.load_side(zm.plane(k0), i, sd[c]);
        }
        // the lower z faces of each column's pair, carried from plane to plane
        // (one marching column per thread: with more, the registers are spoken for)
        constexpr bool kZC = COEF == 0 && Z::CPT == 1;
        T zc[Z::CPT][2];
        for (int f = 0; f < Z::KM / Z::KF; ++f) {
            T tacc[2] = {T(0), T(0)};
            // fully unrolled, so that the rotation of the plane registers below
            // is a renaming and not a copy that would wait for the prefetched loads
#pragma unroll
            for (int q = 0; q < Z::KF; ++q) {
                const int k = k0 + f * Z::KF + q;
                const bool valid = jvalid && k < (int)nz;
                // the next step's plane and side fly while this step computes (also
                // on the tile's last step, wrapped in z and unused, so that the wait
                // counts are the same every step)
                PlaneRows<T> nn[Z::CPT];
                PlaneSide<T> ns[Z::CPT];
                // waves issuing loads go first, so that the memory requests of
                // all resident waves are out before any spends its step computing
                __builtin_amdgcn_s_setprio(2);
#pragma unroll
                for (int c = 0; c < Z::CPT; ++c) {
                    const unsigned i = col0 + c * C::NT;
                    zm.load_rows(zm.plane(k + 2), i, nn[c]);
                    zm.load_side(zm.plane(k + 1), i, ns[c]);
                }
                __builtin_amdgcn_s_setprio(0);
                T* eb = edge + ((q & 1) * Z::SUB + sidx) * Z::EDGE;
#pragma unroll
                for (int c = 0; c < Z::CPT; ++c) zm.edge_put(eb, col0 + c * C::NT, pl[c][1]);
                __syncthreads();
#pragma unroll
                for (int c = 0; c < Z::CPT; ++c) {
                    const unsigned i = col0 + c * C::NT;
                    PairIn<T> in;
                    zm.pair(pl[c][0], pl[c][1], pl[c][2], sd[c], zm.edge_get(eb, i), in);
                    cpx<T> qv = {T(0), T(0)};
                    if (valid) {
                        if constexpr (kZC)
                            if (q == 0 && f == 0) z_faces_below(in, v.rinv, zc[c]);
                        const PairOut<T> o = pair_eval<T, COEF, WEIGHT, kZC>(g, in, v.rhs_mean, v.rmax, v.rinv,
                                                                             BCX ? x_walls(g, i) : 0u, zc[c]);
                        qv = {o.a.w * o.a.r, o.b.w * o.b.r};
                        if constexpr (sizeof(T) == 8) {
                            acc[0] += o.a.r * o.a.r + o.b.r * o.b.r;
                            acc[1] += o.a.bt * o.a.bt + o.b.bt * o.b.bt;
                            acc[2] += o.a.pc + o.b.pc;
                            acc[3] += o.a.pc * o.a.pc + o.b.pc * o.b.pc;
                        } else {
                            // FP32 inner sweeps: only the two norms are used (the
                            // stopping test), summed in FP32 over the flush
                            tacc[0] += o.a.r * o.a.r + o.b.r * o.b.r;
                            tacc[1] += o.a.bt * o.a.bt + o.b.bt * o.b.bt;
                        }
                    }
                    lds[(sidx * Z::KF + q) * C::LS + C::pos(x_slot(i, N, BCX))] = qv;
                }
#pragma unroll
                for (int c = 0; c < Z::CPT; ++c) {
                    pl[c][0] = pl[c][1];
                    pl[c][1] = pl[c][2];
                    pl[c][2] = nn[c];
                    sd[c] = ns[c];
                }
            }
            if constexpr (sizeof(T) == 4) {
                acc[0] += (double)tacc[0];
                acc[1] += (double)tacc[1];
            }
            __syncthreads();
            fft_block_lines<T, N>(lds, tw);
#pragma unroll
            for (int it = 0; it < C::IT; ++it) {
                const int e = threadIdx.x + it * C::NT;
                const int l = e / N, k = e % N;
                const unsigned ljp = tj * Z::SUB + l / Z::KF;
                const unsigned lk = (unsigned)(k0 + f * Z::KF) + l % Z::KF;
                if (ljp < nyh && lk < nz) {
                    const unsigned P = lk * nyh + ljp;  // row pair index, rows 2P and 2P + 1
                    const cpx<T> h = x_forward_out<T, N>(lds + l * C::LS, k, BCX, twc);
                    // streaming stores: the transformed lines are not read
                    // again by this sweep, and left out of L2 they do not push
                    // out the rows that neighbouring tiles read as y halo
                    // (FP64 at 512^3: 1.09 -> 1.02 of the algorithmic bytes)
                    __builtin_nontemporal_store(h.x, &v.W[(2 * P) * N + k]);
                    __builtin_nontemporal_store(h.y, &v.W[(2 * P + 1) * N + k]);
                }
            }
            __syncthreads();  // the next flush overwrites the lines
        }
        put_unit_sums<C::NT, 4>(acc, red, s.partial + (unsigned long long)tile * kPartialStride);
    }
}

// FP32_REFINE: the FP64 outer residual of a refinement step fused with the
// residual half of its first FP32 inner sweep.  The inner correction starts at
// zero, so that sweep's weighted residual is q = w r32 with r32 = r s^-1 of the
// FP64 residual r = b~ - A p: the tile's FP64 residual (z-marching as in P1)
// gives r32 (stored for the later inner sweeps) and q, whose lines are
// transformed along x into W32 exactly as the FP32 P1 would.  The mean of r32,
// which the FP32 P1 removes, is FP64 rounding noise here and is not removed.
// Per tile: r^2, bt^2, p, p^2, r in FP64.  One column per thread.  write = 0:
// the sums alone (the final check of a solve, which usually ends it: no r32,
// no transform, no W32).
template <int N, int COEF, int WEIGHT, int BCX>
__global__ void __launch_bounds__((LineCfg<float, N>::NT), (LineCfg<float, N>::MINB))
k_outer_resid_dhtx(GridArgs g, const Slot* __restrict__ slots, Tables tb, int write) {
    using C = LineCfg<float, N>;
    using Z = OuterTile<N>;
    static_assert(Z::CPT == 1, "one marching column per thread");
    __shared__ cpx<float> lds[C::L * C::LS];
    __shared__ cpx<float> tw[N];
    __shared__ double red[(C::NT / 64) * 5];
    __shared__ double edge[2 * Z::SUB * Z::EDGE];
    const Slot& s = slots[blockIdx.y];
    SolveState* st = s.st;
    if (st->done || st->stage != 0) return;
    const cpx<float>* twg = twiddles<float>(tb, 0);
    const cpx<float>* twc = dct_twiddles<float>(tb);
    for (int e = threadIdx.x; e < N; e += C::NT) tw[e] = twg[e];
    const double bm = st->b_mean, inv_s = st->inv_s, rmax = st->rho_max, rinv = recip(st->rho_max);

    const unsigned nyh = (unsigned)g.ny / 2, nz = (unsigned)g.nz;
    const unsigned ngj = (nyh + Z::SUB - 1) / Z::SUB, ngk = (nz + Z::KM - 1) / Z::KM;
    const unsigned ntiles = ngj * ngk;
    const int sidx = (N >= C::NT) ? 0 : (int)threadIdx.x / N;
    const unsigned i = (N >= C::NT) ? threadIdx.x : threadIdx.x % N;
    POIS_GLOBAL float* r32 = gptr(s.r32);
    POIS_GLOBAL float* W32 = gptr(s.W32);
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
        const unsigned jp = tj * Z::SUB + sidx;
        const bool jvalid = jp < nyh;
        zm.rows_of(jvalid ? jp : 0u, (unsigned)g.ny);
        const int k0 = (int)(tk * Z::KM);
        PlaneRows<double> pl[3];
        PlaneSide<double> sd;
        zm.load_rows(zm.plane(k0 - 1), i, pl[0]);
        zm.load_rows(zm.plane(k0), i, pl[1]);
        zm.load_rows(zm.plane(k0 + 1), i, pl[2]);
        zm.load_side(zm.plane(k0), i, sd);
        double zc[2];  // the lower z faces of the pair, carried from plane to plane (COEF 0)
        for (int f = 0; f < Z::KM / Z::KF; ++f) {
#pragma unroll
            for (int q = 0; q < Z::KF; ++q) {
                const int k = k0 + f * Z::KF + q;
                const bool valid = jvalid && k < (int)nz;
                PlaneRows<double> nn;
                PlaneSide<double> ns;
                __builtin_amdgcn_s_setprio(2);
                zm.load_rows(zm.plane(k + 2), i, nn);
                zm.load_side(zm.plane(k + 1), i, ns);
                __builtin_amdgcn_s_setprio(0);
                double* eb = edge + ((q & 1) * Z::SUB + sidx) * Z::EDGE;
                zm.edge_put(eb, i, pl[1]);
                __syncthreads();
                PairIn<double> in;
                zm.pair(pl[0], pl[1], pl[2], sd, zm.edge_get(eb, i), in);
                cpx<float> qv = {0.0f, 0.0f};
                if (valid) {
                    if constexpr (COEF == 0)
                        if (q == 0 && f == 0) z_faces_below(in, rinv, zc);
                    const PairOut<double> pr =
                        pair_eval<double, COEF, WEIGHT, COEF == 0>(g, in, bm, rmax, rinv, BCX ? x_walls(g, i) : 0u, zc);
                    acc[0] += pr.a.r * pr.a.r + pr.b.r * pr.b.r;
                    acc[1] += pr.a.bt * pr.a.bt + pr.b.bt * pr.b.bt;
                    acc[2] += pr.a.pc + pr.b.pc;
                    acc[3] += pr.a.pc * pr.a.pc + pr.b.pc * pr.b.pc;
                    acc[4] += pr.a.r + pr.b.r;
                    if (write) {
                        const float ra = (float)(pr.a.r * inv_s), rb = (float)(pr.b.r * inv_s);
                        const unsigned a = (unsigned)k * zm.sz + zm.ra + i;
                        __builtin_nontemporal_store(ra, &r32[a]);  // streaming (see k_resid_dhtx_z)
                        __builtin_nontemporal_store(rb, &r32[a + (unsigned)g.nx]);
                        qv = {(float)pr.a.w * ra, (float)pr.b.w * rb};
                    }
                }
                if (write) lds[(sidx * Z::KF + q) * C::LS + C::pos(x_slot(i, N, BCX))] = qv;
                pl[0] = pl[1];
                pl[1] = pl[2];
                pl[2] = nn;
                sd = ns;
            }
            if (!write) continue;  // uniform
            __syncthreads();
            fft_block_lines<float, N>(lds, tw);
#pragma unroll
            for (int it = 0; it < C::IT; ++it) {
                const int e = threadIdx.x + it * C::NT;
                const int l = e / N, kx = e % N;
                const unsigned ljp = tj * Z::SUB + l / Z::KF;
                const unsigned lk = (unsigned)(k0 + f * Z::KF) + l % Z::KF;
                if (ljp < nyh && lk < nz) {
                    const unsigned P = lk * nyh + ljp;
                    const cpx<float> h = x_forward_out<float, N>(lds + l * C::LS, kx, BCX, twc);
                    __builtin_nontemporal_store(h.x, &W32[(2 * P) * N + kx]);
                    __builtin_nontemporal_store(h.y, &W32[(2 * P + 1) * N + kx]);
                }
            }
            __syncthreads();  // the next flush overwrites the lines
        }
        put_unit_sums<C::NT, 5>(acc, red, s.partial + (unsigned long long)tile * kPartialStride);
    }
}

// Rows that fill whole waves, and a register budget for CPT marching columns.
template <typename T, int N>
constexpr bool use_zmarch() {
    using C = LineCfg<T, N>;
    if constexpr (N % 64 != 0) return false;
    else return (N >= C::NT ? N / C::NT : 1) * (int)sizeof(T) <= 32;
}

// Minimum waves per SIMD the residual sweep's registers are sized for (the
// second __launch_bounds__ argument, which caps the registers per thread): one
// where four FP64 marching columns per thread need the accumulation registers
// too.  The FP32 sweep on 512-cell rows runs 512-thread blocks whose LDS leaves
// room for two per CU: asking for four waves per SIMD (128 registers) lets both
// be resident, 16 waves per CU instead of 8 (6% faster at 512^3; the FP32 y, z
// and x-update sweeps spill at 128 registers and lose 2x, so they keep one).
template <typename T, int N>
constexpr int p1_min_blocks() {
    using C = LineCfg<T, N>;
    if constexpr (sizeof(T) == 4 && N == 512 && C::NT == 512) return 4;
    return (N >= C::NT ? N / C::NT : 1) * (int)sizeof(T) > 16 ? 1 : C::MINB;
}

// ---- P2 / P4: Hartley along y (AX = 1) of the pair-packed columns -------------
// Line = (o, m): complex column m (real columns 2m, 2m+1) at outer index o;
// element e along the axis.  y: address (o*ny + e)*nxh + m; z: (e*ny + o)*nxh + m.
// Thread t of a block always works on line t % L of the group, elements
// t / L + it TT.
template <int AX>
__device__ __forceinline__ unsigned col_base(const GridArgs& g, unsigned line) {
    const unsigned nxh = g.nxh, o = line / nxh, m = line - o * nxh;
    return (AX == 1) ? o * (unsigned)g.ny * nxh + m : o * nxh + m;
}

template <typename T, int N, int AX, int MODE>
__global__ void __launch_bounds__((LineCfg<T, N>::NT), (LineCfg<T, N>::MINB))
k_dht_cols(GridArgs g, const Slot* __restrict__ slots, Tables tb, int stage) {
    using C = LineCfg<T, N>;
    __shared__ cpx<T> lds[C::L * C::LS];
    __shared__ cpx<T> tw[N];
    const Slot& s = slots[blockIdx.y];
    if (MODE == 0 && IterView<T>::skip(s.st, stage)) return;
    const cpx<T>* twg = twiddles<T>(tb, AX);
    for (int e = threadIdx.x; e < N; e += C::NT) tw[e] = twg[e];
    POIS_GLOBAL T* Wc = MODE == 0 ? IterView<T>(s).W : (POIS_GLOBAL T*)gptr(s.W);  // complex-indexed
    const unsigned nlines = (AX == 1) ? (unsigned)(g.nxh * g.nz) : (unsigned)(g.nxh * g.ny);
    const unsigned ngroups = (nlines + C::L - 1) / C::L;
    const unsigned se = (AX == 1) ? (unsigned)g.nxh : (unsigned)(g.nxh * g.ny);
    constexpr bool kRegs = (N == 256 || N == 512) && C::L == 16;
    const int l = threadIdx.x % C::L;
    const int e0 = kRegs ? reg_col<kRegs ? N : 256>((int)threadIdx.x / 16) : (int)threadIdx.x / C::L;

    // element e0 + it TT of a line at base + e0 se + (it TT) se: the lane's part
    // in one register, the rest wave-uniform (no per-element address registers
    // live across the transform).  A line past the end (in the last group)
    // loads line 0 and is not stored: no branch per element.
    const unsigned lane_off = (unsigned)e0 * se;
    cpx<T> buf[C::IT];
    auto load = [&](unsigned grp, bool& valid, unsigned& base) {
        const unsigned line = grp * C::L + l;
        valid = line < nlines;
        base = valid ? col_base<AX>(g, line) : 0u;
#pragma unroll
        for (int it = 0; it < C::IT; ++it) buf[it] = gload_c(Wc, base + lane_off + (unsigned)(it * C::TT) * se);
    };
    unsigned grp = blockIdx.x, base;
    bool valid;
    load(grp, valid, base);
    if constexpr (kRegs) {
        // the line stays in registers; LDS only for the transpose of the
        // transform and the exchange of the (k, N-k) partners, which stays
        // within the wave (reg_col, exchange_write)
        __syncthreads();  // twiddles
        cpx<T>* ln = lds + l * C::LS;
        while (true) {
            cpx<T> v[16];
#pragma unroll
            for (int a = 0; a < 16; ++a) v[a] = buf[a];
            const bool cur_valid = valid;
            const unsigned cur_base = base;
            const unsigned ng = grp + gridDim.x;
            __builtin_amdgcn_s_setprio(2);
            if (ng < ngroups) load(ng, valid, base);  // in flight during the FFT
            __builtin_amdgcn_s_setprio(0);
            // the column, opaque within each group: the lane-dependent
            // addresses derived from it are formed here rather than held in
            // registers across the loop
            int c = e0;
            asm volatile("" : "+v"(c));
            if constexpr (N == 256) fft256_regs<T>(v, ln, c, tw);
            else fft512_regs<T>(v, ln, c, tw);
            exchange_write<T, N>(ln, c, v);
            wave_lds_sync();
            if (cur_valid) {
                const cpx<T>* pp = exchange_partner<T, N>(ln, c);
                // k = kb + 16 b
                const unsigned kb = N == 256 ? (unsigned)c : (unsigned)((c >> 1) + 256 * (c & 1));
                const unsigned st_base = cur_base + kb * se;
#pragma unroll
                for (int b = 0; b < 16; ++b)
                    gstore_c(Wc, st_base + (unsigned)(16 * b) * se, hartley(v[b], pp[17 * (15 - b)]));
            }
            grp = ng;
            if (grp >= ngroups) break;
            // N = 256: the next transpose writes this thread's own column, read
            // only by its wave; N = 512: it writes every wave's positions
            if constexpr (N == 256) wave_lds_sync();
            else __syncthreads();
        }
        return;
    }
    while (true) {
#pragma unroll
        for (int it = 0; it < C::IT; ++it) lds[l * C::LS + C::pos(e0 + it * C::TT)] = buf[it];
        const bool cur_valid = valid;
        const unsigned cur_base = base;
        const unsigned ng = grp + gridDim.x;
        __builtin_amdgcn_s_setprio(2);
        if (ng < ngroups) load(ng, valid, base);  // in flight during the FFT
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        fft_block_lines<T, N>(lds, tw);
        if (cur_valid) {
#pragma unroll
            for (int it = 0; it < C::IT; ++it) {
                const int idx = e0 + it * C::TT;
                gstore_c(Wc, cur_base + (unsigned)idx * se,
                         hartley(lds[l * C::LS + C::pos(idx)], lds[l * C::LS + C::pos((idx == 0 ? 0 : N - idx))]));
            }
        }
        grp = ng;
        if (grp >= ngroups) break;
        __syncthreads();
    }
}

// ---- P3: Hartley along z, divide by n * symbol, Hartley along z ----------------
// The z symbol is even in k_z, so Hartley-scale-Hartley equals an FFT, a scaling
// of each packed row's spectrum, and an inverse FFT: the two rows of a pair
// (x wavenumbers 2m and 2m+1, symbols s_a and s_b) are separated as
// A_k = (Z_k + conj Z_{N-k})/2 and i B_k = (Z_k - conj Z_{N-k})/2, so the scaled
// spectrum is Z'_k = (s_a + s_b)/2 Z_k + (s_a - s_b)/2 conj Z_{N-k}; the inverse is
// taken as conj(FFT(conj Z')), which needs no exchange of (k, N-k) partners.
template <typename T>
__device__ __forceinline__ cpx<T> scaled_conj_h(cpx<T> zk, cpx<T> zm, T hp, T hm) {
    return {hp * zk.x + hm * zm.x, hm * zm.y - hp * zk.y};  // conj(hp Z_k + hm conj Z_{N-k})
}
template <typename T>
__device__ __forceinline__ cpx<T> scaled_conj(cpx<T> zk, cpx<T> zm, T sa, T sb) {
    return scaled_conj_h(zk, zm, T(0.5) * (sa + sb), T(0.5) * (sa - sb));
}

// The register paths take hp = (s_a + s_b)/2 and hm = (s_a - s_b)/2 with one
// reciprocal per wavenumber instead of two.  The symbols are scaled by a power
// of two sc (exact, and the product of two of them then stays in range): with
// ta = sc lam_a, tb = sc lam_b and kn = n / sc, s_a = 1 / (n lam_a) = 1 / (kn ta)
// and
//     hp = (ta + tb) / (2 kn ta tb),   hm = (tb - ta) / (2 kn ta tb).
// Only the constant mode has a zero symbol; the one value per thread that may
// hold it takes pair_coefs0, which inverts each symbol on its own (0 for 0).
template <typename T>
__device__ __forceinline__ void pair_coefs(T ta, T tb, T dt, T kn2, T& hp, T& hm) {
    const T r = recip(ta * tb * kn2);
    hp = (ta + tb) * r;
    hm = dt * r;
}
template <typename T>
__device__ __forceinline__ void pair_coefs0(T ta, T tb, T kn, T& hp, T& hm) {
    const T sa = ta == T(0) ? T(0) : recip(kn * ta), sb = tb == T(0) ? T(0) : recip(kn * tb);
    hp = T(0.5) * (sa + sb);
    hm = T(0.5) * (sa - sb);
}
// sc = 2^-e, with every symbol's magnitude (at most 4 (1/hx^2 + 1/hy^2 + 1/hz^2))
// below 2^e
template <typename T>
__device__ __forceinline__ T symbol_scale(const GridArgs& g) {
    int e;
    (void)frexp(4.0 * (g.ihx2 + g.ihy2 + g.ihz2), &e);
    e = e < -120 ? -120 : (e > 120 ? 120 : e);
    return T(ldexp(1.0, -e));
}

// Launch shape of the z sweep: ZL lines per block, PF whether the next line
// group is loaded during this one's transforms, MINW the waves per SIMD its
// registers are sized for (the second __launch_bounds__ argument).  Measured
// (MI355X): the FP32 256-point path runs four blocks per CU with the prefetch
// (111 registers); the FP32 512-point path runs two 512-thread blocks per CU
// without it (no spills; 14% faster than one block with it); the FP64 paths
// prefetch (no spills at 2 and 1 blocks per CU).
template <typename T, int N>
constexpr int z_min_blocks() {
    if constexpr (sizeof(T) == 4 && N == 256) return 4;
    else if constexpr (sizeof(T) == 4 && N == 512) return 4;
    else return LineCfg<T, N>::MINB;
}

template <typename T, int N>
struct ZCfg {
    static constexpr int ZL = LineCfg<T, N>::L;
    static constexpr bool PF = !(sizeof(T) == 4 && N == 512);
    static constexpr int MINW = z_min_blocks<T, N>();
};

template <typename T, int N, int MODE, int ZL, bool PF, int MINW>
__global__ void __launch_bounds__((LineShape<T, N, ZL>::NT), (MINW))
k_dht_z_solve(GridArgs g, const Slot* __restrict__ slots, Tables tb, int stage) {
    using C = LineShape<T, N, ZL>;
    __shared__ cpx<T> lds[C::L * C::LS];
    __shared__ cpx<T> tw[N];
    // the z symbol of the register path, in LDS: a global load of it after the
    // next group's prefetch would make the wait for it a wait for the prefetch
    __shared__ T lzs[(N == 256 || N == 512) ? N : 1];
    const Slot& s = slots[blockIdx.y];
    if (MODE == 0 && IterView<T>::skip(s.st, stage)) return;
    const cpx<T>* twg = twiddles<T>(tb, 2);
    for (int e = threadIdx.x; e < N; e += C::NT) tw[e] = twg[e];
    const T sc = symbol_scale<T>(g);
    if constexpr (N == 256 || N == 512)
        for (int e = threadIdx.x; e < N; e += C::NT) lzs[e] = symbol<T>(tb, 2)[e] * sc;
    POIS_GLOBAL T* Wc = MODE == 0 ? IterView<T>(s).W : (POIS_GLOBAL T*)gptr(s.W);  // complex-indexed
    const unsigned nlines = (unsigned)(g.nxh * g.ny);
    const unsigned ngroups = (nlines + C::L - 1) / C::L;
    const unsigned se = (unsigned)(g.nxh * g.ny);
    constexpr bool kRegs = (N == 256 || N == 512) && C::L == 16;
    const int l = threadIdx.x % C::L;
    const int e0 = kRegs ? reg_col<kRegs ? N : 256>((int)threadIdx.x / 16) : (int)threadIdx.x / C::L;
    const T* lamx = symbol<T>(tb, 0);
    const T* lamy = symbol<T>(tb, 1);
    const T* lamz = symbol<T>(tb, 2);
    const T nn = T(g.n);
    const T kn = nn / sc, kn2 = T(2) * kn;  // exact: sc is a power of two

    // element e0 + it TT of a line at base + e0 se + (it TT) se; a line past
    // the end loads line 0 and is not stored (see k_dht_cols)
    const unsigned lane_off = (unsigned)e0 * se;
    cpx<T> buf[C::IT];
    auto load = [&](unsigned grp, bool& valid, unsigned& base) {
        const unsigned line = grp * C::L + l;
        valid = line < nlines;
        base = valid ? col_base<2>(g, line) : 0u;
#pragma unroll
        for (int it = 0; it < C::IT; ++it) buf[it] = gload_c(Wc, base + lane_off + (unsigned)(it * C::TT) * se);
    };
    unsigned grp = blockIdx.x, base;
    bool valid;
    if constexpr (PF) load(grp, valid, base);
    if constexpr (N == 256 && kRegs) {
        // the line stays in registers (see fft256_regs); LDS only for the
        // transposes and the exchange of the (k, N-k) partners, which stays
        // within the wave (reg_col): 4 block barriers per line group
        __syncthreads();  // twiddles
        cpx<T>* ln = lds + l * C::LS;
        while (true) {
            if constexpr (!PF) load(grp, valid, base);
            cpx<T> v[16];
#pragma unroll
            for (int a = 0; a < 16; ++a) v[a] = buf[a];
            const bool cur_valid = valid;
            const unsigned cur_base = base;
            const unsigned line = grp * C::L + l;
            const unsigned j = cur_valid ? line / (unsigned)g.nxh : 0u, m = cur_valid ? line - j * (unsigned)g.nxh : 0u;
            const T lxe = lamx[2 * m], lxo = lamx[2 * m + 1], lyj = lamy[j];
            const T ta0 = (lxe + lyj) * sc, tb0 = (lxo + lyj) * sc, dt = (lxo - lxe) * sc;
            const unsigned ng = grp + gridDim.x;
            if constexpr (PF) {
                __builtin_amdgcn_s_setprio(2);
                if (ng < ngroups) load(ng, valid, base);  // in flight during the two FFTs
                __builtin_amdgcn_s_setprio(0);
            }
            int c = e0;  // opaque within each group (see k_dht_cols)
            asm volatile("" : "+v"(c));
            fft256_regs<T>(v, ln, c, tw);  // v[b] = X[c + 16 b]
            exchange_write<T, N>(ln, c, v);
            wave_lds_sync();
            {
                const cpx<T>* pp = exchange_partner<T, N>(ln, c);
                const T* lz = lzs + c;  // sc times the z symbol at k = c + 16 b (zero only for k = 0)
#pragma unroll
                for (int b = 0; b < 16; ++b) {
                    const T lzk = lz[16 * b];
                    T hp, hm;
                    if (b == 0) pair_coefs0(ta0 + lzk, tb0 + lzk, kn, hp, hm);
                    else pair_coefs(ta0 + lzk, tb0 + lzk, dt, kn2, hp, hm);
                    // the second transform's input x[c + 16 b]
                    v[b] = scaled_conj_h(v[b], pp[17 * (15 - b)], hp, hm);
                }
            }
            wave_lds_sync();  // the partner lanes' reads before this wave's transpose writes
            fft256_regs<T>(v, ln, c, tw);
            if (cur_valid) {
                const unsigned st_base = cur_base + (unsigned)c * se;
#pragma unroll
                for (int b = 0; b < 16; ++b)
                    gstore_c(Wc, st_base + (unsigned)(16 * b) * se, cpx<T>{v[b].x, -v[b].y});
            }
            grp = ng;
            if (grp >= ngroups) break;
        }
        return;
    }
    if constexpr (N == 512 && kRegs) {
        // the line stays in registers: thread e0 of a line holds x[e0 + 32 a];
        // after fft512_regs it holds X[k] for k = k1 + 16 b + 256 h (k1 = e0 / 2,
        // h = e0 % 2).  The spectrum goes through the line's LDS row once, which
        // hands each thread its natural-order input of the second transform and
        // the (k, N-k) partners: 6 block barriers per line group, with the fewest
        // registers (two 512-thread FP32 blocks per CU).
        static_assert(C::TT == 32 && C::IT == 16, "512-point lines: 32 threads of 16 values");
        __syncthreads();  // twiddles, symbol
        cpx<T>* ln = lds + l * C::LS;
        while (true) {
            if constexpr (!PF) load(grp, valid, base);
            cpx<T> v[16];
#pragma unroll
            for (int a = 0; a < 16; ++a) v[a] = buf[a];
            const bool cur_valid = valid;
            const unsigned cur_base = base;
            const unsigned line = grp * C::L + l;
            const unsigned j = cur_valid ? line / (unsigned)g.nxh : 0u, m = cur_valid ? line - j * (unsigned)g.nxh : 0u;
            const T lxe = lamx[2 * m], lxo = lamx[2 * m + 1], lyj = lamy[j];
            const T ta0 = (lxe + lyj) * sc, tb0 = (lxo + lyj) * sc, dt = (lxo - lxe) * sc;
            const unsigned ng = grp + gridDim.x;
            if constexpr (PF) {
                __builtin_amdgcn_s_setprio(2);
                if (ng < ngroups) load(ng, valid, base);  // in flight during the two FFTs
                __builtin_amdgcn_s_setprio(0);
            }
            int c = e0;  // opaque within each group (see k_dht_cols)
            asm volatile("" : "+v"(c));
            fft512_regs<T>(v, ln, c, tw);  // v[b] = X[c/2 + 16 b + 256 (c mod 2)]
            exchange_write<T, N>(ln, c, v);
            // the whole spectrum through LDS: the second forward transform
            // takes its input x[c + 32 a] in natural order, at pos(c + 32 a) =
            // c + c/16 + 34 a, its partner at pos(N - c - 32 a) = p2 - 34 a
            // (for c = 0 the padding slot holding X[0] at a = 0)
            __syncthreads();
            {
                const cpx<T>* pk = ln + c + (c >> 4);
                const int p2 = c == 0 ? 544 : (512 - c) + ((512 - c) >> 4);
                const cpx<T>* pm = ln + (p2 - 510);
                const T* lz = lzs + c;  // sc times the z symbol at k = c + 32 a (zero only for k = 0)
#pragma unroll
                for (int a = 0; a < 16; ++a) {
                    const T lzk = lz[32 * a];
                    T hp, hm;
                    if (a == 0) pair_coefs0(ta0 + lzk, tb0 + lzk, kn, hp, hm);
                    else pair_coefs(ta0 + lzk, tb0 + lzk, dt, kn2, hp, hm);
                    v[a] = scaled_conj_h(pk[34 * a], pm[34 * (15 - a)], hp, hm);
                }
            }
            __syncthreads();
            fft512_regs<T>(v, ln, c, tw);  // v[b] = conj(x'[c/2 + 16 b + 256 (c mod 2)])
            if (cur_valid) {
                const unsigned st_base = cur_base + (unsigned)((c >> 1) + 256 * (c & 1)) * se;
#pragma unroll
                for (int b = 0; b < 16; ++b)
                    gstore_c(Wc, st_base + (unsigned)(16 * b) * se, cpx<T>{v[b].x, -v[b].y});
            }
            // fft512_regs ends on a barrier: the next group's writes are safe
            grp = ng;
            if (grp >= ngroups) break;
        }
        return;
    }
    while (true) {
        if constexpr (!PF) load(grp, valid, base);
#pragma unroll
        for (int it = 0; it < C::IT; ++it) lds[l * C::LS + C::pos(e0 + it * C::TT)] = buf[it];
        const bool cur_valid = valid;
        const unsigned cur_base = base;
        // symbol of this thread's line: x wavenumbers 2m, 2m+1 (the pair), y wavenumber j
        const unsigned line = grp * C::L + l;
        const unsigned j = cur_valid ? line / (unsigned)g.nxh : 0u, m = cur_valid ? line - j * (unsigned)g.nxh : 0u;
        const T lxe = lamx[2 * m], lxo = lamx[2 * m + 1], lyj = lamy[j];
        const unsigned ng = grp + gridDim.x;
        if constexpr (PF) {
            __builtin_amdgcn_s_setprio(2);
            if (ng < ngroups) load(ng, valid, base);  // in flight during the two FFTs
            __builtin_amdgcn_s_setprio(0);
        }
        __syncthreads();
        fft_block_lines<T, N>(lds, tw);
        // scaled spectra of the pairs (k, N-k) of this thread's line (the symbol is
        // even in k), conjugated for the inverse
        for (int k = e0; k <= N / 2; k += C::TT) {
            const int km = (k == 0) ? 0 : N - k;
            const cpx<T> zk = lds[l * C::LS + C::pos(k)], zm = lds[l * C::LS + C::pos(km)];
            const T lzk = lamz[k];
            const T sa = inv_symbol(lxe, lyj, lzk, nn), sb = inv_symbol(lxo, lyj, lzk, nn);
            lds[l * C::LS + C::pos(k)] = scaled_conj(zk, zm, sa, sb);
            lds[l * C::LS + C::pos(km)] = scaled_conj(zm, zk, sa, sb);
        }
        __syncthreads();
        fft_block_lines<T, N>(lds, tw);
        if (cur_valid) {
#pragma unroll
            for (int it = 0; it < C::IT; ++it) {
                const int idx = e0 + it * C::TT;
                const cpx<T> r = lds[l * C::LS + C::pos(idx)];
                gstore_c(Wc, cur_base + (unsigned)idx * se, cpx<T>{r.x, -r.y});
            }
        }
        grp = ng;
        if (grp >= ngroups) break;
        __syncthreads();
    }
}

// ---- P5: Hartley along x, update -----------------------------------------------
// MODE 0: FP64 p += dp - mean(p) (or FP32 d32 += dp); MODE 1: assign to p (L^+
// sweep); MODE 2: FP32 d32 = dp, the first inner sweep after a fused outer
// residual (d32 holds nothing yet).
// The FP32 x-update sweep on periodic rows of 256 is sized for four blocks per
// CU (what its LDS allows; 128 registers, no spills): it then loads the values
// it updates after the transform, their latency covered by the other blocks
// instead of a second register buffer.
template <typename T, int N, int BCX>
constexpr int update_min_waves() {
    return (sizeof(T) == 4 && N == 256 && BCX == 0) ? 4 : 1;
}

template <typename T, int N, int MODE, int BCX>
__global__ void __launch_bounds__((LineCfg<T, N>::NT), (update_min_waves<T, N, BCX>()))
k_dhtx_update(GridArgs g, const Slot* __restrict__ slots, Tables tb, int stage) {
    using C = LineCfg<T, N>;
    __shared__ cpx<T> lds[C::L * C::LS];
    __shared__ cpx<T> tw[N];
    const Slot& s = slots[blockIdx.y];
    if (MODE != 1 && IterView<T>::skip(s.st, stage)) return;
    // the update of the last inner evaluation is applied here: the next inner
    // residual sweep may run (no other block of this launch reads the flag)
    if constexpr (MODE == 0 && sizeof(T) == 4)
        if (blockIdx.x == 0 && threadIdx.x == 0) s.st->upd_due = 0;
    const cpx<T>* twg = twiddles<T>(tb, 0);
    const cpx<T>* twc = dct_twiddles<T>(tb);
    for (int e = threadIdx.x; e < N; e += C::NT) tw[e] = twg[e];
    const POIS_GLOBAL T* W = (MODE != 1) ? IterView<T>(s).W : (const POIS_GLOBAL T*)gptr(s.W);
    POIS_GLOBAL T* out;
    if constexpr (sizeof(T) == 8) out = (POIS_GLOBAL T*)gptr(s.p);
    else out = (POIS_GLOBAL T*)gptr(s.d32);
    const T shift = (MODE == 0 && sizeof(T) == 8) ? T(s.st->p_shift) : T(0);
    const unsigned nlines = (unsigned)(g.ny * g.nz / 2);
    const unsigned ngroups = (nlines + C::L - 1) / C::L;

    cpx<T> wb[C::IT], pb[C::IT];
    auto load_w = [&](unsigned grp) {
#pragma unroll
        for (int it = 0; it < C::IT; ++it) {
            const int e = threadIdx.x + it * C::NT;
            const unsigned P = grp * C::L + e / N;
            const int i = e % N;
            wb[it] = (P < nlines) ? cpx<T>{W[(2 * P) * N + i], W[(2 * P + 1) * N + i]} : cpx<T>{T(0), T(0)};
        }
    };
    unsigned grp = blockIdx.x;
    load_w(grp);
    while (true) {
#pragma unroll
        for (int it = 0; it < C::IT; ++it) {
            const int e = threadIdx.x + it * C::NT;
            lds[(e / N) * C::LS + C::pos(e % N)] = wb[it];
        }
        if constexpr (BCX != 0) {
            // cosine transform between walls: the FFT input pairs coefficient k
            // with coefficient N - k of the same line
            __syncthreads();
#pragma unroll
            for (int it = 0; it < C::IT; ++it) {
                const int e = threadIdx.x + it * C::NT;
                const int l = e / N, k = e % N;
                const cpx<T> cm = (k == 0) ? cpx<T>{T(0), T(0)} : lds[l * C::LS + C::pos(N - k)];
                wb[it] = idct_in(wb[it], cm, twc[k]);
            }
            __syncthreads();
#pragma unroll
            for (int it = 0; it < C::IT; ++it) {
                const int e = threadIdx.x + it * C::NT;
                lds[(e / N) * C::LS + C::pos(e % N)] = wb[it];
            }
        }
        // FP32: the values to update are loaded now and are in flight during the
        // FFT; FP64 has no registers to spare for them and loads them after it
        constexpr bool kEarly = MODE == 0 && sizeof(T) == 4 && update_min_waves<T, N, BCX>() == 1;
        if (kEarly) {
#pragma unroll
            for (int it = 0; it < C::IT; ++it) {
                const int e = threadIdx.x + it * C::NT;
                const unsigned P = grp * C::L + e / N;
                const int k = e % N;
                pb[it] = (P < nlines) ? cpx<T>{out[(2 * P) * N + k], out[(2 * P + 1) * N + k]} : cpx<T>{T(0), T(0)};
            }
        }
        const unsigned ng = grp + gridDim.x;
        __builtin_amdgcn_s_setprio(2);
        if (ng < ngroups) load_w(ng);
        __builtin_amdgcn_s_setprio(0);
        __syncthreads();
        fft_block_lines<T, N>(lds, tw);
        if (MODE == 0 && !kEarly) {
#pragma unroll
            for (int it = 0; it < C::IT; ++it) {
                const int e = threadIdx.x + it * C::NT;
                const unsigned P = grp * C::L + e / N;
                const int k = e % N;
                pb[it] = (P < nlines) ? cpx<T>{out[(2 * P) * N + k], out[(2 * P + 1) * N + k]} : cpx<T>{T(0), T(0)};
            }
        }
#pragma unroll
        for (int it = 0; it < C::IT; ++it) {
            const int e = threadIdx.x + it * C::NT;
            const int l = e / N, k = e % N;
            const unsigned P = grp * C::L + l;
            if (P < nlines) {
                cpx<T> h;
                if constexpr (BCX != 0) {
                    const cpx<T> r = lds[l * C::LS + C::pos(x_slot(k, N, 1))];
                    h = {r.x, -r.y};
                } else {
                    h = hartley(lds[l * C::LS + C::pos(k)], lds[l * C::LS + C::pos((k == 0 ? 0 : N - k))]);
                }
                const unsigned a = (2 * P) * N + k, b = a + N;
                if (MODE == 0) {
                    out[a] = pb[it].x + h.x - shift;
                    out[b] = pb[it].y + h.y - shift;
                } else {
                    out[a] = h.x;
                    out[b] = h.y;
                }
            }
        }
        grp = ng;
        if (grp >= ngroups) break;
        __syncthreads();
    }
}

// ---- launch ---------------------------------------------------------------------

// Blocks of a persistent sweep: every resident block of the device, shared by
// the slots of the batch, never more than there are line groups.
// The occupancy of each kernel is asked once and kept in a fixed table (no
// host allocation on the launch path; a kernel beyond the table's capacity is
// asked every time).
static int device_cus() {
    static std::once_flag once;
    static int cus = 256;
    std::call_once(once, [] {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && n >= 1)
            cus = n;
    });
    return cus;
}

static int resident_blocks(const void* kernel, int threads) {
    constexpr int kCap = 4096;  // a power of two, above the number of kernels
    static std::mutex mu;
    static const void* keys[kCap] = {};
    static int vals[kCap] = {};
    const int cus = device_cus();
    std::lock_guard<std::mutex> lock(mu);
    const uintptr_t hsh = (reinterpret_cast<uintptr_t>(kernel) >> 4) * 0x9E3779B97F4A7C15ull;
    for (int probe = 0; probe < kCap; ++probe) {
        const int at = (int)((hsh + (uintptr_t)probe) & (kCap - 1));
        if (keys[at] == kernel) return vals[at] * cus;
        if (keys[at] == nullptr) {
            int nb = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1) nb = 1;
            keys[at] = kernel;
            vals[at] = nb;
            return nb * cus;
        }
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1) nb = 1;
    return nb * cus;
}

// A share of at most one half (a very large size class served beside small
// ones) is a share of the CUs: one block per CU over that share, each block
// reserving the rest of its CU's LDS (reserve_lds), so that no block of
// another kernel shares a CU with it and the dispatcher, which spreads blocks
// over the CUs, leaves the other CUs whole to the small classes.  A larger
// partial share is a share of the resident blocks on every CU.
static unsigned reserve_lds(const void* kernel, float share) {
    if (share > 0.5f) return 0;
    static std::once_flag once;
    static int lds_cu = 0, lds_block = 0;
    std::call_once(once, [] {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return;
        if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess)
            lds_cu = 0;
        if (hipDeviceGetAttribute(&lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            lds_block = 0;
    });
    constexpr int kCap = 1024;  // a power of two, above the number of kernels launched with a half share
    static std::mutex mu;
    static const void* keys[kCap] = {};
    static unsigned vals[kCap] = {};
    std::lock_guard<std::mutex> lock(mu);
    const uintptr_t hsh = (reinterpret_cast<uintptr_t>(kernel) >> 4) * 0x9E3779B97F4A7C15ull;
    int at = -1;
    for (int probe = 0; probe < kCap; ++probe) {
        at = (int)((hsh + (uintptr_t)probe) & (kCap - 1));
        if (keys[at] == kernel) return vals[at];
        if (keys[at] == nullptr) break;
        at = -1;
    }
    unsigned pad = 0;
    hipFuncAttributes fa{};
    if (hipFuncGetAttributes(&fa, kernel) == hipSuccess) {
        const long long total = std::min(lds_cu, lds_block), own = (long long)fa.sharedSizeBytes;
        if (total > own) {
            if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)(total - own)) ==
                hipSuccess)
                pad = (unsigned)(total - own);
            else
                (void)hipGetLastError();  // a refused reservation is not an error of the launch
        }
    } else {
        (void)hipGetLastError();
    }
    if (at >= 0) {
        keys[at] = kernel;
        vals[at] = pad;
    }
    return pad;
}

static int persistent_grid(const void* kernel, int threads, unsigned ngroups, int nslots, float share) {
    int blocks = resident_blocks(kernel, threads);
    if (share <= 0.5f) blocks = std::min(blocks, device_cus());
    const int cap = std::max(1, (int)(blocks * share) / std::max(1, nslots));
    return (int)std::min<unsigned>(ngroups, (unsigned)cap);
}

template <typename T, int MODE>
static hipError_t sweep_t(const GridArgs& g, const Tables& t, const Slot* slots, int nslots, int which,
                          hipStream_t s, int* nunits, float share, int stage) {
    const unsigned rows = (unsigned)(g.ny * g.nz / 2);
    switch (which) {
        case 1:
            return dispatch_len(g.nx, [&]<int N>() {
                using C = LineCfg<T, N>;
                const unsigned ng = (rows + C::L - 1) / C::L;
                return dispatch_op(MODE == 1 ? 0 : g.coef, MODE == 1 ? 0 : g.weight, [&]<int CO, int WE>() {
                    if constexpr (MODE == 0 && use_zmarch<T, N>()) {
                        using Z = P1Tile<T, N>;
                        const unsigned nt = (((unsigned)g.ny / 2 + Z::SUB - 1) / Z::SUB) *
                                            (((unsigned)g.nz + Z::KM - 1) / Z::KM);
                        if (nunits) *nunits = (int)nt;
                        return dispatch_bc(g.bcx, [&]<int BC>() {
                            const void* k = (const void*)&k_resid_dhtx_z<T, N, CO, WE, BC>;
                            const int nb = persistent_grid(k, C::NT, nt, nslots, share);
                            k_resid_dhtx_z<T, N, CO, WE, BC>
                                <<<dim3(nb, nslots), C::NT, reserve_lds(k, share), s>>>(g, slots, t);
                            return hipGetLastError();
                        });
                    } else {
                        const void* k = (const void*)&k_resid_dhtx<T, N, MODE, CO, WE>;
                        const int nb = persistent_grid(k, C::NT, ng, nslots, share);
                        if (nunits) *nunits = (int)ng;
                        k_resid_dhtx<T, N, MODE, CO, WE><<<dim3(nb, nslots), C::NT, reserve_lds(k, share), s>>>(g, slots, t);
                    }
                    return hipGetLastError();
                });
            });
        case 2:
            return dispatch_len(g.ny, [&]<int N>() {
                using C = LineCfg<T, N>;
                const unsigned ng = ((unsigned)(g.nxh * g.nz) + C::L - 1) / C::L;
                const void* k = (const void*)&k_dht_cols<T, N, 1, MODE>;
                const int nb = persistent_grid(k, C::NT, ng, nslots, share);
                k_dht_cols<T, N, 1, MODE><<<dim3(nb, nslots), C::NT, reserve_lds(k, share), s>>>(g, slots, t, stage);
                return hipGetLastError();
            });
        case 3:
            return dispatch_len(g.nz, [&]<int N>() {
                using Z = ZCfg<T, N>;
                using C = LineShape<T, N, Z::ZL>;
                const unsigned ng = ((unsigned)(g.nxh * g.ny) + C::L - 1) / C::L;
                const void* k = (const void*)&k_dht_z_solve<T, N, MODE, Z::ZL, Z::PF, Z::MINW>;
                const int nb = persistent_grid(k, C::NT, ng, nslots, share);
                k_dht_z_solve<T, N, MODE, Z::ZL, Z::PF, Z::MINW>
                    <<<dim3(nb, nslots), C::NT, reserve_lds(k, share), s>>>(g, slots, t, stage);
                return hipGetLastError();
            });
        case 5:
            return dispatch_len(g.nx, [&]<int N>() {
                using C = LineCfg<T, N>;
                const unsigned ng = (rows + C::L - 1) / C::L;
                return dispatch_bc(g.bcx, [&]<int BC>() {
                    const void* k = (const void*)&k_dhtx_update<T, N, MODE, BC>;
                    const int nb = persistent_grid(k, C::NT, ng, nslots, share);
                    if constexpr (MODE == 0 && sizeof(T) == 4) {
                        if (stage == kStageTail) {
                            const void* k2 = (const void*)&k_dhtx_update<T, N, 2, BC>;
                            k_dhtx_update<T, N, 2, BC>
                                <<<dim3(nb, nslots), C::NT, reserve_lds(k2, share), s>>>(g, slots, t, stage);
                            return hipGetLastError();
                        }
                    }
                    k_dhtx_update<T, N, MODE, BC><<<dim3(nb, nslots), C::NT, reserve_lds(k, share), s>>>(g, slots, t, stage);
                    return hipGetLastError();
                });
            });
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_mode(const GridArgs& g, const Tables& t, const Slot* slots, int nslots, bool fp32, int which,
                             int mode, hipStream_t s, int* nunits, float share, int stage) {
    if (mode == 1)
        return fp32 ? sweep_t<float, 1>(g, t, slots, nslots, which, s, nunits, share, 1)
                    : sweep_t<double, 1>(g, t, slots, nslots, which, s, nunits, share, 1);
    return fp32 ? sweep_t<float, 0>(g, t, slots, nslots, which, s, nunits, share, stage)
                : sweep_t<double, 0>(g, t, slots, nslots, which, s, nunits, share, 1);
}

template <int N>
constexpr bool outer_fusable_len() {
    if constexpr (N % 64 != 0) return false;
    else return OuterTile<N>::CPT == 1;
}

bool outer_fusable(const GridArgs& g) {
    bool ok = false;
    (void)dispatch_len(g.nx, [&]<int N>() {
        ok = outer_fusable_len<N>();
        return hipSuccess;
    });
    return ok;
}

hipError_t launch_outer_fused(const GridArgs& g, const Tables& t, const Slot* slots, int nslots, hipStream_t s,
                              int* nunits, float share, bool write) {
    return dispatch_len(g.nx, [&]<int N>() {
        if constexpr (outer_fusable_len<N>()) {
            using C = LineCfg<float, N>;
            using Z = OuterTile<N>;
            const unsigned nt = (((unsigned)g.ny / 2 + Z::SUB - 1) / Z::SUB) * (((unsigned)g.nz + Z::KM - 1) / Z::KM);
            if (nunits) *nunits = (int)nt;
            return dispatch_op(g.coef, g.weight, [&]<int CO, int WE>() {
                return dispatch_bc(g.bcx, [&]<int BC>() {
                    const void* k = (const void*)&k_outer_resid_dhtx<N, CO, WE, BC>;
                    const int nb = persistent_grid(k, C::NT, nt, nslots, share);
                    k_outer_resid_dhtx<N, CO, WE, BC>
                        <<<dim3(nb, nslots), C::NT, reserve_lds(k, share), s>>>(g, slots, t, write ? 1 : 0);
                    return hipGetLastError();
                });
            });
        } else {
            return hipErrorInvalidValue;
        }
    });
}

unsigned sweep_groups_x(const GridArgs& g) {
    // line groups of P1 at the FP64 and FP32 configurations (the larger)
    unsigned out = 0;
    (void)dispatch_len(g.nx, [&]<int N>() {
        const unsigned rows = (unsigned)(g.ny * g.nz / 2);
        out = std::max((rows + LineCfg<double, N>::L - 1) / LineCfg<double, N>::L,
                       (rows + LineCfg<float, N>::L - 1) / LineCfg<float, N>::L);
        return hipSuccess;
    });
    return out;
}

}  // namespace pois
