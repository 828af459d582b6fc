// Device-side helpers shared by the sweep kernels (poisson_sweeps.hip) and the
// control and pointwise kernels (poisson_kernels.hip) of libpoisson.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

#include "../../include/poisson.h"
#include "poisson_fft.hpp"
#include "poisson_internal.hpp"

namespace pois {

// Field pointers reach the kernels through the slot records, so the compiler
// sees them as generic (flat) pointers that might alias LDS, which stops it from
// hoisting global loads above LDS stores.  Every field access goes through the
// global address space instead.
#define POIS_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ POIS_GLOBAL T* gptr(T* p) {
    return (POIS_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ const POIS_GLOBAL T* gptr(const T* p) {
    return (const POIS_GLOBAL T*)p;
}

// Complex values in global memory as native two-element vectors (one 8- or
// 16-byte access each).
template <typename T>
struct Vec2;
template <>
struct Vec2<double> {
    typedef double type __attribute__((ext_vector_type(2)));
};
template <>
struct Vec2<float> {
    typedef float type __attribute__((ext_vector_type(2)));
};
template <typename T>
__device__ __forceinline__ cpx<T> gload_c(const POIS_GLOBAL T* base, unsigned idx) {
    const typename Vec2<T>::type v = ((const POIS_GLOBAL typename Vec2<T>::type*)base)[idx];
    return {v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void gstore_c(POIS_GLOBAL T* base, unsigned idx, cpx<T> c) {
    typename Vec2<T>::type v;
    v.x = c.x;
    v.y = c.y;
    ((POIS_GLOBAL typename Vec2<T>::type*)base)[idx] = v;
}

// ---- stencil ------------------------------------------------------------------
// Face coefficients (the paper does not write the discrete operator out):
//   COEF 0: beta = 2 / (rho_a + rho_b)      1/rho with rho averaged to the face
//   COEF 1: beta = (1/rho_a + 1/rho_b) / 2  face average of 1/rho
// The reciprocals of a cell pair come from one hardware reciprocal refined by
// Newton steps (Montgomery's batch trick), branch-free: the values are first
// scaled by 1/rho_max into (0, 2], so that the running products stay normal
// (FP64: one batch, density ratio up to 1e20; FP32: batches of at most four,
// ratio up to 1e8; the set-up rejects larger ratios).

__device__ __forceinline__ double recip(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}
__device__ __forceinline__ float recip(float x) {
    float y = __builtin_amdgcn_rcpf(x);
    const float e = fmaf(-x, y, 1.0f);
    return fmaf(y, e, y);
}

// d[k] <- 1 / d[k], k < K, with one reciprocal
template <typename T, int K>
__device__ __forceinline__ void batch_recip(T* d) {
    T pre[K];
    pre[0] = d[0];
#pragma unroll
    for (int k = 1; k < K; ++k) pre[k] = pre[k - 1] * d[k];
    T inv = recip(pre[K - 1]);
#pragma unroll
    for (int k = K - 1; k > 0; --k) {
        const T r = inv * pre[k - 1];
        inv = inv * d[k];
        d[k] = r;
    }
    d[0] = inv;
}

template <typename T, int K, int OFF>
__device__ __forceinline__ void recip_groups(T* d) {
    if constexpr (OFF < K) {
        constexpr int G = (sizeof(T) == 8) ? K : ((K - OFF) < 4 ? (K - OFF) : 4);
        batch_recip<T, G>(d + OFF);
        recip_groups<T, K, OFF + G>(d);
    }
}

// reciprocals of K values that the caller scaled into (0, 2]
template <typename T, int K>
__device__ __forceinline__ void scaled_recips(T (&d)[K]) {
    recip_groups<T, K, 0>(d);
}

template <typename T>
struct CellOut {
    T r, w, bt, pc;
};
template <typename T>
struct PairOut {
    CellOut<T> a, b;
};

// The 26 inputs of a row pair: the two cells (i, j0, k0) and (i, j0 + 1, k0)
// (j0 even) and their neighbours.  Fetching them is separate from evaluating
// them so that a sweep can keep one pair's loads in flight while it evaluates
// the previous pair.
template <typename T>
struct PairIn {
    // densities and pressures at: a, b, a x-, a x+, b x-, b x+, a y-, b y+, a z-, a z+, b z-, b z+
    T r[12], q[12];
    T ba, bb;  // right-hand side at a, b
};

// 32-bit indices (grids up to 2^31 cells), periodic neighbours.
template <typename T>
__device__ __forceinline__ void pair_fetch(const GridArgs& g, const POIS_GLOBAL T* __restrict__ p,
                                           const POIS_GLOBAL T* __restrict__ rho,
                                           const POIS_GLOBAL T* __restrict__ rhs, int i, int j0, int k0,
                                           PairIn<T>& in) {
    const unsigned nx = g.nx, ny = g.ny, nz = g.nz, sz = nx * ny;
    const unsigned a = ((unsigned)k0 * ny + j0) * nx + i, b = a + nx;
    const unsigned axm = (i == 0) ? a + (nx - 1) : a - 1;
    const unsigned axp = (i + 1 == g.nx) ? a - (nx - 1) : a + 1;
    const unsigned bxm = axm + nx, bxp = axp + nx;
    const unsigned aym = (j0 == 0) ? a + (ny - 1) * nx : a - nx;
    const unsigned byp = (j0 + 2 == g.ny) ? b - (ny - 1) * nx : b + nx;
    const unsigned azm = (k0 == 0) ? a + (nz - 1) * sz : a - sz, bzm = azm + nx;
    const unsigned azp = (k0 + 1 == g.nz) ? a - (nz - 1) * sz : a + sz, bzp = azp + nx;
    const unsigned at[12] = {a, b, axm, axp, bxm, bxp, aym, byp, azm, azp, bzm, bzp};
#pragma unroll
    for (int k = 0; k < 12; ++k) in.r[k] = rho[at[k]];
#pragma unroll
    for (int k = 0; k < 12; ++k) in.q[k] = p[at[k]];
    in.ba = rhs[a];
    in.bb = rhs[b];
}

// Walls in x (bcx = 1): the faces x = 0 and x = Lx carry no flux.  Bit 0: the
// cell's x- face is a wall (i = 0), bit 1: its x+ face is (i = nx - 1).  The
// neighbour values across a wall are still read (the periodic wrap) but are
// multiplied by a zero coefficient.
__device__ __forceinline__ unsigned x_walls(const GridArgs& g, unsigned i) {
    return g.bcx ? ((i == 0 ? 1u : 0u) | (i + 1 == (unsigned)g.nx ? 2u : 0u)) : 0u;
}

// The lower z-face coefficients of both rows of a pair, COEF 0 (the start of a
// z march; later planes carry them, see pair_eval with ZC).
template <typename T>
__device__ __forceinline__ void z_faces_below(const PairIn<T>& in, T rinv, T* zc) {
    T d[2] = {(in.r[8] + in.r[0]) * rinv, (in.r[10] + in.r[1]) * rinv};
    scaled_recips(d);
    const T c = T(2) * rinv;
    zc[0] = c * d[0];
    zc[1] = c * d[1];
}

// Residual b~ - A p and weight w of the pair; its 11 faces (a x-, a x+, a y-,
// a|b, a z-, a z+, b x-, b x+, b y+, b z-, b z+) share one batched reciprocal.
// rmax = max rho, rinv = 1 / rmax; `walls` from x_walls for the pair's column.
// ZC (COEF 0, a z march): the two lower z faces come in through zc and the two
// upper ones go out through it, 9 faces computed instead of 11.
template <typename T, int COEF, int WEIGHT, bool ZC = false>
__device__ __forceinline__ PairOut<T> pair_eval(const GridArgs& g, const PairIn<T>& in, T rhs_mean, T rmax,
                                                T rinv, unsigned walls, T* zc = nullptr) {
    const T* r = in.r;
    const T* q = in.q;
    T be[11];
    if constexpr (COEF == 0 && ZC) {
        // the lower z faces of both rows are the upper ones of the plane below
        // (the same two densities, summed in the same order): taken from zc,
        // which receives this plane's upper z faces for the plane above
        T d[9] = {r[2] + r[0], r[0] + r[3], r[6] + r[0], r[0] + r[1], r[0] + r[9],
                  r[4] + r[1], r[1] + r[5], r[1] + r[7], r[1] + r[11]};
#pragma unroll
        for (int f = 0; f < 9; ++f) d[f] *= rinv;
        scaled_recips(d);
        const T c = T(2) * rinv;
        be[0] = c * d[0]; be[1] = c * d[1]; be[2] = c * d[2]; be[3] = c * d[3]; be[4] = zc[0];
        be[5] = c * d[4]; be[6] = c * d[5]; be[7] = c * d[6]; be[8] = c * d[7]; be[9] = zc[1];
        be[10] = c * d[8];
        zc[0] = be[5];
        zc[1] = be[10];
    } else if constexpr (COEF == 0) {
        T d[11] = {r[2] + r[0], r[0] + r[3], r[6] + r[0], r[0] + r[1], r[8] + r[0], r[0] + r[9],
                   r[4] + r[1], r[1] + r[5], r[1] + r[7], r[10] + r[1], r[1] + r[11]};
#pragma unroll
        for (int f = 0; f < 11; ++f) d[f] *= rinv;
        scaled_recips(d);
        const T c = T(2) * rinv;
#pragma unroll
        for (int f = 0; f < 11; ++f) be[f] = c * d[f];
    } else {
        T v[12];
#pragma unroll
        for (int k = 0; k < 12; ++k) v[k] = r[k] * rinv;
        scaled_recips(v);  // rmax / rho
        const T c = T(0.5) * rinv;
        be[0] = c * (v[2] + v[0]);  be[1] = c * (v[0] + v[3]);  be[2] = c * (v[6] + v[0]);
        be[3] = c * (v[0] + v[1]);  be[4] = c * (v[8] + v[0]);  be[5] = c * (v[0] + v[9]);
        be[6] = c * (v[4] + v[1]);  be[7] = c * (v[1] + v[5]);  be[8] = c * (v[1] + v[7]);
        be[9] = c * (v[10] + v[1]); be[10] = c * (v[1] + v[11]);
    }
    be[0] = (walls & 1u) ? T(0) : be[0];
    be[6] = (walls & 1u) ? T(0) : be[6];
    be[1] = (walls & 2u) ? T(0) : be[1];
    be[7] = (walls & 2u) ? T(0) : be[7];
    const T pa = q[0], pb = q[1];
    const T hx = T(g.ihx2), hy = T(g.ihy2), hz = T(g.ihz2);
    const T gy = be[3] * (pb - pa);  // flux through the shared face
    const T apa = (be[1] * (q[3] - pa) - be[0] * (pa - q[2])) * hx + (gy - be[2] * (pa - q[6])) * hy +
                  (be[5] * (q[9] - pa) - be[4] * (pa - q[8])) * hz;
    const T apb = (be[7] * (q[5] - pb) - be[6] * (pb - q[4])) * hx + (be[8] * (q[7] - pb) - gy) * hy +
                  (be[10] * (q[11] - pb) - be[9] * (pb - q[10])) * hz;
    PairOut<T> o;
    o.a.bt = in.ba - rhs_mean;
    o.b.bt = in.bb - rhs_mean;
    o.a.pc = pa;
    o.b.pc = pb;
    o.a.r = o.a.bt - apa;
    o.b.r = o.b.bt - apb;
    if constexpr (WEIGHT == 0) {
        o.a.w = r[0];
        o.b.w = r[1];
    } else {
        // w = 6 / (sum of the six face coefficients); sum * rmax / 6 lies in [1, rmax/rmin]
        const T c = rmax * T(1.0 / 6.0);
        T sw[2] = {(be[0] + be[1] + be[2] + be[3] + be[4] + be[5]) * c,
                   (be[6] + be[7] + be[3] + be[8] + be[9] + be[10]) * c};
        batch_recip<T, 2>(sw);
        o.a.w = rmax * sw[0];
        o.b.w = rmax * sw[1];
    }
    return o;
}

// ---- z-marching stencil ---------------------------------------------------------
// The stencil sweeps would otherwise fetch each value of p and rho about four
// times through the vector memory path (x, y and z neighbours of every cell),
// which on gfx950 makes them bound by the texture-address rate, not by HBM.  A
// thread instead owns one column i of a row pair (rows 2jp, 2jp+1) and marches
// along z through a tile of planes, keeping the rows of planes k-1, k, k+1 in
// registers: every plane is loaded once, the x neighbours come from the
// neighbouring lanes by DPP wave shifts (the two edge lanes of a wave get the
// column beyond from the neighbouring wave through LDS), and the two y halo rows
// are loaded once per plane.  Columns are spread over whole waves (N a multiple
// of 64).

// v from the neighbouring lane; the lane without a source (lane 0 for a right
// shift, lane 63 for a left shift) receives `edge`.  No select around the DPP:
// a select may be compiled into a branch that masks the source lanes off.
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v, float edge) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                                 __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v, double edge) {
    const long long b = __builtin_bit_cast(long long, v), o = __builtin_bit_cast(long long, edge);
    const int lo = __builtin_amdgcn_update_dpp((int)o, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
constexpr int kDppWaveShr1 = 0x138;  // lane l receives lane l-1
constexpr int kDppWaveShl1 = 0x130;  // lane l receives lane l+1

// p and rho of the pair's rows a (2jp) and b (2jp+1) at one plane, one column
template <typename T>
struct PlaneRows {
    T pa, pb, ra, rb;
};

// Per plane and column, what the stencil needs besides the z column: the y halo
// rows (2jp-1 of a, 2jp+2 of b) and the right-hand side.
template <typename T>
struct PlaneSide {
    T pym, rym, pyp, ryp;
    T ba, bb;
};

// Raw buffer loads (vector memory, no 64-bit address arithmetic per load): the
// resource holds the base of one plane, so the per-thread offset within the
// plane stays a 32-bit constant of the tile while the plane base is uniform
// and lives in scalar registers.  Offsets past the plane read 0 instead of
// faulting.
constexpr int kBufferWord3 = 0x00020000;  // raw (untyped) buffer access on gfx9

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* base, unsigned long long off,
                                                             unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(static_cast<const char*>(base)) + off, (short)0,
                                             (int)bytes, kBufferWord3);
}

template <typename T>
__device__ __forceinline__ T buffer_load(__amdgpu_buffer_rsrc_t r, unsigned voff) {
    if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 0));
    else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 0));
}

template <typename T>
struct ZMarch {
    const T* p;
    const T* rho;
    const T* rhs;
    unsigned nx, nz, sz;
    unsigned ra, rb, rm, rp;  // row offsets (row * nx) of a, b and the two halo rows
    int lane;

    __device__ void rows_of(unsigned jp, unsigned ny) {
        const unsigned ja = 2 * jp, jb = ja + 1;
        ra = ja * nx;
        rb = jb * nx;
        rm = (ja == 0 ? ny - 1 : ja - 1) * nx;
        rp = (jb + 1 == ny ? 0 : jb + 1) * nx;
    }
    __device__ unsigned plane(int k) const {  // periodic plane index (k >= -1)
        return (unsigned)(k + (int)nz) % nz;
    }
    __device__ __amdgpu_buffer_rsrc_t rsrc(const T* f, unsigned kp) const {
        return plane_rsrc(f, (unsigned long long)kp * sz * sizeof(T), sz * (unsigned)sizeof(T));
    }
    // No load sits under divergent control flow: the compiler's wait counts stay
    // exact, so the loads of the next plane really overlap this plane's work.
    __device__ void load_rows(unsigned kp, unsigned i, PlaneRows<T>& r) const {
        const auto bp = rsrc(p, kp), br = rsrc(rho, kp);
        constexpr unsigned S = sizeof(T);
        r.pa = buffer_load<T>(bp, (ra + i) * S);
        r.pb = buffer_load<T>(bp, (rb + i) * S);
        r.ra = buffer_load<T>(br, (ra + i) * S);
        r.rb = buffer_load<T>(br, (rb + i) * S);
    }
    __device__ void load_side(unsigned kp, unsigned i, PlaneSide<T>& s) const {
        const auto bp = rsrc(p, kp), br = rsrc(rho, kp), bb = rsrc(rhs, kp);
        constexpr unsigned S = sizeof(T);
        s.pym = buffer_load<T>(bp, (rm + i) * S);
        s.rym = buffer_load<T>(br, (rm + i) * S);
        s.pyp = buffer_load<T>(bp, (rp + i) * S);
        s.ryp = buffer_load<T>(br, (rp + i) * S);
        s.ba = buffer_load<T>(bb, (ra + i) * S);
        s.bb = buffer_load<T>(bb, (rb + i) * S);
    }
    // The columns beyond a wave's edges come from the neighbouring waves through
    // LDS: `edge` holds, per strip, two slots (lane 0, lane 63) of 4 values for
    // each group of 64 columns.  put: edge lanes publish their values; get (after
    // a barrier): lane 0 reads the left neighbour group's lane 63, lane 63 the
    // right neighbour group's lane 0 (periodic in x).
    __device__ void edge_put(T* edge, unsigned col, const PlaneRows<T>& c) const {
        if (lane == 0 || lane == 63) {
            T* e = edge + ((col / 64) * 2 + (lane == 63 ? 1 : 0)) * 4;
            e[0] = c.pa;
            e[1] = c.pb;
            e[2] = c.ra;
            e[3] = c.rb;
        }
    }
    __device__ PlaneRows<T> edge_get(const T* edge, unsigned col) const {
        const unsigned grp = nx / 64, g = col / 64;
        const unsigned slot = (lane == 0) ? ((g + grp - 1) % grp) * 2 + 1 : ((g + 1) % grp) * 2;
        const T* e = edge + slot * 4;
        return PlaneRows<T>{e[0], e[1], e[2], e[3]};
    }
    // the 26 stencil inputs of the pair at plane k from planes k-1 (zm), k (c), k+1
    // (zp); x neighbours by DPP, the edge lanes taking `ex` (from edge_get)
    __device__ void pair(const PlaneRows<T>& zm, const PlaneRows<T>& c, const PlaneRows<T>& zp,
                         const PlaneSide<T>& s, const PlaneRows<T>& ex, PairIn<T>& in) const {
        const T pa_xm = dpp_move<kDppWaveShr1>(c.pa, ex.pa);
        const T pa_xp = dpp_move<kDppWaveShl1>(c.pa, ex.pa);
        const T pb_xm = dpp_move<kDppWaveShr1>(c.pb, ex.pb);
        const T pb_xp = dpp_move<kDppWaveShl1>(c.pb, ex.pb);
        const T ra_xm = dpp_move<kDppWaveShr1>(c.ra, ex.ra);
        const T ra_xp = dpp_move<kDppWaveShl1>(c.ra, ex.ra);
        const T rb_xm = dpp_move<kDppWaveShr1>(c.rb, ex.rb);
        const T rb_xp = dpp_move<kDppWaveShl1>(c.rb, ex.rb);
        // order of PairIn: a, b, a x-, a x+, b x-, b x+, a y-, b y+, a z-, a z+, b z-, b z+
        in.r[0] = c.ra;  in.r[1] = c.rb;  in.r[2] = ra_xm; in.r[3] = ra_xp; in.r[4] = rb_xm; in.r[5] = rb_xp;
        in.r[6] = s.rym; in.r[7] = s.ryp; in.r[8] = zm.ra; in.r[9] = zp.ra; in.r[10] = zm.rb; in.r[11] = zp.rb;
        in.q[0] = c.pa;  in.q[1] = c.pb;  in.q[2] = pa_xm; in.q[3] = pa_xp; in.q[4] = pb_xm; in.q[5] = pb_xp;
        in.q[6] = s.pym; in.q[7] = s.pyp; in.q[8] = zm.pa; in.q[9] = zp.pa; in.q[10] = zm.pb; in.q[11] = zp.pb;
        in.ba = s.ba;
        in.bb = s.bb;
    }
};

// The blocks of a launch go to the chip's 8 XCDs round-robin (block b to XCD
// b % 8), and every XCD has its own L2.  xcd_block renumbers the blocks so that
// the ones on one XCD hold consecutive numbers: neighbouring z-marching tiles,
// which read each other's y halo rows, then meet in the same L2 instead of
// fetching those rows from HBM again.  A bijection of [0, nb); the identity
// when nb is not a multiple of 8.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb) {
    constexpr unsigned kXcds = 8;
    return (nb % kXcds != 0) ? b : (b % kXcds) * (nb / kXcds) + b / kXcds;
}

// Thread layout of a z-marching tile for rows of length N handled by NT
// threads: SUB strips (row pairs) of N threads each when N < NT, or CPT columns
// per thread when N >= NT.  A tile marches KM planes; every KF planes its L = SUB
// KF lines are full and are transformed and written out ("flushed"), so that the
// two z halo planes a tile reads are shared by KM >= KMIN planes however few
// lines the transform's LDS holds.
template <int N, int NT, int L, int KMIN = 16>
struct ZTile {
    static constexpr int CPT = N >= NT ? N / NT : 1;
    static constexpr int SUB = N >= NT ? 1 : NT / N;
    static constexpr int KF = L / SUB;
    static constexpr int KM = KF >= KMIN ? KF : KMIN;
    static constexpr int EDGE = (N / 64) * 2 * 4;  // edge values per strip and buffer
    static_assert(N % 64 == 0, "columns must fill whole waves");
    static_assert(SUB * KF == L && (N >= NT ? N % NT == 0 : NT % N == 0), "tile shape");
    static_assert(KM % KF == 0 && KF % 2 == 0, "flushes");
};

// Tiles of the residual sweep P1 and of the fused FP32 outer residual: 32
// planes (halo planes shared by twice as many) for FP64 and for FP32 rows of
// 1024 cells; the FP32 sweep on shorter rows keeps 16, which keeps it within
// 128 registers (four waves per SIMD) and, at 512 cells, with two blocks per
// CU, lets neighbouring tiles stay closer in z, so that more of the y halo rows
// they read from each other are still in L2 (measured at 512^3: 1.19 instead
// of 1.38 of the algorithmic bytes, 7% faster).
template <typename T, int N>
using P1Tile = ZTile<N, LineCfg<T, N>::NT, LineCfg<T, N>::L, (sizeof(T) == 8 || N >= 1024) ? 32 : 16>;
template <int N>
using OuterTile = ZTile<N, LineCfg<float, N>::NT, LineCfg<float, N>::L, 32>;

// One cell, plain IEEE divisions: the stand-alone operator and residual sweeps
// (parity checks), which need no state and are off the iteration's path.
template <typename T>
__device__ __forceinline__ T face_beta(int coef, T ra, T rb) {
    return coef == 0 ? T(2) / (ra + rb) : (ra + rb) / (T(2) * ra * rb);
}

template <typename T>
__device__ __forceinline__ CellOut<T> cell_residual(const GridArgs& g, const POIS_GLOBAL T* __restrict__ p,
                                                    const POIS_GLOBAL T* __restrict__ rho,
                                                    const POIS_GLOBAL T* __restrict__ rhs, T rhs_mean, int i,
                                                    int j, int k) {
    const unsigned nx = g.nx, ny = g.ny, nz = g.nz, sz = nx * ny;
    const unsigned c = ((unsigned)k * ny + j) * nx + i;
    const unsigned cxm = (i == 0) ? c + (nx - 1) : c - 1;
    const unsigned cxp = (i + 1 == g.nx) ? c - (nx - 1) : c + 1;
    const unsigned cym = (j == 0) ? c + (ny - 1) * nx : c - nx;
    const unsigned cyp = (j + 1 == g.ny) ? c - (ny - 1) * nx : c + nx;
    const unsigned czm = (k == 0) ? c + (nz - 1) * sz : c - sz;
    const unsigned czp = (k + 1 == g.nz) ? c - (nz - 1) * sz : c + sz;
    const T rc = rho[c];
    const unsigned walls = x_walls(g, (unsigned)i);
    const T bxm = (walls & 1u) ? T(0) : face_beta<T>(g.coef, rho[cxm], rc);
    const T bxp = (walls & 2u) ? T(0) : face_beta<T>(g.coef, rc, rho[cxp]);
    const T bym = face_beta<T>(g.coef, rho[cym], rc), byp = face_beta<T>(g.coef, rc, rho[cyp]);
    const T bzm = face_beta<T>(g.coef, rho[czm], rc), bzp = face_beta<T>(g.coef, rc, rho[czp]);
    CellOut<T> o;
    o.bt = rhs ? rhs[c] - rhs_mean : T(0);
    const T pc = p[c];
    o.pc = pc;
    const T ap = (bxp * (p[cxp] - pc) - bxm * (pc - p[cxm])) * T(g.ihx2) +
                 (byp * (p[cyp] - pc) - bym * (pc - p[cym])) * T(g.ihy2) +
                 (bzp * (p[czp] - pc) - bzm * (pc - p[czm])) * T(g.ihz2);
    o.r = o.bt - ap;
    o.w = (g.weight == 0) ? rc : T(6) / (bxm + bxp + bym + byp + bzm + bzp);
    return o;
}

// Block-wide deterministic sum of K values; result valid in thread 0.
template <int NT, int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double* red) {
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) red[w * K + q] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            double s = 0.0;
            for (int u = 0; u < NT / 64; ++u) s += red[u * K + q];
            v[q] = s;
        }
    }
}

// Units' K sums, added by the NT threads of a block in a fixed order; the total
// is in out[] of thread 0.
template <int NT, int K>
__device__ __forceinline__ void sum_units(const double* part, unsigned n, double (&out)[K], double* red) {
#pragma unroll
    for (int q = 0; q < K; ++q) out[q] = 0.0;
    for (unsigned u = threadIdx.x; u < n; u += NT)
#pragma unroll
        for (int q = 0; q < K; ++q) out[q] += part[(unsigned long long)u * kPartialStride + q];
    block_sums<NT, K>(out, red);
}

// Store this block's sums of one unit (thread 0 writes), then clear them.
template <int NT, int K>
__device__ __forceinline__ void put_unit_sums(double (&v)[K], double* red, double* dst) {
    block_sums<NT, K>(v, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < K; ++q) dst[q] = v[q];
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = 0.0;
    __syncthreads();  // red is reused by the next unit
}

template <typename T>
struct IterView;

template <>
struct IterView<double> {
    const POIS_GLOBAL double* p; const POIS_GLOBAL double* rhs; const POIS_GLOBAL double* rho;
    POIS_GLOBAL double* W; double rhs_mean, rmax, rinv;
    __device__ IterView(const Slot& s)
        : p(gptr(s.p)), rhs(gptr(s.b)), rho(gptr(s.rho)), W(gptr(s.W)), rhs_mean(s.st->b_mean),
          rmax(s.st->rho_max), rinv(recip(s.st->rho_max)) {}
    static __device__ bool skip(const SolveState* st, int stage = 1) {
        (void)stage;
        return st->done != 0;
    }
    static __device__ bool skip_p1(const SolveState* st) { return st->done != 0; }
};

template <>
struct IterView<float> {
    const POIS_GLOBAL float* p; const POIS_GLOBAL float* rhs; const POIS_GLOBAL float* rho;
    POIS_GLOBAL float* W; float rhs_mean, rmax, rinv;
    __device__ IterView(const Slot& s)
        : p(gptr(s.d32)), rhs(gptr(s.r32)), rho(gptr(s.rho32)), W(gptr(s.W32)),
          rhs_mean((float)s.st->rhs_mean32), rmax((float)s.st->rho_max), rinv(recip((float)s.st->rho_max)) {}
    // `stage`: 1 for the inner sweeps, kStageTail for the rest of a first inner
    // sweep whose residual the outer residual sweep produced
    static __device__ bool skip(const SolveState* st, int stage = 1) {
        return st->done != 0 || st->stage != stage || st->inner_done != 0;
    }
    // the inner residual sweep also idles once the phase is known to end after
    // the iteration in progress (its evaluation is not needed), and while the
    // update of the last evaluation is still due (a launch sequence may end on
    // an evaluation and leave that update to the next one)
    static __device__ bool skip_p1(const SolveState* st) {
        return skip(st) || st->stop_next != 0 || st->upd_due != 0;
    }
};

template <typename T>
__device__ __forceinline__ const cpx<T>* twiddles(const Tables& t, int axis);
template <>
__device__ __forceinline__ const cpx<double>* twiddles<double>(const Tables& t, int axis) {
    return reinterpret_cast<const cpx<double>*>(axis == 0 ? t.twx : axis == 1 ? t.twy : t.twz);
}
template <>
__device__ __forceinline__ const cpx<float>* twiddles<float>(const Tables& t, int axis) {
    return reinterpret_cast<const cpx<float>*>(axis == 0 ? t.twx32 : axis == 1 ? t.twy32 : t.twz32);
}

template <typename T>
__device__ __forceinline__ const T* symbol(const Tables& t, int axis);
template <>
__device__ __forceinline__ const double* symbol<double>(const Tables& t, int axis) {
    return axis == 0 ? t.lamx : axis == 1 ? t.lamy : t.lamz;
}
template <>
__device__ __forceinline__ const float* symbol<float>(const Tables& t, int axis) {
    return axis == 0 ? t.lamx32 : axis == 1 ? t.lamy32 : t.lamz32;
}

// ---- cosine transform along x between walls ---------------------------------------
// With walls in x the constant-coefficient operator is diagonalised by
// cos(pi k (i + 1/2) / N) instead of the Fourier modes.  Both the forward
// transform X_k = sum_i q_i cos(pi k (i + 1/2) / N) and its N-scaled inverse
// y_i = X_0 + 2 sum_{k>0} X_k cos(pi k (i + 1/2) / N) (= N q_i) take one length-N
// complex FFT of a reordered line (Makhoul's even/odd reordering): x index i
// sits at slot i/2 (i even) or N - 1 - (i-1)/2 (i odd).  Two real lines a, b
// travel as one complex line a + i b, like the Hartley pairs.
__device__ __forceinline__ unsigned x_slot(unsigned i, unsigned n, int bcx) {
    return bcx ? ((i & 1u) ? n - 1u - (i >> 1) : (i >> 1)) : i;
}

// forward: Z = FFT of the reordered pair line; (X^a_k, X^b_k) from Z_k, Z_{N-k} and
// w_k = exp(-i pi k / (2N))
template <typename T>
__device__ __forceinline__ cpx<T> dct_out(cpx<T> zk, cpx<T> zm, cpx<T> w) {
    const T ax = w.x * zk.x - w.y * zk.y, ay = w.x * zk.y + w.y * zk.x;    // w Z_k
    const T bx = w.x * zm.x + w.y * zm.y, by = w.y * zm.x - w.x * zm.y;    // w conj(Z_{N-k})
    return {T(0.5) * (ax + bx), T(0.5) * (ay - by)};
}

// inverse, step 1: c_k = X^a_k + i X^b_k and c_{N-k} (zero for k = 0) give the
// FFT input conj(U_k), U_k = conj(w_k) ((c_k.x + c_{N-k}.y) + i (c_k.y - c_{N-k}.x));
// step 2: R = FFT(conj U); slot s holds y^a = R_s.x and y^b = -R_s.y
template <typename T>
__device__ __forceinline__ cpx<T> idct_in(cpx<T> c, cpx<T> cm, cpx<T> w) {
    const T sx = c.x + cm.y, sy = cm.x - c.y;  // conj of the bracket
    return {w.x * sx - w.y * sy, w.x * sy + w.y * sx};
}

template <typename T>
__device__ __forceinline__ const cpx<T>* dct_twiddles(const Tables& t);
template <>
__device__ __forceinline__ const cpx<double>* dct_twiddles<double>(const Tables& t) {
    return reinterpret_cast<const cpx<double>*>(t.twcx);
}
template <>
__device__ __forceinline__ const cpx<float>* dct_twiddles<float>(const Tables& t) {
    return reinterpret_cast<const cpx<float>*>(t.twcx32);
}

// Output k of a forward transform along x of one LDS line: the Hartley pair
// (periodic) or the cosine pair (walls).
template <typename T, int N>
__device__ __forceinline__ cpx<T> x_forward_out(const cpx<T>* line, int k, int bcx, const cpx<T>* twc) {
    using C = LineCfg<T, N>;
    const cpx<T> zk = line[C::pos(k)], zm = line[C::pos(k == 0 ? 0 : N - k)];
    return bcx ? dct_out(zk, zm, twc[k]) : hartley(zk, zm);
}

// 1 / (n (lx + ly + lz)), 0 for the constant mode (the zero-mean gauge)
template <typename T>
__device__ __forceinline__ T inv_symbol(T lx, T ly, T lz, T n) {
    const T lam = lx + ly + lz;
    return lam == T(0) ? T(0) : recip(n * lam);
}

// Calls f.template operator()<N>() for the runtime length n.
template <typename F>
inline hipError_t dispatch_len(int n, F&& f) {
    switch (n) {
        case 4: return f.template operator()<4>();
        case 6: return f.template operator()<6>();
        case 8: return f.template operator()<8>();
        case 12: return f.template operator()<12>();
        case 16: return f.template operator()<16>();
        case 24: return f.template operator()<24>();
        case 32: return f.template operator()<32>();
        case 48: return f.template operator()<48>();
        case 64: return f.template operator()<64>();
        case 96: return f.template operator()<96>();
        case 128: return f.template operator()<128>();
        case 192: return f.template operator()<192>();
        case 256: return f.template operator()<256>();
        case 384: return f.template operator()<384>();
        case 512: return f.template operator()<512>();
        case 768: return f.template operator()<768>();
        case 1024: return f.template operator()<1024>();
        default: return hipErrorInvalidValue;
    }
}

// Calls f.template operator()<BCX>() for the runtime boundary condition in x
// (0 periodic, 1 walls): the hot sweeps are compiled for each, so that the
// periodic ones carry no wall logic.
template <typename F>
inline hipError_t dispatch_bc(int bcx, F&& f) {
    return bcx ? f.template operator()<1>() : f.template operator()<0>();
}

// Calls f.template operator()<COEF, WEIGHT>() for the runtime modes.
template <typename F>
inline hipError_t dispatch_op(int coef, int weight, F&& f) {
    if (coef == 0) return weight == 0 ? f.template operator()<0, 0>() : f.template operator()<0, 1>();
    return weight == 0 ? f.template operator()<1, 0>() : f.template operator()<1, 1>();
}


}  // namespace pois
