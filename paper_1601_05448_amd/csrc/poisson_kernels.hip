// gfx950 kernels of the variable-density pressure Poisson solve and their
// launchers.
//
// One iteration of the paper's method (section "Poisson equation", eq. (Pois):
// p = p_g + dp, drop rho grad(1/rho).grad dp, solve the constant-coefficient
// equation by transforms in the periodic directions, p_g <- p_g + dp) is, in
// residual form,
//     r = b~ - A p,  q = w r,  dp = L^+ q,  p += dp,
// and runs as five sweeps over the field plus one tiny reduction:
//   P1 k_resid_dhtx   stencil residual, weight, partial norms, Hartley along x -> W
//   F  k_finalize     ||r|| / ||b~||: convergence, divergence, iteration cap
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

// Residual b~ - A p and weight w of the two cells (i, j0, k0) and (i, j0 + 1, k0)
// of a row pair (j0 even), which share their common y face: 11 faces.  32-bit
// indices (grids up to 2^31 cells), periodic neighbours.  All loads first, then
// the arithmetic.  rmax = max rho, rinv = 1 / rmax.
template <typename T, int COEF, int WEIGHT>
__device__ __forceinline__ PairOut<T> pair_residual(const GridArgs& g, const POIS_GLOBAL T* __restrict__ p,
                                                    const POIS_GLOBAL T* __restrict__ rho,
                                                    const POIS_GLOBAL T* __restrict__ rhs, T rhs_mean, T rmax,
                                                    T rinv, int i, int j0, int k0) {
    const unsigned nx = g.nx, ny = g.ny, nz = g.nz, sz = nx * ny;
    const unsigned a = ((unsigned)k0 * ny + j0) * nx + i, b = a + nx;
    const unsigned axm = (i == 0) ? a + (nx - 1) : a - 1;
    const unsigned axp = (i + 1 == g.nx) ? a - (nx - 1) : a + 1;
    const unsigned bxm = axm + nx, bxp = axp + nx;
    const unsigned aym = (j0 == 0) ? a + (ny - 1) * nx : a - nx;
    const unsigned byp = (j0 + 2 == g.ny) ? b - (ny - 1) * nx : b + nx;
    const unsigned azm = (k0 == 0) ? a + (nz - 1) * sz : a - sz, bzm = azm + nx;
    const unsigned azp = (k0 + 1 == g.nz) ? a - (nz - 1) * sz : a + sz, bzp = azp + nx;
    // densities: a, b, a x-, a x+, b x-, b x+, a y-, b y+, a z-, a z+, b z-, b z+
    const T r[12] = {rho[a], rho[b], rho[axm], rho[axp], rho[bxm], rho[bxp],
                     rho[aym], rho[byp], rho[azm], rho[azp], rho[bzm], rho[bzp]};
    const T q[12] = {p[a], p[b], p[axm], p[axp], p[bxm], p[bxp], p[aym], p[byp], p[azm], p[azp], p[bzm], p[bzp]};
    const T ba = rhs[a], bb = rhs[b];
    // faces: a x-, a x+, a y-, a|b, a z-, a z+, b x-, b x+, b y+, b z-, b z+
    T be[11];
    if constexpr (COEF == 0) {
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
    const T pa = q[0], pb = q[1];
    const T hx = T(g.ihx2), hy = T(g.ihy2), hz = T(g.ihz2);
    const T gy = be[3] * (pb - pa);  // flux through the shared face
    const T apa = (be[1] * (q[3] - pa) - be[0] * (pa - q[2])) * hx + (gy - be[2] * (pa - q[6])) * hy +
                  (be[5] * (q[9] - pa) - be[4] * (pa - q[8])) * hz;
    const T apb = (be[7] * (q[5] - pb) - be[6] * (pb - q[4])) * hx + (be[8] * (q[7] - pb) - gy) * hy +
                  (be[10] * (q[11] - pb) - be[9] * (pb - q[10])) * hz;
    PairOut<T> o;
    o.a.bt = ba - rhs_mean;
    o.b.bt = bb - rhs_mean;
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
    const T bxm = face_beta<T>(g.coef, rho[cxm], rc), bxp = face_beta<T>(g.coef, rc, rho[cxp]);
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

template <typename T>
struct IterView;

template <>
struct IterView<double> {
    const POIS_GLOBAL double* p; const POIS_GLOBAL double* rhs; const POIS_GLOBAL double* rho;
    POIS_GLOBAL double* W; double rhs_mean, rmax, rinv;
    __device__ IterView(const Slot& s)
        : p(gptr(s.p)), rhs(gptr(s.b)), rho(gptr(s.rho)), W(gptr(s.W)), rhs_mean(s.st->b_mean),
          rmax(s.st->rho_max), rinv(recip(s.st->rho_max)) {}
    static __device__ bool skip(const SolveState* st) { return st->done != 0; }
};

template <>
struct IterView<float> {
    const POIS_GLOBAL float* p; const POIS_GLOBAL float* rhs; const POIS_GLOBAL float* rho;
    POIS_GLOBAL float* W; float rhs_mean, rmax, rinv;
    __device__ IterView(const Slot& s)
        : p(gptr(s.d32)), rhs(gptr(s.r32)), rho(gptr(s.rho32)), W(gptr(s.W32)),
          rhs_mean((float)s.st->rhs_mean32), rmax((float)s.st->rho_max), rinv(recip((float)s.st->rho_max)) {}
    static __device__ bool skip(const SolveState* st) {
        return st->done != 0 || st->stage != 1 || st->inner_done != 0;
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

// ---- P1: residual, weight, Hartley along x --------------------------------------
// MODE 0: stencil residual from the iteration view; MODE 1: q = b (copy, for the
// stand-alone L^+ sweep).
template <typename T, int N, int MODE, int COEF, int WEIGHT>
__global__ void __launch_bounds__((LineCfg<T, N>::NT))
k_resid_dhtx(GridArgs g, const Slot* __restrict__ slots, Tables tb, int nblk) {
    using C = LineCfg<T, N>;
    __shared__ cpx<T> lds[C::L * C::LS];
    __shared__ cpx<T> tw[N];
    __shared__ double red[(C::NT / 64) * 4];
    const Slot& s = slots[blockIdx.y];
    if (MODE == 0 && IterView<T>::skip(s.st)) return;
    const cpx<T>* twg = twiddles<T>(tb, 0);
    for (int e = threadIdx.x; e < N; e += C::NT) tw[e] = twg[e];

    __shared__ int s_j0[C::L], s_k0[C::L];
    const unsigned nlines = (unsigned)(g.ny * g.nz / 2);
    const unsigned line0 = blockIdx.x * C::L;
    if (threadIdx.x < C::L) {
        const unsigned r0 = 2u * (line0 + threadIdx.x);  // first row of the pair, k*ny + j
        s_j0[threadIdx.x] = (int)(r0 % (unsigned)g.ny);
        s_k0[threadIdx.x] = (int)(r0 / (unsigned)g.ny);
    }
    __syncthreads();
    double acc[4] = {0.0, 0.0, 0.0, 0.0};  // sum r^2, sum bt^2, sum p, sum p^2
    const IterView<T> v(s);
#pragma unroll 2
    for (int it = 0; it < C::IT; ++it) {
        const int e = threadIdx.x + it * C::NT;
        const int l = e / N, i = e % N;
        const unsigned P = line0 + l;
        cpx<T> q = {T(0), T(0)};
        if (P < nlines) {
            const unsigned r0 = 2u * P;
            if (MODE == 0) {
                const PairOut<T> pr = pair_residual<T, COEF, WEIGHT>(g, v.p, v.rho, v.rhs, v.rhs_mean, v.rmax, v.rinv,
                                                                     i, s_j0[l], s_k0[l]);
                const CellOut<T>& a = pr.a;
                const CellOut<T>& b = pr.b;
                q = {a.w * a.r, b.w * b.r};
                acc[0] += (double)a.r * a.r + (double)b.r * b.r;
                acc[1] += (double)a.bt * a.bt + (double)b.bt * b.bt;
                acc[2] += (double)a.pc + (double)b.pc;
                acc[3] += (double)a.pc * a.pc + (double)b.pc * b.pc;
            } else {
                q = {T(gptr(s.b)[r0 * N + i]), T(gptr(s.b)[(r0 + 1) * N + i])};
            }
        }
        lds[l * C::LS + i] = q;
    }
    __syncthreads();
    fft_block_lines<T, N>(lds, tw);
    POIS_GLOBAL T* W = (MODE == 0) ? v.W : (POIS_GLOBAL T*)gptr(s.W);
#pragma unroll
    for (int it = 0; it < C::IT; ++it) {
        const int e = threadIdx.x + it * C::NT;
        const int l = e / N, k = e % N;
        const unsigned P = line0 + l;
        if (P < nlines) {
            const cpx<T> h = hartley(lds[l * C::LS + k], lds[l * C::LS + (k == 0 ? 0 : N - k)]);
            W[(2 * P) * N + k] = h.x;
            W[(2 * P + 1) * N + k] = h.y;
        }
    }
    if (MODE == 0) {
        block_sums<C::NT, 4>(acc, red);
        if (threadIdx.x == 0) {
            double* out = s.partial + (long long)blockIdx.x * kPartialStride;
            out[0] = acc[0]; out[1] = acc[1]; out[2] = acc[2]; out[3] = acc[3];
        }
    }
    (void)nblk;
}

// ---- P2 / P4: Hartley along y (AX = 1) of the pair-packed columns -------------
// Line = (o, m): complex column m (real columns 2m, 2m+1) at outer index o;
// element e along the axis.  y: address (o*ny + e)*nxh + m; z: (e*ny + o)*nxh + m.
// Each block computes the base address of its lines once.
template <int AX>
__device__ __forceinline__ void line_bases(const GridArgs& g, unsigned line0, int L, unsigned* base) {
    if ((int)threadIdx.x < L) {
        const unsigned line = line0 + threadIdx.x;
        const unsigned nxh = g.nxh, o = line / nxh, m = line - o * nxh;
        base[threadIdx.x] = (AX == 1) ? o * (unsigned)g.ny * nxh + m : o * nxh + m;
    }
}

template <typename T, int N, int AX, int MODE>
__global__ void __launch_bounds__((LineCfg<T, N>::NT))
k_dht_cols(GridArgs g, const Slot* __restrict__ slots, Tables tb) {
    using C = LineCfg<T, N>;
    __shared__ cpx<T> lds[C::L * C::LS];
    __shared__ cpx<T> tw[N];
    __shared__ unsigned base[C::L];
    const Slot& s = slots[blockIdx.y];
    if (MODE == 0 && IterView<T>::skip(s.st)) return;
    const cpx<T>* twg = twiddles<T>(tb, AX);
    for (int e = threadIdx.x; e < N; e += C::NT) tw[e] = twg[e];
    POIS_GLOBAL T* Wc = MODE == 0 ? IterView<T>(s).W : (POIS_GLOBAL T*)gptr(s.W);  // complex-indexed
    const unsigned nlines = (AX == 1) ? (unsigned)(g.nxh * g.nz) : (unsigned)(g.nxh * g.ny);
    const unsigned se = (AX == 1) ? (unsigned)g.nxh : (unsigned)(g.nxh * g.ny);
    const unsigned line0 = blockIdx.x * C::L;
    line_bases<AX>(g, line0, C::L, base);
    __syncthreads();
#pragma unroll
    for (int it = 0; it < C::IT; ++it) {
        const int e = threadIdx.x + it * C::NT;
        const int l = e % C::L, idx = e / C::L;
        cpx<T> q = {T(0), T(0)};
        if (line0 + l < nlines) q = gload_c(Wc, base[l] + idx * se);
        lds[l * C::LS + idx] = q;
    }
    __syncthreads();
    fft_block_lines<T, N>(lds, tw);
#pragma unroll
    for (int it = 0; it < C::IT; ++it) {
        const int e = threadIdx.x + it * C::NT;
        const int l = e % C::L, idx = e / C::L;
        if (line0 + l < nlines)
            gstore_c(Wc, base[l] + idx * se, hartley(lds[l * C::LS + idx], lds[l * C::LS + (idx == 0 ? 0 : N - idx)]));
    }
}

// ---- P3: Hartley along z, divide by n * symbol, Hartley along z ----------------
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

// 1 / (n (lx + ly + lz)), 0 for the constant mode (the zero-mean gauge)
template <typename T>
__device__ __forceinline__ T inv_symbol(T lx, T ly, T lz, T n) {
    const T lam = lx + ly + lz;
    return lam == T(0) ? T(0) : recip(n * lam);
}

template <typename T, int N, int MODE>
__global__ void __launch_bounds__((LineCfg<T, N>::NT))
k_dht_z_solve(GridArgs g, const Slot* __restrict__ slots, Tables tb) {
    using C = LineCfg<T, N>;
    __shared__ cpx<T> lds[C::L * C::LS];
    __shared__ cpx<T> tw[N];
    __shared__ unsigned base[C::L];
    __shared__ T lxe[C::L], lxo[C::L], lyj[C::L];
    const Slot& s = slots[blockIdx.y];
    if (MODE == 0 && IterView<T>::skip(s.st)) return;
    const cpx<T>* twg = twiddles<T>(tb, 2);
    for (int e = threadIdx.x; e < N; e += C::NT) tw[e] = twg[e];
    POIS_GLOBAL T* Wc = MODE == 0 ? IterView<T>(s).W : (POIS_GLOBAL T*)gptr(s.W);  // complex-indexed
    const unsigned nlines = (unsigned)(g.nxh * g.ny);
    const unsigned se = (unsigned)(g.nxh * g.ny);
    const unsigned line0 = blockIdx.x * C::L;
    const T* lx = symbol<T>(tb, 0);
    const T* ly = symbol<T>(tb, 1);
    const T* lz = symbol<T>(tb, 2);
    line_bases<2>(g, line0, C::L, base);
    if ((int)threadIdx.x < C::L) {
        const unsigned line = line0 + threadIdx.x;
        const unsigned j = line / (unsigned)g.nxh, m = line - j * (unsigned)g.nxh;
        const bool in = line < nlines;
        lxe[threadIdx.x] = in ? lx[2 * m] : T(0);
        lxo[threadIdx.x] = in ? lx[2 * m + 1] : T(0);
        lyj[threadIdx.x] = in ? ly[j] : T(0);
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < C::IT; ++it) {
        const int e = threadIdx.x + it * C::NT;
        const int l = e % C::L, idx = e / C::L;
        cpx<T> q = {T(0), T(0)};
        if (line0 + l < nlines) q = gload_c(Wc, base[l] + idx * se);
        lds[l * C::LS + idx] = q;
    }
    __syncthreads();
    fft_block_lines<T, N>(lds, tw);
    // Hartley coefficients of the pair (k, N-k), scaled by 1/(n lambda).
    const T nn = T(g.n);
    constexpr int NP = N / 2 + 1;
    for (int e = threadIdx.x; e < C::L * NP; e += C::NT) {
        const int l = e % C::L, k = e / C::L;
        const int km = (k == 0) ? 0 : N - k;
        const cpx<T> zk = lds[l * C::LS + k], zm = lds[l * C::LS + km];
        cpx<T> hk = hartley(zk, zm), hm = hartley(zm, zk);
        const T lzk = lz[k], lzm = lz[km];
        hk.x *= inv_symbol(lxe[l], lyj[l], lzk, nn);
        hk.y *= inv_symbol(lxo[l], lyj[l], lzk, nn);
        hm.x *= inv_symbol(lxe[l], lyj[l], lzm, nn);
        hm.y *= inv_symbol(lxo[l], lyj[l], lzm, nn);
        lds[l * C::LS + k] = hk;
        lds[l * C::LS + km] = hm;
    }
    __syncthreads();
    fft_block_lines<T, N>(lds, tw);
#pragma unroll
    for (int it = 0; it < C::IT; ++it) {
        const int e = threadIdx.x + it * C::NT;
        const int l = e % C::L, idx = e / C::L;
        if (line0 + l < nlines)
            gstore_c(Wc, base[l] + idx * se, hartley(lds[l * C::LS + idx], lds[l * C::LS + (idx == 0 ? 0 : N - idx)]));
    }
}

// ---- P5: Hartley along x, update -----------------------------------------------
// MODE 0: FP64 p += dp - p_shift (or FP32 d32 += dp); MODE 1: assign to p (L^+ sweep).
template <typename T, int N, int MODE>
__global__ void __launch_bounds__((LineCfg<T, N>::NT))
k_dhtx_update(GridArgs g, const Slot* __restrict__ slots, Tables tb) {
    using C = LineCfg<T, N>;
    __shared__ cpx<T> lds[C::L * C::LS];
    __shared__ cpx<T> tw[N];
    const Slot& s = slots[blockIdx.y];
    if (MODE == 0 && IterView<T>::skip(s.st)) return;
    const cpx<T>* twg = twiddles<T>(tb, 0);
    for (int e = threadIdx.x; e < N; e += C::NT) tw[e] = twg[e];
    const POIS_GLOBAL T* W = (MODE == 0) ? IterView<T>(s).W : (const POIS_GLOBAL T*)gptr(s.W);
    const unsigned nlines = (unsigned)(g.ny * g.nz / 2);
    const unsigned line0 = blockIdx.x * C::L;
#pragma unroll
    for (int it = 0; it < C::IT; ++it) {
        const int e = threadIdx.x + it * C::NT;
        const int l = e / N, i = e % N;
        const unsigned P = line0 + l;
        cpx<T> q = {T(0), T(0)};
        if (P < nlines) q = {W[(2 * P) * N + i], W[(2 * P + 1) * N + i]};
        lds[l * C::LS + i] = q;
    }
    __syncthreads();
    fft_block_lines<T, N>(lds, tw);
    POIS_GLOBAL T* out;
    if constexpr (sizeof(T) == 8) out = (POIS_GLOBAL T*)gptr(s.p);
    else out = (POIS_GLOBAL T*)gptr(s.d32);
    const T shift = (MODE == 0 && sizeof(T) == 8) ? T(s.st->p_shift) : T(0);
#pragma unroll
    for (int it = 0; it < C::IT; ++it) {
        const int e = threadIdx.x + it * C::NT;
        const int l = e / N, k = e % N;
        const unsigned P = line0 + l;
        if (P < nlines) {
            const cpx<T> h = hartley(lds[l * C::LS + k], lds[l * C::LS + (k == 0 ? 0 : N - k)]);
            const unsigned a = (2 * P) * N + k, b = (2 * P + 1) * N + k;
            if (MODE == 0) {
                out[a] = out[a] + h.x - shift;
                out[b] = out[b] + h.y - shift;
            } else {
                out[a] = h.x;
                out[b] = h.y;
            }
        }
    }
}

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
    for (long long c = (long long)blockIdx.x * kPtThreads + threadIdx.x; c < g.n; c += stride) {
        const double r = gptr(s.rho)[c], b = gptr(s.b)[c];
        if (!(r > 0.0) || !isfinite(r) || !isfinite(b)) bad += 1.0;
        mn = fmin(mn, r);
        mx = fmax(mx, r);
        sb += b;
        sb2 += b * b;
        if (write_rho32) gptr(s.rho32)[c] = (float)r;
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

// ---- convergence control -----------------------------------------------------------

template <int K>
__device__ void sum_partials(const double* part, int nblk, double* out, double* red) {
    // fixed-order two-level sum of K values over nblk blocks (256 threads)
    double v[K];
#pragma unroll
    for (int q = 0; q < K; ++q) v[q] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256)
#pragma unroll
        for (int q = 0; q < K; ++q) v[q] += part[(long long)b * kPartialStride + q];
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        const double t = wave_sum(v[q]);
        if (lane == 0) red[w * K + q] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int q = 0; q < K; ++q) out[q] = red[q] + red[K + q] + red[2 * K + q] + red[3 * K + q];
}

// FP64 path, after P1 of iteration st->iter.
__global__ void __launch_bounds__(256) k_finalize(GridArgs g, const Slot* __restrict__ slots, int nblk) {
    __shared__ double red[16];
    const Slot& s = slots[blockIdx.x];
    SolveState* st = s.st;
    if (st->done) return;
    double sums[4];  // sum r^2, sum bt^2, sum p, sum p^2
    sum_partials<4>(s.partial, nblk, sums, red);
    if (threadIdx.x != 0) return;
    const int k = st->iter;
    st->p_sum = sums[2];
    st->p_sumsq = sums[3];
    // the update of this iteration also removes the mean of p (the zero-mean
    // gauge), so rounding in dp never accumulates a constant
    st->p_shift = sums[2] / (double)g.n;
    if (k == 0) {
        st->b_norm = sqrt(sums[1]);
        if (st->b_norm == 0.0) {
            st->rel = 0.0;
            st->r_norm = 0.0;
            st->hist[0] = 0.0;
            st->done = 1;
            st->status = POISSON_OK;
            return;
        }
    }
    const double rn = sqrt(sums[0]);
    const double rel = rn / st->b_norm;
    st->r_norm = rn;
    st->rel = rel;
    if (k < kHistCap) st->hist[k] = rel;
    if (rel <= st->tol) {
        st->done = 1;
        st->status = POISSON_OK;
    } else if (!(rel < 1e8)) {
        st->done = 1;
        st->status = POISSON_EDIVERGED;
    } else if (k >= st->max_iter) {
        st->done = 1;
        st->status = POISSON_ENOCONV;
    } else {
        st->iter = k + 1;
    }
}

// FP32_REFINE: after the FP64 outer residual of outer step st->iter.
__global__ void __launch_bounds__(256) k_finalize_outer(GridArgs g, const Slot* __restrict__ slots, int nblk) {
    __shared__ double red[20];
    const Slot& s = slots[blockIdx.x];
    SolveState* st = s.st;
    if (st->done || st->stage != 0) return;
    double sums[5];  // sum r^2, sum bt^2, sum p, sum p^2, sum r
    sum_partials<5>(s.partial, nblk, sums, red);
    if (threadIdx.x != 0) return;
    const int m = st->iter;
    st->p_sum = sums[2];
    st->p_sumsq = sums[3];
    if (m == 0) {
        // the mean of the incoming p, removed by the update of step 0
        st->p_shift = sums[2] / (double)g.n;
        st->b_norm = sqrt(sums[1]);
        if (st->b_norm == 0.0) {
            st->rel = 0.0;
            st->r_norm = 0.0;
            st->hist[0] = 0.0;
            st->done = 1;
            st->status = POISSON_OK;
            return;
        }
    }
    const double rn = sqrt(sums[0]);
    const double rel = rn / st->b_norm;
    st->r_norm = rn;
    st->rel = rel;
    if (m < kHistCap) st->hist[m] = rel;
    if (rel <= st->tol) {
        st->done = 1;
        st->status = POISSON_OK;
    } else if (!(rel < 1e8)) {
        st->done = 1;
        st->status = POISSON_EDIVERGED;
    } else if (m >= st->max_outer || st->inner_total >= st->max_iter) {
        st->done = 1;
        st->status = POISSON_ENOCONV;
    } else {
        st->rhs_mean32 = sums[4] * st->inv_s / (double)g.n;
        st->stage = 1;
        st->inner_iter = 0;
        st->inner_done = 0;
        st->since_best = 0;
        st->best_in = INFINITY;
        st->rel_in = 1.0;
    }
}

// FP32_REFINE: after the FP32 P1 of an inner iteration.
__global__ void __launch_bounds__(256) k_finalize_inner(GridArgs g, const Slot* __restrict__ slots, int nblk,
                                                        int max_inner) {
    __shared__ double red[16];
    const Slot& s = slots[blockIdx.x];
    SolveState* st = s.st;
    if (st->done || st->stage != 1 || st->inner_done) return;
    double sums[2];
    sum_partials<2>(s.partial, nblk, sums, red);
    if (threadIdx.x != 0) return;
    const int t = st->inner_iter;
    if (t == 0) st->rhs_norm32 = sqrt(sums[1]);
    const double rel = (st->rhs_norm32 > 0.0) ? sqrt(sums[0]) / st->rhs_norm32 : 0.0;
    st->rel_in = rel;
    bool stop = false;
    if (!(rel < 1e8)) stop = true;  // non-finite or blown up: let the FP64 step judge
    if (rel <= st->inner_tol) stop = true;
    if (rel < 0.9 * st->best_in) {
        st->best_in = rel;
        st->since_best = 0;
    } else {
        ++st->since_best;
    }
    // Stagnation at the FP32 rounding floor: no 10% gain in 8 sweeps after the
    // residual has come down.  The iteration can first grow by orders of
    // magnitude on rough density before it contracts, so no stop counts before
    // the best residual is below half its start.
    if (st->best_in < 0.5 && st->since_best >= 8) stop = true;
    if (t >= max_inner || st->inner_total >= st->max_iter) stop = true;
    if (stop) {
        st->inner_done = 1;
        st->stage = 2;
    } else {
        st->inner_iter = t + 1;
        st->inner_total += 1;
    }
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

// FP32_REFINE outer residual in FP64 on row pairs (the layout of P1, so that the
// neighbour rows of a block are read once from HBM): r = b~ - A p, r32 = r inv_s,
// d32 = 0.  Partials: sum r^2, sum bt^2, sum p, sum p^2, sum r.
constexpr int kOuterElems = 2048;  // (pair, column) elements per block

template <int N, int COEF, int WEIGHT>
__global__ void __launch_bounds__(kPtThreads) k_outer_resid(GridArgs g, const Slot* __restrict__ slots) {
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
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
    for (int e = threadIdx.x; e < RPB * N; e += kPtThreads) {
        const int l = e / N, i = e % N;
        const unsigned P = pair0 + l;
        if (P >= npairs) continue;
        const PairOut<double> pr = pair_residual<double, COEF, WEIGHT>(g, gptr(s.p), gptr(s.rho), gptr(s.b), bm, rmax,
                                                                       rinv, i, s_j0[l], s_k0[l]);
        const unsigned a = (2 * P) * N + i, b = a + N;
        acc[0] += pr.a.r * pr.a.r + pr.b.r * pr.b.r;
        acc[1] += pr.a.bt * pr.a.bt + pr.b.bt * pr.b.bt;
        acc[2] += pr.a.pc + pr.b.pc;
        acc[3] += pr.a.pc * pr.a.pc + pr.b.pc * pr.b.pc;
        acc[4] += pr.a.r + pr.b.r;
        POIS_GLOBAL float* r32 = gptr(s.r32);
        POIS_GLOBAL float* d32 = gptr(s.d32);
        r32[a] = (float)(pr.a.r * inv_s);
        r32[b] = (float)(pr.b.r * inv_s);
        d32[a] = 0.0f;
        d32[b] = 0.0f;
    }
    block_sums<kPtThreads, 5>(acc, red);
    if (threadIdx.x == 0) {
        double* o = s.partial + (unsigned long long)blockIdx.x * kPartialStride;
        o[0] = acc[0]; o[1] = acc[1]; o[2] = acc[2]; o[3] = acc[3]; o[4] = acc[4];
    }
}

template <int N>
static int blocks_outer(const GridArgs& g) {
    constexpr int RPB = N >= kOuterElems ? 1 : kOuterElems / N;
    const long long np = (long long)g.ny * g.nz / 2;
    return (int)((np + RPB - 1) / RPB);
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

// ---- launch helpers ------------------------------------------------------------------

bool length_supported(int n) {
    if (n < 4 || n > 1024) return false;
    int m = n;
    if (m % 3 == 0) m /= 3;
    return (m & (m - 1)) == 0 && m >= 1 && (n % 2 == 0);
}

template <typename T, int N>
static int blocks_rows(const GridArgs& g) {
    const long long nl = (long long)g.ny * g.nz / 2;
    return (int)((nl + LineCfg<T, N>::L - 1) / LineCfg<T, N>::L);
}
template <typename T, int N>
static int blocks_cols(const GridArgs& g, int ax) {
    const long long nl = (ax == 1) ? (long long)g.nxh * g.nz : (long long)g.nxh * g.ny;
    return (int)((nl + LineCfg<T, N>::L - 1) / LineCfg<T, N>::L);
}

// Calls f.template operator()<N>() for the runtime length n.
template <typename F>
static hipError_t dispatch_len(int n, F&& f) {
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

// Calls f.template operator()<COEF, WEIGHT>() for the runtime modes.
template <typename F>
static hipError_t dispatch_op(int coef, int weight, F&& f) {
    if (coef == 0) return weight == 0 ? f.template operator()<0, 0>() : f.template operator()<0, 1>();
    return weight == 0 ? f.template operator()<1, 0>() : f.template operator()<1, 1>();
}

static int pt_blocks(const GridArgs& g) {
    const long long b = (g.n + kPtThreads - 1) / kPtThreads;
    return (int)(b < 4096 ? b : 4096);
}

Geometry make_geometry(const GridArgs& g) {
    Geometry geo{};
    // the FP32 kernels may use other line groups; partial buffers take the larger
    (void)dispatch_len(g.nx, [&]<int N>() {
        geo.blocks_x = std::max(blocks_rows<double, N>(g), blocks_rows<float, N>(g));
        return hipSuccess;
    });
    (void)dispatch_len(g.ny, [&]<int N>() {
        geo.blocks_y = std::max(blocks_cols<double, N>(g, 1), blocks_cols<float, N>(g, 1));
        return hipSuccess;
    });
    (void)dispatch_len(g.nz, [&]<int N>() {
        geo.blocks_z = std::max(blocks_cols<double, N>(g, 2), blocks_cols<float, N>(g, 2));
        return hipSuccess;
    });
    geo.blocks_pt = pt_blocks(g);
    int nbo = 0;
    (void)dispatch_len(g.nx, [&]<int N>() {
        nbo = blocks_outer<N>(g);
        return hipSuccess;
    });
    geo.max_blocks = std::max(std::max(std::max(geo.blocks_x, geo.blocks_pt), nbo), kMaxSetupBlocks);
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

// The five sweeps of one iteration.  MODE 0: iteration on the slot's fields;
// MODE 1: the stand-alone L^+ q sweep (q in slot.b, result in slot.p).
template <typename T, int MODE>
static hipError_t sweeps(const GridArgs& g, const Tables& t, const Slot* slots, int nslots, hipStream_t s,
                         int max_inner) {
    hipError_t e;
    int nbx = 0;
    e = dispatch_len(g.nx, [&]<int N>() {
        nbx = blocks_rows<T, N>(g);
        if constexpr (MODE == 1) {
            k_resid_dhtx<T, N, 1, 0, 0><<<dim3(nbx, nslots), LineCfg<T, N>::NT, 0, s>>>(g, slots, t, nbx);
            return hipGetLastError();
        } else {
            return dispatch_op(g.coef, g.weight, [&]<int C, int W>() {
                k_resid_dhtx<T, N, 0, C, W><<<dim3(nbx, nslots), LineCfg<T, N>::NT, 0, s>>>(g, slots, t, nbx);
                return hipGetLastError();
            });
        }
    });
    if (e != hipSuccess) return e;
    if (MODE == 0) {
        if (sizeof(T) == 8) k_finalize<<<nslots, 256, 0, s>>>(g, slots, nbx);
        else k_finalize_inner<<<nslots, 256, 0, s>>>(g, slots, nbx, max_inner);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    auto ysweep = [&]<int N>() {
        k_dht_cols<T, N, 1, MODE><<<dim3(blocks_cols<T, N>(g, 1), nslots), LineCfg<T, N>::NT, 0, s>>>(g, slots, t);
        return hipGetLastError();
    };
    if ((e = dispatch_len(g.ny, ysweep)) != hipSuccess) return e;
    e = dispatch_len(g.nz, [&]<int N>() {
        k_dht_z_solve<T, N, MODE><<<dim3(blocks_cols<T, N>(g, 2), nslots), LineCfg<T, N>::NT, 0, s>>>(g, slots, t);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    if ((e = dispatch_len(g.ny, ysweep)) != hipSuccess) return e;
    return dispatch_len(g.nx, [&]<int N>() {
        k_dhtx_update<T, N, MODE><<<dim3(blocks_rows<T, N>(g), nslots), LineCfg<T, N>::NT, 0, s>>>(g, slots, t);
        return hipGetLastError();
    });
}

// One sweep of an iteration alone (1: P1, 2: P2, 3: P3, 4: finalize, 5: P5), for timing.
template <typename T>
static hipError_t one_sweep(const GridArgs& g, const Tables& t, const Slot* slots, int nslots, int which,
                            hipStream_t s) {
    switch (which) {
        case 1:
            return dispatch_len(g.nx, [&]<int N>() {
                const int nb = blocks_rows<T, N>(g);
                return dispatch_op(g.coef, g.weight, [&]<int C, int W>() {
                    k_resid_dhtx<T, N, 0, C, W><<<dim3(nb, nslots), LineCfg<T, N>::NT, 0, s>>>(g, slots, t, nb);
                    return hipGetLastError();
                });
            });
        case 2:
            return dispatch_len(g.ny, [&]<int N>() {
                k_dht_cols<T, N, 1, 0><<<dim3(blocks_cols<T, N>(g, 1), nslots), LineCfg<T, N>::NT, 0, s>>>(g, slots,
                                                                                                           t);
                return hipGetLastError();
            });
        case 3:
            return dispatch_len(g.nz, [&]<int N>() {
                k_dht_z_solve<T, N, 0><<<dim3(blocks_cols<T, N>(g, 2), nslots), LineCfg<T, N>::NT, 0, s>>>(g, slots,
                                                                                                            t);
                return hipGetLastError();
            });
        case 5:
            return dispatch_len(g.nx, [&]<int N>() {
                k_dhtx_update<T, N, 0><<<dim3(blocks_rows<T, N>(g), nslots), LineCfg<T, N>::NT, 0, s>>>(g, slots, t);
                return hipGetLastError();
            });
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep(const GridArgs& g, const Tables& t, const Slot* slots, int nslots, bool fp32, int which,
                        hipStream_t s) {
    return fp32 ? one_sweep<float>(g, t, slots, nslots, which, s) : one_sweep<double>(g, t, slots, nslots, which, s);
}

hipError_t launch_iteration(const GridArgs& g, const Geometry& geo, const Tables& t, const Slot* slots,
                            int nslots, bool fp32, hipStream_t s) {
    (void)geo;
    return fp32 ? sweeps<float, 0>(g, t, slots, nslots, s, kMaxInnerPerStep)
                : sweeps<double, 0>(g, t, slots, nslots, s, kMaxInnerPerStep);
}

hipError_t launch_outer_residual(const GridArgs& g, const Geometry& geo, const Slot* slots, int nslots,
                                 hipStream_t s) {
    (void)geo;
    int nb = 0;
    hipError_t e = dispatch_len(g.nx, [&]<int N>() {
        nb = blocks_outer<N>(g);
        return dispatch_op(g.coef, g.weight, [&]<int C, int W>() {
            k_outer_resid<N, C, W><<<dim3(nb, nslots), kPtThreads, 0, s>>>(g, slots);
            return hipGetLastError();
        });
    });
    if (e != hipSuccess) return e;
    k_finalize_outer<<<nslots, 256, 0, s>>>(g, slots, nb);
    return hipGetLastError();
}

hipError_t launch_outer_update(const GridArgs& g, const Geometry& geo, const Slot* slots, int nslots,
                               hipStream_t s) {
    k_outer_update<<<dim3(geo.blocks_pt, nslots), kPtThreads, 0, s>>>(g, slots);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_outer_advance<<<nslots, 64, 0, s>>>(g, slots);
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

hipError_t launch_lap_pinv(const GridArgs& g, const Geometry& geo, const Tables& t, const Slot* slot,
                           hipStream_t s) {
    (void)geo;
    return sweeps<double, 1>(g, t, slot, 1, s, kMaxInnerPerStep);
}

}  // namespace pois
