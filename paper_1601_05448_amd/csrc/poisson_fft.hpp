// Device building blocks for the separable real (Hartley) transforms that
// diagonalise the periodic constant-coefficient 7-point Laplacian.
//
// The paper solves the constant-coefficient Poisson equation of eq. (Pois) by
// Fourier transform in the periodic directions (section "Poisson equation").
// Here the transform along each direction is the discrete Hartley transform
//     H(a)_k = sum_j a_j cas(2 pi j k / N),   cas = cos + sin,
// a real, self-inverse (H H = N I) transform whose basis vectors are
// eigenvectors of every symmetric circulant matrix, in particular of the 1-D
// periodic second difference (eigenvalue -4 sin^2(pi k/N)/h^2).  The product
// of the three 1-D transforms therefore diagonalises the 7-point Laplacian on
// the real field itself: no complex spectrum, no layout change, and the same
// kernel serves for the forward and the inverse sweep.
//
// Two real lines a, b are transformed together as one complex line z = a + ib:
// with Z = DFT(z) (kernel exp(-2 pi i jk/N)),
//     H(z)_k = H(a)_k + i H(b)_k = ((1+i) Z_k + (1-i) Z_{N-k}) / 2.
// Row pairs supply (a, b) for the x direction; for y and z the interleaved
// columns (2m, 2m+1) of the x-fastest layout already form complex numbers.
//
// The complex DFT is a Stockham autosort FFT over lines held in LDS: stage s
// of radix R takes butterfly j (of N/R) from elements j + r N/R, twiddles by
// exp(-2 pi i (j mod Ns) r / (Ns R)) (Ns = product of the previous radices),
// applies a length-R DFT in registers and writes to (j div Ns) Ns R + (j mod
// Ns) + r Ns; after the last stage the line is in natural order.  Lengths are
// 2^a or 3*2^a; radices 16, 8, 4, 2 and one final 3.
#pragma once

#include <hip/hip_runtime.h>

namespace pois {

template <typename T>
struct cpx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * (-i)
template <typename T>
__device__ __forceinline__ cpx<T> cmi(cpx<T> a) { return {a.y, -a.x}; }

// Mathematical constants (not tabulated from any library).
constexpr double kSqrtHalf = 0.70710678118654752440084436210484903928;
constexpr double kCosPi8 = 0.92387953251128675612818318939678828682;
constexpr double kSinPi8 = 0.38268343236508977172845998403039886676;
constexpr double kSin2Pi3 = 0.86602540378443864676372317075293618347;  // sqrt(3)/2

// ---- length-R forward DFTs in registers ------------------------------------

template <typename T>
__device__ __forceinline__ void dft2(cpx<T>* v) {
    const cpx<T> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename T>
__device__ __forceinline__ void dft3(cpx<T>* v) {
    const cpx<T> s = cadd(v[1], v[2]);
    const cpx<T> d = csub(v[1], v[2]);
    const cpx<T> a = v[0];
    const cpx<T> m = {a.x - T(0.5) * s.x, a.y - T(0.5) * s.y};
    // -i sin(2pi/3) d
    const cpx<T> t = {T(kSin2Pi3) * d.y, -T(kSin2Pi3) * d.x};
    v[0] = cadd(a, s);
    v[1] = cadd(m, t);
    v[2] = csub(m, t);
}

template <typename T>
__device__ __forceinline__ void dft4v(cpx<T>& v0, cpx<T>& v1, cpx<T>& v2, cpx<T>& v3) {
    const cpx<T> t0 = cadd(v0, v2), t1 = csub(v0, v2);
    const cpx<T> t2 = cadd(v1, v3), t3 = cmi(csub(v1, v3));
    v0 = cadd(t0, t2);
    v2 = csub(t0, t2);
    v1 = cadd(t1, t3);
    v3 = csub(t1, t3);
}

template <typename T>
__device__ __forceinline__ void dft4(cpx<T>* v) { dft4v(v[0], v[1], v[2], v[3]); }

template <typename T>
__device__ __forceinline__ void dft8(cpx<T>* v) {
    cpx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cpx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4v(e0, e1, e2, e3);
    dft4v(o0, o1, o2, o3);
    const T c = T(kSqrtHalf);
    o1 = {c * (o1.x + o1.y), c * (o1.y - o1.x)};   // * exp(-i pi/4)
    o2 = cmi(o2);                                  // * exp(-i pi/2)
    o3 = {c * (o3.y - o3.x), -c * (o3.x + o3.y)};  // * exp(-3i pi/4)
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

// multiply by exp(-2 pi i M / 16) for the M = n2 * k1 values of a 4 x 4 split
template <typename T, int M>
__device__ __forceinline__ cpx<T> tw16(cpx<T> a) {
    if constexpr (M == 0) {
        return a;
    } else if constexpr (M == 4) {
        return cmi(a);
    } else {
        constexpr double c = (M == 1) ? kCosPi8 : (M == 2) ? kSqrtHalf : (M == 3) ? kSinPi8
                             : (M == 6) ? -kSqrtHalf : -kCosPi8;  // M == 9
        constexpr double s = (M == 1) ? -kSinPi8 : (M == 2) ? -kSqrtHalf : (M == 3) ? -kCosPi8
                             : (M == 6) ? -kSqrtHalf : kSinPi8;
        return cmul(a, cpx<T>{T(c), T(s)});
    }
}

template <typename T, int N2>
__device__ __forceinline__ void dft16_col(cpx<T>* v) {
    // length-4 DFT over n1 of v[4 n1 + N2], then twiddle by exp(-2pi i N2 k1/16)
    dft4v(v[N2], v[4 + N2], v[8 + N2], v[12 + N2]);
    v[4 + N2] = tw16<T, N2 * 1>(v[4 + N2]);
    v[8 + N2] = tw16<T, N2 * 2>(v[8 + N2]);
    v[12 + N2] = tw16<T, N2 * 3>(v[12 + N2]);
}

template <typename T>
__device__ __forceinline__ void dft16(cpx<T>* v) {
    // index n = 4 n1 + n2, k = k1 + 4 k2; after the column pass v[4 k1 + n2]
    // holds Y[n2][k1]; the row pass over n2 gives X[k1 + 4 k2].
    dft16_col<T, 0>(v);
    dft16_col<T, 1>(v);
    dft16_col<T, 2>(v);
    dft16_col<T, 3>(v);
    cpx<T> out[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cpx<T> a = v[4 * k1 + 0], b = v[4 * k1 + 1], c = v[4 * k1 + 2], d = v[4 * k1 + 3];
        dft4v(a, b, c, d);
        out[k1] = a;
        out[k1 + 4] = b;
        out[k1 + 8] = c;
        out[k1 + 12] = d;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = out[r];
}

template <typename T, int R>
__device__ __forceinline__ void dft(cpx<T>* v) {
    if constexpr (R == 2) dft2(v);
    else if constexpr (R == 3) dft3(v);
    else if constexpr (R == 4) dft4(v);
    else if constexpr (R == 8) dft8(v);
    else dft16(v);
}

// ---- line geometry ------------------------------------------------------------

constexpr int pick_radix(int rem) {
    return rem % 16 == 0 ? 16 : rem % 8 == 0 ? 8 : rem % 4 == 0 ? 4 : rem % 2 == 0 ? 2 : 3;
}

// LDS words of a line of n complex values: one pad after every 16 values (the
// radix-16 stages of a Stockham FFT access a line at stride 16) and an odd
// total, so that both in-line strides and the line-to-line stride spread over
// the banks.
constexpr int line_stride(int n) { return n >= 16 ? ((n + n / 16) | 1) : (n | 1); }

// Lines of 512 elements (and FP32 lines of 1024) take 512 threads' worth of
// lines (one block of 8 waves per CU, up to 150000 bytes of LDS), so that the
// column sweeps read runs of 8 or 16 complex values per row and the z-marching
// stencil has one column per thread; other lines take 256 (or 192) threads, two
// blocks per CU (82000 bytes of LDS each).  (FP64 lines of 1024 in 512-thread
// blocks would leave their update sweep too few registers.)  The budget halves
// the lines where needed.
constexpr int lines_per_block(int tt, int n, int elem_bytes) {
    const bool big = tt >= 32 && 512 % tt == 0 && (n <= 512 || elem_bytes <= 8);
    int l = big ? 512 / tt : (256 % tt == 0) ? 256 / tt : 192 / tt;
    const int budget = big ? 150000 : 82000;
    while (l * line_stride(n) * elem_bytes > budget && ((l / 2) * tt) % 64 == 0) l /= 2;
    return l;
}

// Threads per line TT (one radix-16 butterfly per thread in the first stage),
// LL lines per block (threads a multiple of 64), LDS line stride LS and the LDS
// position pos(e) of element e within a line (see line_stride).
template <typename T, int N, int LL>
struct LineShape {
    static constexpr int TT = N >= 16 ? N / 16 : 1;
    static constexpr int L = LL;
    static constexpr int NT = L * TT;
    static constexpr int IT = N / TT;  // elements per thread when a block walks its L lines
    static constexpr int LS = line_stride(N);
    static_assert(NT % 64 == 0, "block must be whole wavefronts");
    static __device__ __forceinline__ constexpr int pos(int e) { return N >= 16 ? e + e / 16 : e; }
};

// The line shape of the sweeps, L from lines_per_block.
template <typename T, int N>
struct LineCfg : LineShape<T, N, lines_per_block(N >= 16 ? N / 16 : 1, N, (int)sizeof(cpx<T>))> {
    using S = LineShape<T, N, lines_per_block(N >= 16 ? N / 16 : 1, N, (int)sizeof(cpx<T>))>;
    using S::TT, S::L, S::NT, S::IT, S::LS;
    // minimum waves per SIMD (the second __launch_bounds__ argument, which caps
    // the registers per thread) a sweep is sized for: 2 for blocks of up to 256
    // threads (two blocks per CU); 1 for 512-thread blocks, which hold two waves
    // per SIMD by themselves (one block per CU)
    static constexpr int MINB = NT > 256 ? 1 : 2;
};

// One Stockham stage on a line in LDS (all threads of the block call it).
template <typename T, int N, int R, int NS, int TT>
__device__ __forceinline__ void stockham_stage(cpx<T>* ln, int t, const cpx<T>* tw) {
    auto pad = [](int e) { return LineCfg<T, N>::pos(e); };
    constexpr int NB = N / R;
    constexpr int BPT = (NB + TT - 1) / TT;
    cpx<T> v[BPT][R];
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        const int j = t + u * TT;
        if (NB % TT == 0 || j < NB) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[u][r] = ln[pad(j + r * NB)];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        const int j = t + u * TT;
        if (NB % TT == 0 || j < NB) {
            const int jm = j % NS;
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) v[u][r] = cmul(v[u][r], tw[jm * r * (N / (NS * R))]);
            }
            dft<T, R>(v[u]);
            const int base = (j / NS) * NS * R + jm;
#pragma unroll
            for (int r = 0; r < R; ++r) ln[pad(base + r * NS)] = v[u][r];
        }
    }
    __syncthreads();
}

template <typename T, int N, int NS, int TT>
__device__ __forceinline__ void fft_stages(cpx<T>* ln, int t, const cpx<T>* tw) {
    if constexpr (NS < N) {
        constexpr int R = pick_radix(N / NS);
        stockham_stage<T, N, R, NS, TT>(ln, t, tw);
        fft_stages<T, N, NS * R, TT>(ln, t, tw);
    }
}

// Forward complex DFT of every line of the block, in place in LDS.
// Expects the lines written and a barrier passed; ends with a barrier.
template <typename T, int N>
__device__ __forceinline__ void fft_block_lines(cpx<T>* lds, const cpx<T>* tw) {
    using C = LineCfg<T, N>;
    const int line = threadIdx.x / C::TT;
    const int t = threadIdx.x % C::TT;
    fft_stages<T, N, 1, C::TT>(lds + line * C::LS, t, tw);
}

// Forward DFT of the block's lines for N = 256 = 16 x 16 with the line held in
// registers: the thread with column index c (0..15) of a line enters with
// v[a] = x[c + 16 a] and leaves with v[b] = X[c + 16 b].  Writing n = c + 16 a
// and k = k1 + 16 b, X[k] = sum_c W16^(c b) W256^(c k1) sum_a x[c + 16 a] W16^(a k1):
// a length-16 DFT over a in registers, the twiddles W256^(c k1), one transpose
// through the line's LDS row (thread c writes (c, k1) to position 16 k1 + c and
// then reads row 16 c + .., taking over the role k1 = c), and a length-16 DFT
// in registers.  `ln` is the thread's line in LDS (LineCfg<T, 256> layout),
// `tw` the 256 twiddles exp(-2 pi i t/256).  All threads of the block call it:
// it holds two barriers, the second one guarding `ln` for its next writer.
template <typename T>
__device__ __forceinline__ void fft256_regs(cpx<T> (&v)[16], cpx<T>* ln, int c, const cpx<T>* tw) {
    dft16(v);
    // c masked to its range: the twiddle offsets then take full-rate 24-bit
    // multiplies instead of 32-bit ones
    const unsigned cm = (unsigned)c & 15u;
#pragma unroll
    for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmul(v[k1], tw[cm * (unsigned)k1]);
    // the LDS positions pos(e) = e + e/16 in closed form (c < 16), one base
    // register and immediate offsets: pos(16 k1 + c) = 17 k1 + c, pos(16 c + a) =
    // 17 c + a
    cpx<T>* wp = ln + c;
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) wp[17 * k1] = v[k1];
    __syncthreads();
    const cpx<T>* rp = ln + 17 * c;
#pragma unroll
    for (int a = 0; a < 16; ++a) v[a] = rp[a];
    __syncthreads();
    dft16(v);
}

// Forward DFT of the block's lines for N = 512 = 16 x 32, the line held in
// registers by its 32 threads.  The thread with column index c (0..31) enters
// with v[a] = x[c + 32 a] (a = 0..15).  Writing n = c + 32 a and
// k = k1 + 16 k2 (k1 < 16, k2 < 32),
//     X[k] = sum_c W32^(c k2) W512^(c k1) sum_a x[c + 32 a] W16^(a k1):
// a length-16 DFT over a in registers and the twiddles W512^(c k1); one
// transpose through the line's LDS row, after which thread t takes k1 = t/2
// and the half h = t mod 2 of the columns, c = 2 c' + h; a length-16 DFT over
// c' (times W32^(k2') for h = 1) gives the even (h = 0) and odd (h = 1) halves
// of the length-32 DFT over c, which the two partner threads combine:
//     X[k1 + 16 k2'] = E[k2'] + O[k2'],  X[k1 + 16 k2' + 256] = E[k2'] - O[k2'].
// The thread leaves with v[b] = X[k1 + 16 b + 256 h].  The partner of column c
// is column c ^ 1: the lanes of even columns sit in the even rows of 16 lanes of
// their wave and their partners in the row above (reg_col), so one
// v_permlane16_swap per 32-bit word hands both threads of a pair the E and the
// O value.  All threads of the block call it: it holds two barriers, the
// second one guarding `ln` for its next writer.
__device__ __forceinline__ void row_pair(float x, float& ev, float& od) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    ev = __uint_as_float(r[0]);  // the value of the pair's even row
    od = __uint_as_float(r[1]);  // the value of its odd row
}
__device__ __forceinline__ void row_pair(double x, double& ev, double& od) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)u, (unsigned)u, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(u >> 32), (unsigned)(u >> 32), false, false);
    ev = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
    od = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}

template <typename T>
__device__ __forceinline__ void fft512_regs(cpx<T> (&v)[16], cpx<T>* ln, int c, const cpx<T>* tw) {
    dft16(v);
    const unsigned cm = (unsigned)c & 31u;  // as in fft256_regs
#pragma unroll
    for (int k1 = 1; k1 < 16; ++k1) v[k1] = cmul(v[k1], tw[cm * (unsigned)k1]);
    // the LDS positions pos(e) = e + e/16 in closed form (c < 32), one base
    // register and immediate offsets: pos(32 k1 + c) = 34 k1 + c + c/16, and
    // with k1 = c/2, h = c mod 2, pos(32 k1 + 2 q + h) = 34 k1 + h + 2 q + q/8
    cpx<T>* wp = ln + c + (c >> 4);
#pragma unroll
    for (int k1 = 0; k1 < 16; ++k1) wp[34 * k1] = v[k1];
    __syncthreads();
    const int k1 = c >> 1, h = c & 1;
    const cpx<T>* rp = ln + 34 * k1 + h;
#pragma unroll
    for (int q = 0; q < 16; ++q) v[q] = rp[2 * q + (q >> 3)];
    __syncthreads();
    dft16(v);
    // both threads of the pair take E (h = 0) and O (h = 1), apply the odd
    // half's twiddles W32^q = tw[16 q] to O and keep E + O (h = 0) or E - O
    const T sg = h ? T(-1) : T(1);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        cpx<T> e, o;
        row_pair(v[q].x, e.x, o.x);
        row_pair(v[q].y, e.y, o.y);
        if (q > 0) o = cmul(o, tw[16 * q]);
        v[q] = {fma(sg, o.x, e.x), fma(sg, o.y, e.y)};
    }
}

// Column index of the threads of a line in the register paths (N = 256, 512;
// 16 lines per block, so a wave holds four columns of each of its 16 lines,
// lane = line + 16 r): the four columns of wave w are closed under the map
// that pairs the thread holding X[k] with the one holding X[N - k] after the
// forward transform, so that the (k, N - k) exchange stays within the wave.
//   N = 256 (thread c holds X[c + 16 b]; partner column 16 - c, or c for
//   c = 0, 8): wave w holds {2w, 16 - 2w, 2w + 1, 15 - 2w}, wave 0 {0, 8, 1, 15}.
//   N = 512 (thread c holds X[c/2 + 16 b + 256 (c mod 2)]; partner column
//   33 - c, or c ^ 1 for c < 2): wave w holds {2w, 2w + 1, 32 - 2w, 33 - 2w},
//   wave 0 {0, 1, 16, 17}; the column pairs (c, c ^ 1) of fft512_regs stay
//   16 lanes apart.
template <int N>
__device__ __forceinline__ int reg_col(int q) {
    const int w = q >> 2, r = q & 3;
    if constexpr (N == 256) {
        return r == 0 ? 2 * w : r == 1 ? (w == 0 ? 8 : 16 - 2 * w) : r == 2 ? 2 * w + 1 : 15 - 2 * w;
    } else {
        static_assert(N == 512, "register paths: 256 and 512");
        return r == 0 ? 2 * w : r == 1 ? 2 * w + 1 : r == 2 ? (w == 0 ? 16 : 32 - 2 * w) : (w == 0 ? 17 : 33 - 2 * w);
    }
}

// The (k, N - k) exchange after a register transform of a line (N = 256: the
// thread with column c holds X[k] = X[c + 16 b]; N = 512: X[c/2 + 16 b +
// 256 (c mod 2)]) goes through the line's LDS row at the positions pos(k),
// which only the thread's wave writes and reads (reg_col).  X[0] is also
// written to the row's last padding slot, so that the partner of every b sits
// at one base position minus 17 b: the addresses take one register and
// immediate offsets.
template <typename T, int N>
__device__ __forceinline__ void exchange_write(cpx<T>* ln, int c, const cpx<T> (&v)[16]) {
    static_assert(N == 256 || N == 512, "register paths: 256 and 512");
    cpx<T>* w = ln + (N == 256 ? c : (c >> 1) + 272 * (c & 1));  // pos(k) = that + 17 b
#pragma unroll
    for (int b = 0; b < 16; ++b) w[17 * b] = v[b];
    if (c == 0) ln[N == 256 ? 272 : 544] = v[0];
}

// Base of the partner values: X[N - k] of the thread's b-th value is at
// [17 (15 - b)] from the returned pointer (wave order: after exchange_write
// and wave_lds_sync).
template <typename T, int N>
__device__ __forceinline__ const cpx<T>* exchange_partner(const cpx<T>* ln, int c) {
    int pb;
    if constexpr (N == 256) {
        pb = c == 0 ? 272 : 271 - c;
    } else {
        const int k1 = c >> 1, h = c & 1;
        pb = k1 == 0 ? (h == 0 ? 544 : 272) : 271 - k1 + 272 * (1 - h);
    }
    return ln + (pb - 255);
}

// Orders the LDS accesses of one wave: the LDS serves a wave's instructions in
// issue order, so after this point a lane reads what every lane of its wave
// wrote before it (the compiler may not move LDS accesses across it).  Other
// waves are not ordered.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    __builtin_amdgcn_sched_barrier(0);
}

// Hartley value of the pair-packed line at k from its DFT Z:
// ((1+i) Z_k + (1-i) Z_{N-k}) / 2.
template <typename T>
__device__ __forceinline__ cpx<T> hartley(cpx<T> zk, cpx<T> zmk) {
    return {T(0.5) * ((zk.x - zk.y) + (zmk.x + zmk.y)), T(0.5) * ((zk.x + zk.y) + (zmk.y - zmk.x))};
}

// ---- reductions -----------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

}  // namespace pois
