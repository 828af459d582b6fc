// The projection step around the pressure solve (appendix A of the paper: the
// time advance divides the predicted momentum by the new density, takes its
// divergence, solves the variable-coefficient Poisson equation, and corrects
// the momentum with the pressure gradient).  Periodic box, or walls in x.
//
//   k_divergence   out = div(u), u = beta m on the faces (MODE 0), or the right-
//                  hand side of the pressure equation (div(u) - RHS^div) / (C dt)
//                  (MODE 1)
//   k_correct      m_d -= C dt (p_{c+e_d} - p_c) / h_d on every face
//
// m_d[c] is the normal momentum on the face between cell c and c + e_d; beta is
// the operator's face coefficient (1 / rho_face), so that the divergence of beta
// times the face gradient of p is exactly the operator A p of the solve.  With
// walls in x the two end faces of every x row are closed: the momentum stored
// for the face between the last and the first cell takes no part in the
// divergence and is not corrected.
//
// Both kernels are single passes over the fields, bound by HBM bandwidth: a
// thread owns one (i, j) column and marches along z through kProjPlanes planes,
// keeping the z neighbours it needs in registers; the x and y neighbours are
// loaded again (the neighbouring lanes and rows of the same block, or the L2).
#include <hip/hip_runtime.h>

#include "poisson_device.hpp"

namespace pois {

constexpr int kProjThreads = 256;
constexpr int kProjPlanes = 16;

template <int MODE>
__global__ void __launch_bounds__(kProjThreads)
k_divergence(GridArgs g, const double* __restrict__ rho_in, const double* __restrict__ mx_in,
             const double* __restrict__ my_in, const double* __restrict__ mz_in, const double* __restrict__ rhs_in,
             double inv_cdt, double* __restrict__ out_in) {
    const unsigned nx = g.nx, ny = g.ny, nz = g.nz, sz = nx * ny;
    const unsigned col = blockIdx.x * kProjThreads + threadIdx.x;
    if (col >= sz) return;
    const POIS_GLOBAL double* rho = gptr(rho_in);
    const POIS_GLOBAL double* mx = gptr(mx_in);
    const POIS_GLOBAL double* my = gptr(my_in);
    const POIS_GLOBAL double* mz = gptr(mz_in);
    POIS_GLOBAL double* out = gptr(out_in);
    const unsigned i = col % nx, j = col / nx;
    const unsigned oxm = (i == 0) ? nx - 1 : (unsigned)-1;  // offsets, modulo 2^32
    const unsigned oxp = (i + 1 == nx) ? (unsigned)-(int)(nx - 1) : 1u;
    const unsigned oym = (j == 0) ? (ny - 1) * nx : (unsigned)-(int)nx;
    const unsigned oyp = (j + 1 == ny) ? (unsigned)-(int)((ny - 1) * nx) : nx;
    const double rhx = std::sqrt(g.ihx2), rhy = std::sqrt(g.ihy2), rhz = std::sqrt(g.ihz2);  // 1 / h_d
    // walls: the coefficient of a closed end face is 0 (multiplied in, so that
    // every load stays unconditional)
    const double open_m = (g.bcx && i == 0) ? 0.0 : 1.0, open_p = (g.bcx && i + 1 == nx) ? 0.0 : 1.0;
    const unsigned k0 = blockIdx.y * kProjPlanes;
    const unsigned k1 = (k0 + kProjPlanes < nz) ? k0 + kProjPlanes : nz;
    unsigned cm = ((k0 + nz - 1) % nz) * sz + col;
    double r_m = rho[cm], mz_m = mz[cm];
    unsigned c = k0 * sz + col;
    double r_c = rho[c];
    for (unsigned k = k0; k < k1; ++k, c += sz) {
        const unsigned cp = (k + 1 == nz) ? col : c + sz;
        const double r_p = rho[cp];
        const double bxm = open_m * face_beta<double>(g.coef, rho[c + oxm], r_c);
        const double bxp = open_p * face_beta<double>(g.coef, r_c, rho[c + oxp]);
        const double bym = face_beta<double>(g.coef, rho[c + oym], r_c), byp = face_beta<double>(g.coef, r_c, rho[c + oyp]);
        const double bzm = face_beta<double>(g.coef, r_m, r_c), bzp = face_beta<double>(g.coef, r_c, r_p);
        const double mzc = mz[c];
        const double d = (bxp * mx[c] - bxm * mx[c + oxm]) * rhx + (byp * my[c] - bym * my[c + oym]) * rhy +
                         (bzp * mzc - bzm * mz_m) * rhz;
        out[c] = (MODE == 0) ? d : (d - rhs_in[c]) * inv_cdt;
        r_m = r_c;
        r_c = r_p;
        mz_m = mzc;
    }
}

__global__ void __launch_bounds__(kProjThreads)
k_correct(GridArgs g, const double* __restrict__ p_in, double* __restrict__ mx_in, double* __restrict__ my_in,
          double* __restrict__ mz_in, double c_dt) {
    const unsigned nx = g.nx, ny = g.ny, nz = g.nz, sz = nx * ny;
    const unsigned col = blockIdx.x * kProjThreads + threadIdx.x;
    if (col >= sz) return;
    const POIS_GLOBAL double* p = gptr(p_in);
    POIS_GLOBAL double* mx = gptr(mx_in);
    POIS_GLOBAL double* my = gptr(my_in);
    POIS_GLOBAL double* mz = gptr(mz_in);
    const unsigned i = col % nx, j = col / nx;
    // walls: the end face's neighbour is the cell itself, so the gradient across
    // it is 0 and the face keeps its momentum (m - C dt 0 / h == m exactly)
    const unsigned oxp = (i + 1 == nx) ? (g.bcx ? 0u : (unsigned)-(int)(nx - 1)) : 1u;
    const unsigned oyp = (j + 1 == ny) ? (unsigned)-(int)((ny - 1) * nx) : nx;
    const double cx = c_dt * std::sqrt(g.ihx2), cy = c_dt * std::sqrt(g.ihy2), cz = c_dt * std::sqrt(g.ihz2);
    const unsigned k0 = blockIdx.y * kProjPlanes;
    const unsigned k1 = (k0 + kProjPlanes < nz) ? k0 + kProjPlanes : nz;
    unsigned c = k0 * sz + col;
    double p_c = p[c];
    for (unsigned k = k0; k < k1; ++k, c += sz) {
        const unsigned cp = (k + 1 == nz) ? col : c + sz;
        const double p_p = p[cp];
        mx[c] -= cx * (p[c + oxp] - p_c);
        my[c] -= cy * (p[c + oyp] - p_c);
        mz[c] -= cz * (p_p - p_c);
        p_c = p_p;
    }
}

static dim3 proj_grid(const GridArgs& g) {
    const unsigned sz = (unsigned)g.nx * (unsigned)g.ny;
    return dim3((sz + kProjThreads - 1) / kProjThreads, ((unsigned)g.nz + kProjPlanes - 1) / kProjPlanes);
}

hipError_t launch_divergence(const GridArgs& g, const double* rho, const double* mx, const double* my,
                             const double* mz, const double* rhs, double c_dt, double* out, hipStream_t s) {
    if (rhs) k_divergence<1><<<proj_grid(g), kProjThreads, 0, s>>>(g, rho, mx, my, mz, rhs, 1.0 / c_dt, out);
    else k_divergence<0><<<proj_grid(g), kProjThreads, 0, s>>>(g, rho, mx, my, mz, nullptr, 1.0, out);
    return hipGetLastError();
}

hipError_t launch_correct(const GridArgs& g, const double* p, double* mx, double* my, double* mz, double c_dt,
                          hipStream_t s) {
    k_correct<<<proj_grid(g), kProjThreads, 0, s>>>(g, p, mx, my, mz, c_dt);
    return hipGetLastError();
}

}  // namespace pois
