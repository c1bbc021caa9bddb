// Pseudofermion force: the derivative of S = phi^dagger r(A) phi with respect
// to the links (the quantity the molecular-dynamics step of Sec. 2.1 needs
// the shifted solutions for).  For U_mu(n) -> exp(i eps T) U_mu(n),
//   dS/deps = i Tr(T F_mu(n)),  F_mu(n) = TA(U_mu(n) M_mu(n)),
//   M_mu(n) = s_mu(n) sum_i alpha_i  y_i(n+mu) x_i(n)^dagger   (n even)
//                                   -x_i(n+mu) y_i(n)^dagger   (n odd)
// with x_i = (A + beta_i)^-1 phi, y_i = D_oe x_i, s_mu(n) = eta_mu(n) times the
// time-boundary sign of the hop n -> n+mu, TA the traceless anti-Hermitian part.
#include "force.h"

#include "algebra.h"

namespace rhmc {

// One thread per (site of one parity, direction); blockIdx.y = mu, blockIdx.z =
// parity.  The sum over right-hand sides and poles runs in the thread, so M
// is formed once per link; each link is written once (or added to, for a
// later group of right-hand sides).
template <typename LT>
__global__ __launch_bounds__(kBlock) void k_force(const LT* __restrict__ links, int nlinks,
                                                  ForceArgs a) {
    const int eo = blockIdx.x * kBlock + threadIdx.x;
    const int mu = blockIdx.y, par = blockIdx.z;
    const Geom& g = a.g;
    if (eo >= g.Vh) return;
    int x, y, z, t;
    site_coords(g, eo, par, x, y, z, t);
    const Hops h = make_hops(g, eo, x, y, z, t);
    const int nb = h.nb[mu];
    const double s = 2.0 * (double)h.coef[mu];   // eta_mu(n) * boundary sign, exactly +-1
    // own vector: x_i(n) at even n, y_i(n) at odd n; neighbour: the other one
    const double2* own = par == 0 ? a.x : a.y;
    const double2* oth = par == 0 ? a.y : a.x;
    const double sg = par == 0 ? s : -s;
    double mr[3][3], mi[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) mr[i][j] = mi[i][j] = 0.0;
    for (int r = 0; r < a.nrhs; ++r) {
        for (int p = 0; p < a.npole; ++p) {
            const size_t base = ((size_t)r * a.npole + p) * 3 * (size_t)g.Vh;
            const double w = sg * a.alpha[p];
            double2 u[3], v[3];   // u = vector at n+mu, v = vector at n
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                u[c] = oth[base + (size_t)c * g.Vh + nb];
                v[c] = own[base + (size_t)c * g.Vh + eo];
            }
            // M += w u v^dagger
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    mr[i][j] += w * (u[i].x * v[j].x + u[i].y * v[j].y);
                    mi[i][j] += w * (u[i].y * v[j].x - u[i].x * v[j].y);
                }
        }
    }
    Link<double> U;
    load_link<false>(links, nlinks, (2 * mu + par) * g.Vh + eo, U);
    // X = U M
    double xr[3][3], xi[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                sr += U.re[i][k] * mr[k][j] - U.im[i][k] * mi[k][j];
                si += U.re[i][k] * mi[k][j] + U.im[i][k] * mr[k][j];
            }
            xr[i][j] = sr;
            xi[i][j] = si;
        }
    if (a.mom) {
        // momentum kick: the coefficients of F = TA(X) in the algebra
        Mat3 Xm;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                Xm.re[i][j] = xr[i][j];
                Xm.im[i][j] = xi[i][j];
            }
        double cf[8];
        algebra_coef(Xm, 1.0, cf);
        const int nl = 8 * g.Vh;
        const int k = (2 * mu + par) * g.Vh + eo;
#pragma unroll
        for (int i = 0; i < 8; ++i) a.mom[(size_t)i * nl + k] -= a.eps * cf[i];
        return;
    }
    // F = (X - X^dagger)/2 - Tr(X - X^dagger)/6
    const double tr = (xi[0][0] + xi[1][1] + xi[2][2]) / 3.0;   // imaginary part of the trace / 3
    const int lex = x + g.Lx * (y + g.Ly * (z + g.Lz * t));
    double2* out = a.out + ((size_t)lex * 4 + mu) * 9;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double fr = 0.5 * (xr[i][j] - xr[j][i]);
            double fi = 0.5 * (xi[i][j] + xi[j][i]);
            if (i == j) fi -= tr;
            if (a.accumulate) {
                const double2 o = out[3 * i + j];
                fr += o.x;
                fi += o.y;
            }
            out[3 * i + j] = make_double2(fr, fi);
        }
}

hipError_t launch_force(const rhmc_gauge* g, const ForceArgs& a, hipStream_t s) {
    const int nlinks = (int)(4 * g->lat.V);
    const dim3 grid((unsigned)((g->lat.Vh + kBlock - 1) / kBlock), 4, 2);
    if (g->u64c)
        hipLaunchKernelGGL(k_force<Fp64x12Link>, grid, dim3(kBlock), 0, s,
                           reinterpret_cast<const Fp64x12Link*>(g->u64c), nlinks, a);
    else if (g->u64)
        hipLaunchKernelGGL(k_force<double2>, grid, dim3(kBlock), 0, s, g->u64, nlinks, a);
    else
        hipLaunchKernelGGL(k_force<HiLoLink>, grid, dim3(kBlock), 0, s,
                           reinterpret_cast<const HiLoLink*>(g->u32), nlinks, a);
    return hipGetLastError();
}

}  // namespace rhmc
