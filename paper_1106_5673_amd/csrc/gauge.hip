// Gauge sector of the molecular dynamics (Sec. 2, 2.1 and 4.1): the plaquette
// action, its force accumulated straight into the momenta, the exponential
// link update with FP64 reunitarisation, and a download of the canonical
// links.  One lane per link (or per site for the action); every kernel reads
// the FP64 link storage of the gauge object (FP64-12 > FP64-18 > hi + lo).
//
//   S_g = beta sum_n sum_{mu<nu} (1 - Re Tr P_{mu nu}(n) / 3)
//   P_{mu nu}(n) = U_mu(n) U_nu(n+mu) U_mu(n+nu)^dagger U_nu(n)^dagger
//   F_g = -(beta/3) TA(U_mu(n) Sigma_mu(n)),
//   Sigma_mu(n) = sum_{nu != mu} U_nu(n+mu) U_mu(n+nu)^dagger U_nu(n)^dagger
//                              + U_nu(n+mu-nu)^dagger U_mu(n-nu)^dagger U_nu(n-nu)
#include "gauge.h"

#include "algebra.h"

namespace rhmc {

namespace {

// link index of direction mu at site c (x, y, z, t), all coordinates in range
__device__ __forceinline__ int link_at(const Geom& g, const int c[4], int mu) {
    const int lex = c[0] + g.Lx * (c[1] + g.Ly * (c[2] + g.Lz * c[3]));
    return (2 * mu + ((c[0] + c[1] + c[2] + c[3]) & 1)) * g.Vh + (lex >> 1);
}

__device__ __forceinline__ int extent(const Geom& g, int d) {
    return d == 0 ? g.Lx : d == 1 ? g.Ly : d == 2 ? g.Lz : g.Lt;
}

// c[d] += step (step = +-1), periodic
__device__ __forceinline__ void hop(const Geom& g, int c[4], int d, int step) {
    const int L = extent(g, d);
    int v = c[d] + step;
    c[d] = v < 0 ? v + L : (v >= L ? v - L : v);
}

template <typename LT>
__device__ __forceinline__ void load(const LT* links, int nlinks, int k, Mat3& U) {
    load_link<false>(links, nlinks, k, U);
}

// FP64-12: rows 1-2 as stored, row 3 = conj(row1 x row2) in chains of fused
// multiply-adds (the hopping term rebuilds it without contraction so that its
// launch variants agree bit for bit; these kernels have one variant each).
template <>
__device__ __forceinline__ void load<Fp64x12Link>(const Fp64x12Link* links, int nlinks, int k,
                                                  Mat3& U) {
    const LinkPlanes<Fp64x12Link> P = link_planes(links, nlinks);
    const uint32_t o = byte_off(k, 16);
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const double2 v = ldg<false>(P.at(e, o));
        U.re[e / 3][e % 3] = v.x;
        U.im[e / 3][e % 3] = v.y;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        double pr = U.re[0][j1] * U.re[1][j2];
        pr = __builtin_fma(-U.im[0][j1], U.im[1][j2], pr);
        pr = __builtin_fma(-U.re[0][j2], U.re[1][j1], pr);
        pr = __builtin_fma(U.im[0][j2], U.im[1][j1], pr);
        double pi = U.re[0][j1] * U.im[1][j2];
        pi = __builtin_fma(U.im[0][j1], U.re[1][j2], pi);
        pi = __builtin_fma(-U.re[0][j2], U.im[1][j1], pi);
        pi = __builtin_fma(-U.im[0][j2], U.re[1][j1], pi);
        U.re[2][j] = pr;
        U.im[2][j] = -pi;
    }
}

// E = exp(i Q) for Hermitian Q: the series of the matrix scaled to Frobenius
// norm <= 1/2 (terms fall below 1e-17 within 16 orders), then squared back.
__device__ void exp_i(const Mat3& Q, Mat3& E) {
    double n2 = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) n2 += Q.re[i][j] * Q.re[i][j] + Q.im[i][j] * Q.im[i][j];
    int s = 0;
    double f = 1.0;
    while (n2 > 0.25 && s < 60) {
        n2 *= 0.25;
        f *= 0.5;
        ++s;
    }
    Mat3 P, T, N;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            P.re[i][j] = -f * Q.im[i][j];
            P.im[i][j] = f * Q.re[i][j];
        }
    mat_identity(T);
    mat_identity(E);
    for (int k = 1; k <= 24; ++k) {
        mat_mul<false, false>(T, P, N);
        const double inv = 1.0 / (double)k;
        double mx = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                T.re[i][j] = N.re[i][j] * inv;
                T.im[i][j] = N.im[i][j] * inv;
                E.re[i][j] += T.re[i][j];
                E.im[i][j] += T.im[i][j];
                mx = fmax(mx, fabs(T.re[i][j]) + fabs(T.im[i][j]));
            }
        if (mx < 1e-17) break;
    }
    for (int j = 0; j < s; ++j) {
        mat_mul<false, false>(E, E, N);
        E = N;
    }
}

// Rows 1-2 Gram-Schmidt orthonormalised, row 3 = conj(row1 x row2).
__device__ __forceinline__ void reunitarize(Mat3& U) {
    double n0 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) n0 += U.re[0][j] * U.re[0][j] + U.im[0][j] * U.im[0][j];
    const double r0 = 1.0 / sqrt(n0);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        U.re[0][j] *= r0;
        U.im[0][j] *= r0;
    }
    double pr = 0.0, pi = 0.0;   // <row1, row2> = sum conj(row1_j) row2_j
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        pr += U.re[0][j] * U.re[1][j] + U.im[0][j] * U.im[1][j];
        pi += U.re[0][j] * U.im[1][j] - U.im[0][j] * U.re[1][j];
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        U.re[1][j] -= pr * U.re[0][j] - pi * U.im[0][j];
        U.im[1][j] -= pr * U.im[0][j] + pi * U.re[0][j];
    }
    double n1 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) n1 += U.re[1][j] * U.re[1][j] + U.im[1][j] * U.im[1][j];
    const double r1 = 1.0 / sqrt(n1);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        U.re[1][j] *= r1;
        U.im[1][j] *= r1;
    }
    rebuild_row3(U);
}

// Write one link into every storage the gauge object holds (the layouts of
// the link pack: FP64-18 entry planes, FP64-12 rows 1-2, FP32-12 rows 1-2 and
// their FP32 remainders for hi + lo).
__device__ __forceinline__ void store_link(const Mat3& U, int k, int nlinks, double2* u64,
                                           double2* u64c, float4* u32, int hilo, float2* u32f) {
    if (u32f) {
#pragma unroll
        for (int e = 0; e < 9; ++e)
            u32f[(size_t)e * nlinks + k] =
                make_float2((float)U.re[e / 3][e % 3], (float)U.im[e / 3][e % 3]);
    }
    if (u64) {
#pragma unroll
        for (int e = 0; e < 9; ++e)
            u64[(size_t)e * nlinks + k] = make_double2(U.re[e / 3][e % 3], U.im[e / 3][e % 3]);
    }
    if (u64c) {
#pragma unroll
        for (int e = 0; e < 6; ++e)
            u64c[(size_t)e * nlinks + k] = make_double2(U.re[e / 3][e % 3], U.im[e / 3][e % 3]);
    }
    if (u32) {
        double v[12];
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            v[2 * e] = U.re[e / 3][e % 3];
            v[2 * e + 1] = U.im[e / 3][e % 3];
        }
        float h[12], l[12];
#pragma unroll
        for (int i = 0; i < 12; ++i) {
            h[i] = (float)v[i];
            l[i] = (float)(v[i] - (double)h[i]);
        }
#pragma unroll
        for (int p = 0; p < 3; ++p)
            u32[(size_t)p * nlinks + k] = make_float4(h[4 * p], h[4 * p + 1], h[4 * p + 2], h[4 * p + 3]);
        if (hilo) {
#pragma unroll
            for (int p = 0; p < 3; ++p)
                u32[(size_t)(3 + p) * nlinks + k] =
                    make_float4(l[4 * p], l[4 * p + 1], l[4 * p + 2], l[4 * p + 3]);
        }
    }
}

// ------------------------------------------------------------------ kernels
// One lane per link: the six staples, X = U Sigma, and
// mom^a -= eps * scale * i Tr(T^a TA(X)).  The 8 (mu, parity) link classes
// of one range of sites are consecutive blocks, and each XCD takes a
// contiguous run of blocks.  Within a class the sites run x fastest, then t,
// then z inside a slab of sz planes, then y, then slab, so that the t and z
// neighbours of a wave's links are a few blocks away and each XCD holds
// whole slabs.  The kernel is bound by its FP64 arithmetic and load latency
// more than by its bytes: the products are fused multiply-add chains.
template <typename LT>
__global__ __launch_bounds__(kBlock) void k_gauge_force(const LT* links, int nlinks, Geom g,
                                                        FastDiv dsz, double scale, double eps,
                                                        double* __restrict__ mom) {
    const int blk = xcd_remap(blockIdx.x, gridDim.x);
    const int cls = blk & 7;
    const int mu = cls >> 1, par = cls & 1;
    const int p = (blk >> 3) * kBlock + threadIdx.x;
    if (p >= g.Vh) return;
    int n[4];
    {
        int xh, r, zz, slab;
        fdivmod(p, g.dhx, r, xh);
        fdivmod(r, g.dLt, r, n[3]);
        fdivmod(r, dsz, r, zz);
        fdivmod(r, g.dLy, slab, n[1]);
        n[2] = slab * (int)dsz.d + zz;
        n[0] = 2 * xh + ((par + n[1] + n[2] + n[3]) & 1);
    }
    const int eo = (n[0] >> 1) + g.hx * (n[1] + g.Ly * (n[2] + g.Lz * n[3]));
    Mat3 S, A, B, C;
    mat_zero(S);
#pragma unroll 1
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        int a[4] = {n[0], n[1], n[2], n[3]};   // n + mu
        hop(g, a, mu, 1);
        int b[4] = {n[0], n[1], n[2], n[3]};   // n + nu
        hop(g, b, nu, 1);
        int c[4] = {n[0], n[1], n[2], n[3]};   // n - nu
        hop(g, c, nu, -1);
        int d[4] = {c[0], c[1], c[2], c[3]};   // n + mu - nu
        hop(g, d, mu, 1);
        // upper: U_nu(n+mu) U_mu(n+nu)^dagger U_nu(n)^dagger
        load(links, nlinks, link_at(g, a, nu), A);
        load(links, nlinks, link_at(g, b, mu), B);
        mat_mul<false, true>(A, B, C);
        load(links, nlinks, link_at(g, n, nu), A);
        mat_mul<false, true, true>(C, A, S);
        // lower: U_nu(n+mu-nu)^dagger U_mu(n-nu)^dagger U_nu(n-nu)
        load(links, nlinks, link_at(g, d, nu), A);
        load(links, nlinks, link_at(g, c, mu), B);
        mat_mul<true, true>(A, B, C);
        load(links, nlinks, link_at(g, c, nu), A);
        mat_mul<false, false, true>(C, A, S);
    }
    const int k = (2 * mu + par) * g.Vh + eo;
    load(links, nlinks, k, A);
    mat_mul<false, false>(A, S, B);
    double cf[8];
    algebra_coef(B, scale, cf);
#pragma unroll
    for (int i = 0; i < 8; ++i) mom[(size_t)i * nlinks + k] -= eps * cf[i];
}

// One lane per link: U -> reunitarise(exp(i eps H) U), written to every
// storage.  Each lane reads and writes only its own link, so the update is
// in place.
template <typename LT>
__global__ __launch_bounds__(kBlock) void k_update_links(const LT* links, int nlinks, double eps,
                                                         const double* __restrict__ mom,
                                                         double2* u64, double2* u64c, float4* u32,
                                                         int hilo, float2* u32f) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= nlinks) return;
    Mat3 U, H, E, N;
    load(links, nlinks, k, U);
    double w[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) w[i] = eps * mom[(size_t)i * nlinks + k];
    algebra_matrix(w, H);
    exp_i(H, E);
    mat_mul<false, false>(E, U, N);
    reunitarize(N);
    store_link(N, k, nlinks, u64, u64c, u32, hilo, u32f);
}

// Sum over the sites of this lane of sum_{mu<nu} (1 - Re Tr P / 3); one
// partial sum per block.  Re Tr(X Y^dagger) with X = U_mu(n) U_nu(n+mu) and
// Y = U_nu(n) U_mu(n+nu) is the plaquette's.
template <typename LT>
__global__ __launch_bounds__(kBlock) void k_plaquette(const LT* links, int nlinks, Geom g,
                                                      double* __restrict__ partial) {
    double acc = 0.0;
    const int V = 2 * g.Vh;
    for (int i = blockIdx.x * kBlock + threadIdx.x; i < V; i += gridDim.x * kBlock) {
        const int par = i >= g.Vh ? 1 : 0;
        const int eo = i - par * g.Vh;
        int n[4];
        site_coords(g, eo, par, n[0], n[1], n[2], n[3]);
#pragma unroll 1
        for (int mu = 0; mu < 3; ++mu) {
#pragma unroll 1
            for (int nu = mu + 1; nu < 4; ++nu) {
                Mat3 A, B, X, Y;
                int a[4] = {n[0], n[1], n[2], n[3]};
                hop(g, a, mu, 1);
                int b[4] = {n[0], n[1], n[2], n[3]};
                hop(g, b, nu, 1);
                load(links, nlinks, (2 * mu + par) * g.Vh + eo, A);
                load(links, nlinks, link_at(g, a, nu), B);
                mat_mul<false, false>(A, B, X);
                load(links, nlinks, (2 * nu + par) * g.Vh + eo, A);
                load(links, nlinks, link_at(g, b, mu), B);
                mat_mul<false, false>(A, B, Y);
                acc += 1.0 - re_tr_mul_dagger(X, Y) / 3.0;
            }
        }
    }
    __shared__ double sm[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) s += sm[w];
        partial[blockIdx.x] = s;
    }
}

template <typename LT>
__global__ __launch_bounds__(kBlock) void k_get_links(const LT* links, int nlinks, Geom g,
                                                      double2* __restrict__ out) {
    const int eo = blockIdx.x * kBlock + threadIdx.x;
    const int mu = blockIdx.y, par = blockIdx.z;
    if (eo >= g.Vh) return;
    int x, y, z, t;
    site_coords(g, eo, par, x, y, z, t);
    Mat3 U;
    load(links, nlinks, (2 * mu + par) * g.Vh + eo, U);
    const size_t lex = (size_t)x + (size_t)g.Lx * (y + (size_t)g.Ly * (z + (size_t)g.Lz * t));
    double2* o = out + (lex * 4 + mu) * 9;
#pragma unroll
    for (int e = 0; e < 9; ++e) o[e] = make_double2(U.re[e / 3][e % 3], U.im[e / 3][e % 3]);
}

constexpr int kPlaqBlocks = 1024;

}  // namespace

// Dispatch on the FP64 link storage of the gauge object.
#define RHMC_GAUGE_DISPATCH(KERNEL, GRID, ...)                                                   \
    do {                                                                                       \
        const int nl_ = (int)(4 * g->lat.V);                                                   \
        if (g->u64c)                                                                           \
            hipLaunchKernelGGL(KERNEL<Fp64x12Link>, GRID, dim3(kBlock), 0, s,                  \
                               reinterpret_cast<const Fp64x12Link*>(g->u64c), nl_, __VA_ARGS__); \
        else if (g->u64)                                                                       \
            hipLaunchKernelGGL(KERNEL<double2>, GRID, dim3(kBlock), 0, s,                      \
                               (const double2*)g->u64, nl_, __VA_ARGS__);                      \
        else                                                                                   \
            hipLaunchKernelGGL(KERNEL<HiLoLink>, GRID, dim3(kBlock), 0, s,                     \
                               reinterpret_cast<const HiLoLink*>(g->u32), nl_, __VA_ARGS__);   \
    } while (0)

static dim3 link_grid(const rhmc_gauge* g) {
    return dim3((unsigned)((g->lat.Vh + kBlock - 1) / kBlock), 4, 2);
}

hipError_t launch_gauge_force_mom(const rhmc_gauge* g, double beta, double eps, double* mom,
                                  hipStream_t s) {
    const dim3 grid((unsigned)(8 * ((g->lat.Vh + kBlock - 1) / kBlock)));
    // z slabs: Lz / 8 planes (one slab per XCD) when that divides Lz, else the
    // largest divisor of Lz below it (any divisor gives the same momenta)
    const int Lz = g->lat.geom.Lz;
    int sz = Lz / 8 > 0 ? Lz / 8 : 1;
    while (Lz % sz) --sz;
    RHMC_GAUGE_DISPATCH(k_gauge_force, grid, g->lat.geom, make_fastdiv((uint32_t)sz), -beta / 3.0,
                        eps, mom);
    return hipGetLastError();
}

hipError_t launch_update_links(rhmc_gauge* g, double eps, const double* mom, hipStream_t s) {
    const dim3 grid((unsigned)((4 * g->lat.V + kBlock - 1) / kBlock));
    RHMC_GAUGE_DISPATCH(k_update_links, grid, eps, mom, g->u64, g->u64c, g->u32, g->hilo, g->u32f);
    return hipGetLastError();
}

int plaquette_blocks(const rhmc_gauge* g) {
    const int64_t need = (g->lat.V + kBlock - 1) / kBlock;
    return (int)(need < kPlaqBlocks ? need : kPlaqBlocks);
}

hipError_t launch_plaquette(const rhmc_gauge* g, double* partial, hipStream_t s) {
    RHMC_GAUGE_DISPATCH(k_plaquette, dim3((unsigned)plaquette_blocks(g)), g->lat.geom, partial);
    return hipGetLastError();
}

hipError_t launch_get_links(const rhmc_gauge* g, double2* out, hipStream_t s) {
    RHMC_GAUGE_DISPATCH(k_get_links, link_grid(g), g->lat.geom, out);
    return hipGetLastError();
}

}  // namespace rhmc
