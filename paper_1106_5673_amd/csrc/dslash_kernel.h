// Staggered hopping term (Eq. stag, Sec. 2) between the two parities: link
// loaders for every storage of Sec. 4.2 and the hopping kernel, shared by the
// translation units that instantiate it for one link storage each.
//
// One lane owns one output site and every right-hand side of the launch, so
// each link is read once per application however many vectors are batched.
// Links are structure-of-arrays over the link index k = (2*mu + parity)*Vh + eo,
// so the 64 lanes of a wave read 64 consecutive links per load; neighbour
// vectors are colour-major [3][Vh] arrays, read by consecutive sites.
#pragma once

#include "common.h"

namespace rhmc {

// ------------------------------------------------------------------ links
template <typename RT>
struct Link {
    RT re[3][3], im[3][3];
};

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ double2 ldg(const double2* p) {
    if constexpr (NT) {
        const d2v v = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
        return make_double2(v.x, v.y);
    } else {
        return *p;
    }
}

typedef float f2v __attribute__((ext_vector_type(2)));

template <bool NT>
__device__ __forceinline__ float2 ldg(const float2* p) {
    if constexpr (NT) {
        const f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(p));
        return make_float2(v.x, v.y);
    } else {
        return *p;
    }
}

template <bool NT>
__device__ __forceinline__ float4 ldg(const float4* p) {
    if constexpr (NT) {
        const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
        return make_float4(v.x, v.y, v.z, v.w);
    } else {
        return *p;
    }
}

template <bool NT>
__device__ __forceinline__ void load_link(const double2* __restrict__ u, int nlinks, int k,
                                          Link<double>& L) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const double2 v = ldg<NT>(u + (size_t)(3 * i + j) * nlinks + k);
            L.re[i][j] = v.x;
            L.im[i][j] = v.y;
        }
}

// Row 3 of an SU(3) matrix from rows 1-2: conj(row1 x row2) (valid for det U = 1).
template <typename RT>
__device__ __forceinline__ void rebuild_row3(Link<RT>& L) {
    // No contraction into FMA here: which products fuse would otherwise depend
    // on the surrounding code, and every launch variant must give the same bits.
#pragma clang fp contract(off)
    // (row1 x row2)_j = row1_{j+1} row2_{j+2} - row1_{j+2} row2_{j+1}
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        const RT pr = L.re[0][j1] * L.re[1][j2] - L.im[0][j1] * L.im[1][j2]
                    - (L.re[0][j2] * L.re[1][j1] - L.im[0][j2] * L.im[1][j1]);
        const RT pi = L.re[0][j1] * L.im[1][j2] + L.im[0][j1] * L.re[1][j2]
                    - (L.re[0][j2] * L.im[1][j1] + L.im[0][j2] * L.re[1][j1]);
        L.re[2][j] = pr;
        L.im[2][j] = -pi;
    }
}

// 12-real link: rows 1-2 stored, row 3 = conj(row1 x row2) (valid for det U = 1).
template <bool NT>
__device__ __forceinline__ void load_link(const float4* __restrict__ u, int nlinks, int k,
                                          Link<float>& L) {
    const float4 a = ldg<NT>(u + k);
    const float4 b = ldg<NT>(u + (size_t)nlinks + k);
    const float4 c = ldg<NT>(u + (size_t)2 * nlinks + k);
    L.re[0][0] = a.x; L.im[0][0] = a.y; L.re[0][1] = a.z; L.im[0][1] = a.w;
    L.re[0][2] = b.x; L.im[0][2] = b.y; L.re[1][0] = b.z; L.im[1][0] = b.w;
    L.re[1][1] = c.x; L.im[1][1] = c.y; L.re[1][2] = c.z; L.im[1][2] = c.w;
    rebuild_row3(L);
}

// FP64 link from hi + lo planes: rows 1-2 = hi + lo in FP64, row 3 rebuilt in
// FP64 as conj(row1 x row2).
template <bool NT>
__device__ __forceinline__ void load_link(const HiLoLink* __restrict__ uh, int nlinks, int k,
                                          Link<double>& L) {
    const float4* u = reinterpret_cast<const float4*>(uh);
    float4 h[3], l[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        h[i] = ldg<NT>(u + (size_t)i * nlinks + k);
        l[i] = ldg<NT>(u + (size_t)(3 + i) * nlinks + k);
    }
    const double w[12] = {(double)h[0].x + (double)l[0].x, (double)h[0].y + (double)l[0].y,
                          (double)h[0].z + (double)l[0].z, (double)h[0].w + (double)l[0].w,
                          (double)h[1].x + (double)l[1].x, (double)h[1].y + (double)l[1].y,
                          (double)h[1].z + (double)l[1].z, (double)h[1].w + (double)l[1].w,
                          (double)h[2].x + (double)l[2].x, (double)h[2].y + (double)l[2].y,
                          (double)h[2].z + (double)l[2].z, (double)h[2].w + (double)l[2].w};
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        L.re[e / 3][e % 3] = w[2 * e];
        L.im[e / 3][e % 3] = w[2 * e + 1];
    }
    rebuild_row3(L);
}

// FP32 link from 18 stored floats (no reconstruction: any complex 3x3 matrix).
template <bool NT>
__device__ __forceinline__ void load_link(const Fp32x18Link* __restrict__ uf, int nlinks, int k,
                                          Link<float>& L) {
    const float2* u = reinterpret_cast<const float2*>(uf);
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const float2 v = ldg<NT>(u + (size_t)e * nlinks + k);
        L.re[e / 3][e % 3] = v.x;
        L.im[e / 3][e % 3] = v.y;
    }
}

// FP64 link from 12 stored doubles (rows 1-2), row 3 rebuilt in FP64.
template <bool NT>
__device__ __forceinline__ void load_link(const Fp64x12Link* __restrict__ uc, int nlinks, int k,
                                          Link<double>& L) {
    const double2* u = reinterpret_cast<const double2*>(uc);
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const double2 v = ldg<NT>(u + (size_t)e * nlinks + k);
        L.re[e / 3][e % 3] = v.x;
        L.im[e / 3][e % 3] = v.y;
    }
    rebuild_row3(L);
}

template <typename VT> struct RealOf;
template <> struct RealOf<double2> { using T = double; };
template <> struct RealOf<float2> { using T = float; };

// ------------------------------------------------------------------ hopping kernel
template <typename VT, typename LT, int NR, int MODE, bool NT, int BATCH>
__global__ __launch_bounds__(kBlock) void k_dslash(const LT* __restrict__ links, int nlinks,
                                                    DslashArgs<VT> a) {
    using RT = typename RealOf<VT>::T;
    if (a.all_done && *a.all_done) return;
    const int nblk = gridDim.x;
    const int blk = xcd_remap(blockIdx.x, nblk);
    const int Vh = a.g.Vh;
    const int p = blk * kBlock + threadIdx.x;

    // Every lane loads all NR vectors of a hop with no branch in between, so
    // the compiler can keep every load of a hop in flight at once; slots of
    // finished or absent right-hand sides read rhs 0 (valid, cached) and only
    // their stores are suppressed.
    bool act[NR];
    const VT* inp[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        act[r] = (r < a.nrhs) && !(a.skip && a.skip[r * a.skip_stride]);
        inp[r] = (r < a.nrhs) ? a.in[r] : a.in[0];
    }

    double dot[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) dot[r] = 0.0;

    if (p < Vh) {
        int eo, x, y, z, t;
        process_site(a.g, p, a.out_par, a.variant & 3, eo, x, y, z, t);
        const Hops h = make_hops(a.g, eo, x, y, z, t);
        RT ar[NR][3], ai[NR][3];
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) ar[r][c] = ai[r][c] = RT(0);

        // Hops in the order +x, -x, +y, -y, +z, -z, +t, -t: both uses of an
        // input site along one direction fall in the same load batch, and the
        // sums run in this order in every launch variant (same bits).
        int nbh = h.nb[0];
#pragma unroll
        for (int hop = 0; hop < 8; ++hop) {
            const int mu = hop >> 1;
            const bool fwd = (hop & 1) == 0;
            const int slot = fwd ? mu : 4 + mu;   // index into Hops (0..3 forward, 4..7 backward)
            const int nb = nbh;
            // forward: U_mu(n) at this site; backward: U_mu(n-mu) at the neighbour
            const int k = fwd ? (2 * mu + a.out_par) * Vh + eo : (2 * mu + 1 - a.out_par) * Vh + nb;
            Link<RT> U;
            load_link<NT>(links, nlinks, k, U);
            VT v[NR][3];
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                v[r][0] = inp[r][nb];
                v[r][1] = inp[r][Vh + nb];
                v[r][2] = inp[r][2 * Vh + nb];
            }
            const RT s = (RT)h.coef[slot];
#pragma unroll
            for (int r = 0; r < NR; ++r) {
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    RT tr, ti;
                    if (fwd) {  // (U v)_i = sum_j U_ij v_j
                        tr = U.re[i][0] * v[r][0].x - U.im[i][0] * v[r][0].y + U.re[i][1] * v[r][1].x -
                             U.im[i][1] * v[r][1].y + U.re[i][2] * v[r][2].x - U.im[i][2] * v[r][2].y;
                        ti = U.re[i][0] * v[r][0].y + U.im[i][0] * v[r][0].x + U.re[i][1] * v[r][1].y +
                             U.im[i][1] * v[r][1].x + U.re[i][2] * v[r][2].y + U.im[i][2] * v[r][2].x;
                    } else {    // (U^dagger v)_i = sum_j conj(U_ji) v_j
                        tr = U.re[0][i] * v[r][0].x + U.im[0][i] * v[r][0].y + U.re[1][i] * v[r][1].x +
                             U.im[1][i] * v[r][1].y + U.re[2][i] * v[r][2].x + U.im[2][i] * v[r][2].y;
                        ti = U.re[0][i] * v[r][0].y - U.im[0][i] * v[r][0].x + U.re[1][i] * v[r][1].y -
                             U.im[1][i] * v[r][1].x + U.re[2][i] * v[r][2].y - U.im[2][i] * v[r][2].x;
                    }
                    ar[r][i] += s * tr;
                    ai[r][i] += s * ti;
                }
            }
            if (hop + 1 < 8) {
                // Empty volatile asms (no instruction) pin the sums after every
                // BATCH hops and make the next hop's index depend on them: each
                // wave then issues the loads of BATCH hops together and finishes
                // their arithmetic before the next batch, instead of the
                // scheduler hoisting all eight hops' loads and keeping them live
                // (one wave per SIMD).  Latency is hidden by the other resident
                // waves.  BATCH = 8 leaves the schedule to the compiler.
                if ((hop + 1) % BATCH == 0) {
#pragma unroll
                    for (int r = 0; r < NR; ++r)
#pragma unroll
                        for (int i = 0; i < 3; ++i) asm volatile("" : "+v"(ar[r][i]), "+v"(ai[r][i]));
                }
                const int next = hop + 1;
                nbh = h.nb[(next & 1) ? 4 + (next >> 1) : (next >> 1)];
                asm volatile("" : "+v"(nbh));
            }
        }

#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (!act[r]) continue;
            if (MODE == kModeD) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    VT o;
                    o.x = ar[r][c];
                    o.y = ai[r][c];
                    a.out[r][c * Vh + eo] = o;
                }
            } else if (MODE == kModeA) {
                const RT cr = (RT)a.c[r];
                double d = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const VT p = a.self[r][c * Vh + eo];
                    VT o;
                    o.x = cr * p.x - ar[r][c];
                    o.y = cr * p.y - ai[r][c];
                    a.out[r][c * Vh + eo] = o;
                    d += (double)p.x * (double)o.x + (double)p.y * (double)o.y;
                }
                dot[r] = d;
            } else {  // kModeResid (FP64 operator)
                const double cr = a.c[r];
                double d = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const VT xv = a.self[r][c * Vh + eo];
                    const double2 bv = a.rhs[r][c * Vh + eo];
                    double2 o;
                    o.x = bv.x - cr * (double)xv.x + (double)ar[r][c];
                    o.y = bv.y - cr * (double)xv.y + (double)ai[r][c];
                    if (a.out[r]) {
                        VT w;
                        w.x = o.x;
                        w.y = o.y;
                        a.out[r][c * Vh + eo] = w;
                    }
                    if (a.out32[r]) a.out32[r][c * Vh + eo] = make_float2((float)o.x, (float)o.y);
                    d += o.x * o.x + o.y * o.y;
                }
                dot[r] = d;
            }
        }
    }

    if (MODE != kModeD) {
        // deterministic block reduction -> one partial per rhs and block
        __shared__ double sm[NR][kBlock / 64];
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            double v = dot[r];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) sm[r][wid] = v;
        }
        __syncthreads();
        if (threadIdx.x < NR && threadIdx.x < a.nrhs) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < kBlock / 64; ++w) t += sm[threadIdx.x][w];
            a.partial[(size_t)threadIdx.x * nblk + blk] = t;
        }
    }
}

template <typename VT, typename LT, int MODE, bool NT, int BATCH>
inline hipError_t dispatch_nt(const LT* links, int nlinks, const DslashArgs<VT>& a, size_t lds,
                              hipStream_t s) {
    const dim3 grid(dslash_grid(a.g.Vh)), block(kBlock);
    if (a.nrhs <= 1)
        hipLaunchKernelGGL((k_dslash<VT, LT, 1, MODE, NT, BATCH>), grid, block, lds, s, links, nlinks, a);
    else if (a.nrhs <= 2)
        hipLaunchKernelGGL((k_dslash<VT, LT, 2, MODE, NT, BATCH>), grid, block, lds, s, links, nlinks, a);
    else if (a.nrhs <= 4)
        hipLaunchKernelGGL((k_dslash<VT, LT, 4, MODE, NT, BATCH>), grid, block, lds, s, links, nlinks, a);
    else
        hipLaunchKernelGGL((k_dslash<VT, LT, 8, MODE, NT, BATCH>), grid, block, lds, s, links, nlinks, a);
    return hipGetLastError();
}

template <typename VT, typename LT, int MODE, bool NT>
inline hipError_t dispatch_batch(const LT* links, int nlinks, const DslashArgs<VT>& a, int batch,
                                 size_t lds, hipStream_t s) {
    switch (batch) {
        case 0: return dispatch_nt<VT, LT, MODE, NT, 1>(links, nlinks, a, lds, s);
        case 1: return dispatch_nt<VT, LT, MODE, NT, 2>(links, nlinks, a, lds, s);
        case 2: return dispatch_nt<VT, LT, MODE, NT, 4>(links, nlinks, a, lds, s);
        default: return dispatch_nt<VT, LT, MODE, NT, 8>(links, nlinks, a, lds, s);
    }
}

template <typename VT, typename LT, int MODE>
inline hipError_t dispatch(const LT* links, int nlinks, const DslashArgs<VT>& a0, hipStream_t s) {
    DslashArgs<VT> a = a0;
    int v = a.variant & (kHopVariants - 1);
    if ((v & 3) == 2 && a.g.Lz % 4 != 0) v = (v & ~3) | 1;   // z-tiles of 4 need Lz % 4 == 0
    a.variant = v;
    const bool nt = (v >> 2) & 1;
    const int batch = (v >> 3) & 3;
    const size_t lds = (size_t)kOccLds[(v >> 5) & 3];
    if (nt) return dispatch_batch<VT, LT, MODE, true>(links, nlinks, a, batch, lds, s);
    return dispatch_batch<VT, LT, MODE, false>(links, nlinks, a, batch, lds, s);
}

}  // namespace rhmc
