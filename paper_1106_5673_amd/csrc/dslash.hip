// Link packing (storage layouts of Sec. 4.2), the neighbour-table debug
// kernel and the FP32-12 hopping-term launches (Eq. stag); the kernel itself
// is in dslash_kernel.h.
#include "dslash_kernel.h"

namespace rhmc {

// ------------------------------------------------------------------ pack
__global__ __launch_bounds__(kBlock) void k_pack_links(const double2* __restrict__ canon, Geom g,
                                                        double2* __restrict__ u64,
                                                        float4* __restrict__ u32, int hilo,
                                                        double2* __restrict__ u64c,
                                                        float2* __restrict__ u32f, int nlinks) {
    const int id = blockIdx.x * blockDim.x + threadIdx.x;  // lex * 4 + mu
    const int V = 2 * g.Vh;
    if (id >= 4 * V) return;
    const int lex = id >> 2, mu = id & 3;
    int r = lex / g.Lx;
    const int x = lex - r * g.Lx;
    const int y = r % g.Ly;
    r /= g.Ly;
    const int z = r % g.Lz;
    const int t = r / g.Lz;
    const int par = (x + y + z + t) & 1;
    const int k = (2 * mu + par) * g.Vh + (lex >> 1);
    const double2* src = canon + (size_t)id * 9;
    double2 e[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) e[i] = src[i];
    if (u64) {
#pragma unroll
        for (int i = 0; i < 9; ++i) u64[(size_t)i * nlinks + k] = e[i];
    }
    if (u64c) {
#pragma unroll
        for (int i = 0; i < 6; ++i) u64c[(size_t)i * nlinks + k] = e[i];
    }
    if (u32f) {
        // all 18 reals rounded to nearest FP32
#pragma unroll
        for (int i = 0; i < 9; ++i)
            u32f[(size_t)i * nlinks + k] = make_float2((float)e[i].x, (float)e[i].y);
    }
    if (u32) {
        // rows 1-2 rounded to nearest FP32; row 3 is rebuilt in the kernel
        u32[(size_t)0 * nlinks + k] = make_float4((float)e[0].x, (float)e[0].y, (float)e[1].x, (float)e[1].y);
        u32[(size_t)1 * nlinks + k] = make_float4((float)e[2].x, (float)e[2].y, (float)e[3].x, (float)e[3].y);
        u32[(size_t)2 * nlinks + k] = make_float4((float)e[4].x, (float)e[4].y, (float)e[5].x, (float)e[5].y);
        if (hilo) {
            // lo = the FP32 rounding of what hi leaves out: hi + lo carries
            // about 48 significant bits of each FP64 entry (Sec. 4.2)
            float lo[12];
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                lo[2 * i] = (float)(e[i].x - (double)(float)e[i].x);
                lo[2 * i + 1] = (float)(e[i].y - (double)(float)e[i].y);
            }
            u32[(size_t)3 * nlinks + k] = make_float4(lo[0], lo[1], lo[2], lo[3]);
            u32[(size_t)4 * nlinks + k] = make_float4(lo[4], lo[5], lo[6], lo[7]);
            u32[(size_t)5 * nlinks + k] = make_float4(lo[8], lo[9], lo[10], lo[11]);
        }
    }
}

hipError_t launch_pack_links(const rhmc_gauge* g, const double2* canon, hipStream_t s) {
    const int V = (int)g->lat.V;
    const int nlinks = 4 * V;
    const int grid = (4 * V + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_pack_links, dim3(grid), dim3(kBlock), 0, s, canon, g->lat.geom, g->u64,
                       g->u32, g->hilo, g->u64c, g->u32f, nlinks);
    return hipGetLastError();
}

// ------------------------------------------------------------------ neighbours
__global__ __launch_bounds__(kBlock) void k_neighbors(Geom g, int par, int* nb, int* sign) {
    const int eo = blockIdx.x * blockDim.x + threadIdx.x;
    if (eo >= g.Vh) return;
    int x, y, z, t;
    site_coords(g, eo, par, x, y, z, t);
    const Hops h = make_hops(g, eo, x, y, z, t);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        nb[(size_t)eo * 8 + k] = h.nb[k];
        if (sign) sign[(size_t)eo * 8 + k] = (int)(2.0f * h.coef[k]) * (k < 4 ? 1 : -1);
    }
}

hipError_t launch_neighbors(const Geom& g, int par, int* nb, int* sign, hipStream_t s) {
    hipLaunchKernelGGL(k_neighbors, dim3((g.Vh + kBlock - 1) / kBlock), dim3(kBlock), 0, s, g, par,
                       nb, sign);
    return hipGetLastError();
}


hipError_t launch_dslash32(const float4* u32, int nlinks, const DslashArgs<float2>& a, int mode,
                           hipStream_t s) {
    switch (mode) {
        case kModeD: return dispatch<float2, float4, kModeD>(u32, nlinks, a, s);
        default: return dispatch<float2, float4, kModeA>(u32, nlinks, a, s);
    }
}

}  // namespace rhmc
