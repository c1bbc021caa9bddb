// Staggered hopping term (Eq. stag, Sec. 2) between the two parities: link
// loaders for every storage of Sec. 4.2 and the hopping kernel, shared by the
// translation units that instantiate it for one link storage each.
//
// One lane owns one output site and every right-hand side of the launch, so
// each link is read once per application however many vectors are batched.
// Links are structure-of-arrays over the link index k = (2*mu + parity)*Vh + eo,
// so the 64 lanes of a wave read 64 consecutive links per load; neighbour
// vectors are colour-major [3][Vh] arrays (FP32 sets of several right-hand
// sides: one [3][Vh] array of float4 per pair of them), read by consecutive
// sites (or, for the +-x and +-y hops of a staged block, from LDS).
#pragma once

#include <type_traits>

#include "common.h"

namespace rhmc {

// ------------------------------------------------------------------ links
template <typename RT>
struct Link {
    RT re[3][3], im[3][3];
};

typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));

// Loads from global memory (address space 1); NT: non-temporal (streamed,
// read once by this kernel).
template <typename T>
using gp = const __attribute__((address_space(1))) T*;

template <bool NT>
__device__ __forceinline__ double2 ldg(gp<double2> p) {
    const __attribute__((address_space(1))) d2v* q =
        reinterpret_cast<const __attribute__((address_space(1))) d2v*>(p);
    d2v v;
    if constexpr (NT)
        v = __builtin_nontemporal_load(q);
    else
        v = *q;
    return make_double2(v.x, v.y);
}

template <bool NT>
__device__ __forceinline__ float2 ldg(gp<float2> p) {
    const __attribute__((address_space(1))) f2v* q =
        reinterpret_cast<const __attribute__((address_space(1))) f2v*>(p);
    f2v v;
    if constexpr (NT)
        v = __builtin_nontemporal_load(q);
    else
        v = *q;
    return make_float2(v.x, v.y);
}

template <bool NT>
__device__ __forceinline__ float4 ldg(gp<float4> p) {
    const __attribute__((address_space(1))) f4v* q =
        reinterpret_cast<const __attribute__((address_space(1))) f4v*>(p);
    f4v v;
    if constexpr (NT)
        v = __builtin_nontemporal_load(q);
    else
        v = *q;
    return make_float4(v.x, v.y, v.z, v.w);
}

// Stores of a kernel's output that nothing reads again while the kernel
// runs: non-temporal, so they do not push inputs that neighbouring sites still
// need out of the L2.
__device__ __forceinline__ void stnt(float2* p, float2 v) {
    __builtin_nontemporal_store(f2v{v.x, v.y}, reinterpret_cast<f2v*>(p));
}
__device__ __forceinline__ void stnt(float4* p, float4 v) {
    __builtin_nontemporal_store(f4v{v.x, v.y, v.z, v.w}, reinterpret_cast<f4v*>(p));
}
__device__ __forceinline__ void stnt(double2* p, double2 v) {
    __builtin_nontemporal_store(d2v{v.x, v.y}, reinterpret_cast<d2v*>(p));
}

// The planes of a structure-of-arrays field (link entries, colour planes of
// a vector): every plane's base address is uniform and held in scalar
// registers (readfirstlane keeps the compiler from folding it into per-lane
// address arithmetic), and a lane adds a 32-bit byte offset (the lattice
// volume cap keeps it below 2^32): one offset per lane serves every plane.
typedef const __attribute__((address_space(1))) char* gbl_ptr;   // global memory

__device__ __forceinline__ gbl_ptr uniform_ptr(const void* q) {
    const uint64_t v = reinterpret_cast<uint64_t>(q);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<gbl_ptr>(((uint64_t)hi << 32) | lo);
}

template <typename T, int E>
struct Planes {
    gbl_ptr p[E];
    __device__ __forceinline__ const __attribute__((address_space(1))) T* at(int e, uint32_t byte_off) const {
        return reinterpret_cast<const __attribute__((address_space(1))) T*>(p[e] + byte_off);
    }
};

template <typename T, int E>
__device__ __forceinline__ Planes<T, E> make_planes(const T* base, size_t stride) {
    Planes<T, E> P;
#pragma unroll
    for (int e = 0; e < E; ++e) P.p[e] = uniform_ptr(base + (size_t)e * stride);
    return P;
}

__device__ __forceinline__ uint32_t byte_off(int k, uint32_t size) { return (uint32_t)k * size; }

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

// Link storages as planes of entries: entry type and number of planes.
template <typename LT> struct LinkFmt;
template <> struct LinkFmt<double2> { using T = double2; static constexpr int E = 9; };       // FP64-18
template <> struct LinkFmt<Fp64x12Link> { using T = double2; static constexpr int E = 6; };   // FP64-12
template <> struct LinkFmt<float4> { using T = float4; static constexpr int E = 3; };         // FP32-12
template <> struct LinkFmt<HiLoLink> { using T = float4; static constexpr int E = 6; };       // hi, lo
template <> struct LinkFmt<Fp32x18Link> { using T = float2; static constexpr int E = 9; };    // FP32-18

template <typename LT>
using LinkPlanes = Planes<typename LinkFmt<LT>::T, LinkFmt<LT>::E>;

template <typename LT>
__device__ __forceinline__ LinkPlanes<LT> link_planes(const LT* u, int nlinks) {
    using T = typename LinkFmt<LT>::T;
    return make_planes<T, LinkFmt<LT>::E>(reinterpret_cast<const T*>(u), (size_t)nlinks);
}

// FP64-18: all 18 reals stored.
template <bool NT>
__device__ __forceinline__ void load_link(const Planes<double2, 9>& P, int k, Link<double>& L) {
    const uint32_t o = byte_off(k, 16);
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const double2 v = ldg<NT>(P.at(e, o));
        L.re[e / 3][e % 3] = v.x;
        L.im[e / 3][e % 3] = v.y;
    }
}

// FP32-12: rows 1-2 stored as three float4, row 3 = conj(row1 x row2) (valid
// for det U = 1).
template <bool NT>
__device__ __forceinline__ void load_link(const Planes<float4, 3>& P, int k, Link<float>& L) {
    const uint32_t o = byte_off(k, 16);
    const float4 a = ldg<NT>(P.at(0, o));
    const float4 b = ldg<NT>(P.at(1, o));
    const float4 c = ldg<NT>(P.at(2, o));
    L.re[0][0] = a.x; L.im[0][0] = a.y; L.re[0][1] = a.z; L.im[0][1] = a.w;
    L.re[0][2] = b.x; L.im[0][2] = b.y; L.re[1][0] = b.z; L.im[1][0] = b.w;
    L.re[1][1] = c.x; L.im[1][1] = c.y; L.re[1][2] = c.z; L.im[1][2] = c.w;
    rebuild_row3(L);
}

// FP64 link from hi + lo planes: rows 1-2 = hi + lo in FP64, row 3 rebuilt in
// FP64 as conj(row1 x row2).
template <bool NT>
__device__ __forceinline__ void load_link(const Planes<float4, 6>& P, int k, Link<double>& L) {
    const uint32_t o = byte_off(k, 16);
    float4 h[3], l[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        h[i] = ldg<NT>(P.at(i, o));
        l[i] = ldg<NT>(P.at(3 + i, o));
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

// FP32-18: all 18 reals stored (no reconstruction: any complex 3x3 matrix).
template <bool NT>
__device__ __forceinline__ void load_link(const Planes<float2, 9>& P, int k, Link<float>& L) {
    const uint32_t o = byte_off(k, 8);
#pragma unroll
    for (int e = 0; e < 9; ++e) {
        const float2 v = ldg<NT>(P.at(e, o));
        L.re[e / 3][e % 3] = v.x;
        L.im[e / 3][e % 3] = v.y;
    }
}

// FP64-12: rows 1-2 stored in FP64, row 3 rebuilt in FP64.
template <bool NT>
__device__ __forceinline__ void load_link(const Planes<double2, 6>& P, int k, Link<double>& L) {
    const uint32_t o = byte_off(k, 16);
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const double2 v = ldg<NT>(P.at(e, o));
        L.re[e / 3][e % 3] = v.x;
        L.im[e / 3][e % 3] = v.y;
    }
    rebuild_row3(L);
}

// Link k of a storage given by its base address (kernels outside the
// hopping term).
template <bool NT, typename LT, typename RT>
__device__ __forceinline__ void load_link(const LT* __restrict__ u, int nlinks, int k, Link<RT>& L) {
    load_link<NT>(link_planes(u, nlinks), k, L);
}

template <typename VT> struct RealOf;
template <> struct RealOf<double2> { using T = double; };
template <> struct RealOf<float2> { using T = float; };

__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }

// One hop for every right-hand side: S += s * (U v) (forward) or
// S += s * (U^dagger v) (backward), with s = +-1/2.  The input is scaled by s
// first (exact: a power of two), then each real component of the product is
// accumulated into S by a fixed chain of six fused multiply-adds (the first
// hop starts the chain with a product): every launch shape forms the same
// sequence of roundings, so all give the same bits.
template <bool FWD, bool FIRST, typename RT, typename VT, int NR>
__device__ __forceinline__ void hop_apply(const Link<RT>& U, const VT (&v)[NR][3], RT s,
                                          RT (&sr)[NR][3], RT (&si)[NR][3]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        RT wr[3], wi[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            wr[j] = s * v[r][j].x;
            wi[j] = s * v[r][j].y;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            // forward (U v)_i = sum_j U_ij v_j; backward (U^dagger v)_i = sum_j conj(U_ji) v_j
            RT xr = sr[r][i], xi = si[r][i];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const RT ur = FWD ? U.re[i][j] : U.re[j][i];
                const RT ui = FWD ? U.im[i][j] : -U.im[j][i];
                if (FIRST && j == 0) {
                    xr = ur * wr[j];
                    xi = ur * wi[j];
                } else {
                    xr = fmar(ur, wr[j], xr);
                    xi = fmar(ur, wi[j], xi);
                }
                xr = fmar(-ui, wi[j], xr);
                xi = fmar(ui, wr[j], xi);
            }
            sr[r][i] = xr;
            si[r][i] = xi;
        }
    }
}

// One loaded element into the per-rhs colour components: a vector entry of
// one right-hand side, or (float4) one colour of the pair q of them.
template <typename VT, int NR>
__device__ __forceinline__ void unpack(const VT& w, VT (&v)[NR][3], int q, int c) {
    v[q][c] = w;
}
template <int NR>
__device__ __forceinline__ void unpack(const float4& w, float2 (&v)[NR][3], int q, int c) {
    v[2 * q][c] = make_float2(w.x, w.y);
    v[2 * q + 1][c] = make_float2(w.z, w.w);
}

// ------------------------------------------------------------------ hopping kernel
// One lane owns one output site and every right-hand side of the launch, so
// each link is read once per application however many vectors are batched.
// The eight hops run in the order +x, -x, +y, -y, +z, -z, +t, -t and every
// launch shape forms the same sequence of roundings (hop_apply), so all give
// the same bits.  BATCH is the number of hops whose loads are issued
// together.
//
// STG (staged rows): a block is R whole rows (R * Lx/2 sites) of one xy-plane.
// It first copies the input of its rows and of the row above and below
// (periodic in y) into LDS with coalesced loads, and the +-x and +-y hops
// read their neighbours from LDS.  Every neighbour vector otherwise passes
// through the per-CU vector-memory pipeline (address unit and L1) once per
// hop, eight times per site; staging takes half of those accesses off it.
//
// FP32 with NR >= 2 (PR): the vectors come in pairs of right-hand sides
// (f32_offset), so one 16-byte load brings one colour of two of them and the
// kernel issues half as many vector loads (the pipeline above is limited by
// load instructions more than by bytes).  Pair q is in[2q] / out[2q] / self[2q];
// a pair with one live member is stored whole (the other half, a finished or
// absent right-hand side, receives values nobody reads).
template <typename VT, typename LT, int NR, int MODE, bool NT, int BATCH, bool STG>
__global__ __launch_bounds__(STG ? 512 : kBlock) void k_dslash(const LT* __restrict__ links,
                                                               int nlinks, DslashArgs<VT> a) {
#pragma clang fp contract(off)
    using RT = typename RealOf<VT>::T;
    constexpr bool PR = std::is_same<VT, float2>::value && NR >= 2;
    constexpr int NP = PR ? NR / 2 : NR;                             // vector planes sets
    using LVT = typename std::conditional<PR, float4, VT>::type;    // one load
    static_assert(!PR || MODE != kModeResid, "the residual mode is FP64");
    if (a.all_done && *a.all_done) return;
    const int nblk = gridDim.x;
    const int blk = xcd_remap(blockIdx.x, nblk);
    const int Vh = a.g.Vh;
    const int bsites = (int)blockDim.x;   // sites per block
    const int p_raw = blk * bsites + (int)threadIdx.x;
    if (p_raw >= Vh && MODE == kModeD) return;   // (staged blocks are never partial)
    const bool in_range = p_raw < Vh;
    const int p = in_range ? p_raw : Vh - 1;

    // Every lane loads all NR vectors of a hop with no branch in between, so
    // the compiler can keep every load of a hop in flight at once; slots of
    // finished or absent right-hand sides read rhs 0 (valid, cached) and only
    // their stores are suppressed.
    bool act[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) act[r] = in_range && (r < a.nrhs) && !(a.skip && a.skip[r * a.skip_stride]);
    Planes<LVT, 3> vin[NP];   // colour planes of every input (pair)
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        const int r = PR ? 2 * q : q;
        vin[q] = make_planes<LVT, 3>(reinterpret_cast<const LVT*>((r < a.nrhs) ? a.in[r] : a.in[0]),
                                     (size_t)Vh);
    }
    const LinkPlanes<LT> lp = link_planes(links, nlinks);

    int eo, x, y, z, t;
    process_site(a.g, p, a.out_par, a.zt, eo, x, y, z, t);
    const Hops h = make_hops(a.g, eo, x, y, z, t);

    // staged rows: LDS [NR][3][R + 2][hx], row 0 = y0 - 1, row R + 1 = y0 + R
    extern __shared__ unsigned char lds_stage[];
    LVT* stage = reinterpret_cast<LVT*>(lds_stage);
    int srow = 0, shx = 0, sR2 = 0;   // this site's staged row, hx, R + 2
    if (STG) {
        const int hx = a.g.hx, Ly = a.g.Ly;
        const int R = bsites / hx;
        int eo0, x0, y0, z0, t0;
        process_site(a.g, blk * bsites, a.out_par, a.zt, eo0, x0, y0, z0, t0);
        const int base = hx * Ly * (z0 + a.g.Lz * t0);   // first site of the plane
        const int rows = (R + 2) * hx;
        for (int idx = (int)threadIdx.x; idx < rows; idx += bsites) {
            int rr, xs;
            fdivmod(idx, a.g.dhx, rr, xs);
            int yy = y0 - 1 + rr;
            yy = yy < 0 ? yy + Ly : (yy >= Ly ? yy - Ly : yy);
            const int src = base + hx * yy + xs;
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                const int r = PR ? 2 * q : q;
                if (r >= a.nrhs) break;
                const LVT* in = reinterpret_cast<const LVT*>(a.in[r]);
#pragma unroll
                for (int c = 0; c < 3; ++c) stage[(q * 3 + c) * rows + idx] = in[c * Vh + src];
            }
        }
        srow = y - y0 + 1;
        shx = hx;
        sR2 = R + 2;
        __syncthreads();
    }

    RT ar[NR][3], ai[NR][3];
    int nbh = h.nb[0];
#pragma unroll
    for (int hop = 0; hop < 8; ++hop) {
        const int mu = hop >> 1;
        const bool fwd = (hop & 1) == 0;
        const int slot = fwd ? mu : 4 + mu;   // index into Hops (0..3 forward, 4..7 backward)
        const int nb = nbh;
        // forward: U_mu(n) at this site; backward: U_mu(n-mu) at the neighbour
        const int kl = fwd ? (2 * mu + a.out_par) * Vh + eo : (2 * mu + 1 - a.out_par) * Vh + nb;
        Link<RT> U;
        load_link<NT>(lp, kl, U);
        VT v[NR][3];
        if (STG && mu < 2) {
            // x neighbours: same row, half-index of x +- 1 (periodic); y
            // neighbours: the row above or below, same half-index
            int col, row = srow;
            if (mu == 0)
                col = fwd ? ((x + 1 == a.g.Lx) ? 0 : (x + 1) >> 1) : ((x == 0) ? shx - 1 : (x - 1) >> 1);
            else {
                col = x >> 1;
                row += fwd ? 1 : -1;
            }
            const int li = row * shx + col;
            const int rows = sR2 * shx;
#pragma unroll
            for (int q = 0; q < NP; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c) unpack(stage[(q * 3 + c) * rows + li], v, q, c);
        } else {
            const uint32_t o = byte_off(nb, (uint32_t)sizeof(LVT));
#pragma unroll
            for (int q = 0; q < NP; ++q)
#pragma unroll
                for (int c = 0; c < 3; ++c) unpack(ldg<false>(vin[q].at(c, o)), v, q, c);
        }
        const RT s = (RT)h.coef[slot];
        if (hop == 0)
            hop_apply<true, true>(U, v, s, ar, ai);
        else if (fwd)
            hop_apply<true, false>(U, v, s, ar, ai);
        else
            hop_apply<false, false>(U, v, s, ar, ai);
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

    double dot[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) dot[r] = 0.0;
    if constexpr (PR) {
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int r0 = 2 * q, r1 = 2 * q + 1;
            if (!act[r0] && !act[r1]) continue;
            float4* out = reinterpret_cast<float4*>(a.out[r0]);
            if (MODE == kModeD) {
#pragma unroll
                for (int c = 0; c < 3; ++c)
                    stnt(out + c * Vh + eo, make_float4(ar[r0][c], ai[r0][c], ar[r1][c], ai[r1][c]));
            } else {
                // the site's own p is read once here: non-temporal, so that it
                // does not take L2 room from the neighbour reads
                const float4* self = reinterpret_cast<const float4*>(a.self[r0]);
                const RT c0 = (RT)a.c[r0], c1 = (RT)a.c[r1];
                double d0 = 0.0, d1 = 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float4 pv = ldg<true>((gp<float4>)(self + c * Vh + eo));
                    float4 o;
                    o.x = c0 * pv.x - ar[r0][c];
                    o.y = c0 * pv.y - ai[r0][c];
                    o.z = c1 * pv.z - ar[r1][c];
                    o.w = c1 * pv.w - ai[r1][c];
                    stnt(out + c * Vh + eo, o);
                    d0 = d0 + (double)pv.x * (double)o.x;
                    d0 = d0 + (double)pv.y * (double)o.y;
                    d1 = d1 + (double)pv.z * (double)o.z;
                    d1 = d1 + (double)pv.w * (double)o.w;
                }
                dot[r0] = act[r0] ? d0 : 0.0;
                dot[r1] = act[r1] ? d1 : 0.0;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (PR || !act[r]) continue;
        if (MODE == kModeD) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                VT o;
                o.x = ar[r][c];
                o.y = ai[r][c];
                stnt(a.out[r] + c * Vh + eo, o);
            }
        } else if (MODE == kModeA) {
            const RT cr = (RT)a.c[r];
            double d = 0.0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const VT pv = ldg<true>((gp<VT>)(a.self[r] + c * Vh + eo));
                VT o;
                o.x = cr * pv.x - ar[r][c];
                o.y = cr * pv.y - ai[r][c];
                stnt(a.out[r] + c * Vh + eo, o);
                d = d + (double)pv.x * (double)o.x;
                d = d + (double)pv.y * (double)o.y;
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
                o.x = (bv.x - cr * (double)xv.x) + (double)ar[r][c];
                o.y = (bv.y - cr * (double)xv.y) + (double)ai[r][c];
                if (a.out[r]) {
                    VT w;
                    w.x = o.x;
                    w.y = o.y;
                    a.out[r][c * Vh + eo] = w;
                }
                if (a.out32[r])
                    a.out32[r][(size_t)(c * Vh + eo) << a.out32_paired] = make_float2((float)o.x, (float)o.y);
                d = d + o.x * o.x;
                d = d + o.y * o.y;
            }
            dot[r] = d;
        }
    }

    if (MODE != kModeD) {
        // deterministic block reduction -> one partial per rhs and block
        constexpr int kMaxWaves = (STG ? 512 : kBlock) / 64;
        __shared__ double sm[NR][kMaxWaves];
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
        const int nw = bsites >> 6;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            double v = dot[r];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) sm[r][wid] = v;
        }
        __syncthreads();
        if ((int)threadIdx.x < NR && (int)threadIdx.x < a.nrhs) {
            double t2 = 0.0;
            for (int w = 0; w < nw; ++w) t2 += sm[threadIdx.x][w];
            a.partial[(size_t)threadIdx.x * nblk + blk] = t2;
        }
    }
}

template <typename VT, typename LT, int MODE, int BATCH, bool STG>
inline hipError_t launch_nr(const LT* links, int nlinks, const DslashArgs<VT>& a, int nr,
                            dim3 grid, dim3 block, size_t lds, hipStream_t s) {
    switch (nr) {
        case 1: hipLaunchKernelGGL((k_dslash<VT, LT, 1, MODE, true, BATCH, STG>), grid, block, lds, s, links, nlinks, a); break;
        case 2: hipLaunchKernelGGL((k_dslash<VT, LT, 2, MODE, true, BATCH, STG>), grid, block, lds, s, links, nlinks, a); break;
        case 4: hipLaunchKernelGGL((k_dslash<VT, LT, 4, MODE, true, BATCH, STG>), grid, block, lds, s, links, nlinks, a); break;
        default: hipLaunchKernelGGL((k_dslash<VT, LT, 8, MODE, true, BATCH, STG>), grid, block, lds, s, links, nlinks, a); break;
    }
    return hipGetLastError();
}

template <typename VT, typename LT, int MODE, bool STG>
inline hipError_t launch_batch(const LT* links, int nlinks, const DslashArgs<VT>& a, int nr,
                               int batch, dim3 grid, dim3 block, size_t lds, hipStream_t s) {
    switch (batch) {
        case 0: return launch_nr<VT, LT, MODE, 1, STG>(links, nlinks, a, nr, grid, block, lds, s);
        case 1: return launch_nr<VT, LT, MODE, 2, STG>(links, nlinks, a, nr, grid, block, lds, s);
        default: return launch_nr<VT, LT, MODE, 4, STG>(links, nlinks, a, nr, grid, block, lds, s);
    }
}

// One launch of the kernel for nr right-hand sides in the shape of variant v.
template <typename VT, typename LT, int MODE>
inline hipError_t launch_shape(const LT* links, int nlinks, const DslashArgs<VT>& a, int nr, int v,
                               hipStream_t s) {
    const int shape = hop_stage(v);
    const int R = stage_rows(a.g, shape, nr, (int)sizeof(VT));
    const int batch = hop_batch(v);
    if (R) {
        const int B = R * a.g.hx;
        const size_t lds = (size_t)nr * 3 * (R + 2) * a.g.hx * sizeof(VT);
        return launch_batch<VT, LT, MODE, true>(links, nlinks, a, nr, batch, dim3(a.g.Vh / B),
                                                dim3(B), lds, s);
    }
    const int B = hop_block(shape);
    return launch_batch<VT, LT, MODE, false>(links, nlinks, a, nr, batch,
                                             dim3((a.g.Vh + B - 1) / B), dim3(B), 0, s);
}

// One hopping application in the variant a.variant (see kHopVariants).
template <typename VT, typename LT, int MODE>
inline hipError_t dispatch(const LT* links, int nlinks, const DslashArgs<VT>& a0, hipStream_t s) {
    DslashArgs<VT> a = a0;
    const int v = a.variant >= 0 && a.variant < kHopVariants ? a.variant : 0;
    int zt = kZTile[hop_order(v)];
    if (zt > 0 && a.g.Lz % zt != 0) zt = 1;
    a.zt = zt ? make_fastdiv((uint32_t)zt) : FastDiv{0u, 0u, 0u, 0u};
    int nr = nr_of_class(nr_class(a.nrhs));
    if (std::is_same<VT, float2>::value) {
        // FP32 sets of two or more right-hand sides are paired; a launch over
        // the last, unpaired member of such a set runs the pair kernel
        if (a.paired && nr == 1) nr = 2;
        if (!a.paired && nr > 1) return hipErrorInvalidValue;
    }
    const int nt = hop_tile_nr(v, nr);
    if (nt == nr) return launch_shape<VT, LT, MODE>(links, nlinks, a, nr, v, s);
    // rhs tile: launches over rhs [0, nt) and [nt, nrhs), both with the
    // template (and so the grid) for nt rhs, so that the partial sums of a
    // reducing mode keep one layout; nt is even, so FP32 pairs stay whole
    const int grid = hop_grid(a.g, v, nr, (int)sizeof(VT));
    DslashArgs<VT> hi = a;
    hi.nrhs = a.nrhs - nt;
    for (int r = 0; r < hi.nrhs; ++r) {
        hi.in[r] = a.in[nt + r];
        hi.out[r] = a.out[nt + r];
        hi.self[r] = a.self[nt + r];
        hi.rhs[r] = a.rhs[nt + r];
        hi.out32[r] = a.out32[nt + r];
        hi.c[r] = a.c[nt + r];
    }
    if (a.skip) hi.skip = a.skip + (size_t)nt * a.skip_stride;
    if (a.partial) hi.partial = a.partial + (size_t)nt * grid;
    a.nrhs = nt;
    const hipError_t e = launch_shape<VT, LT, MODE>(links, nlinks, a, nt, v, s);
    if (e != hipSuccess) return e;
    return launch_shape<VT, LT, MODE>(links, nlinks, hi, nt, v, s);
}

}  // namespace rhmc
