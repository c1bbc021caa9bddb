// Internal declarations shared by the HIP sources of librhmc.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "rhmc.h"

namespace rhmc {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);

#define RHMC_HIP_TRY(expr)                                                           \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess) {                                                      \
            ::rhmc::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));    \
            return e_ == hipErrorOutOfMemory ? RHMC_ERR_OOM : RHMC_ERR_HIP;          \
        }                                                                            \
    } while (0)

#define RHMC_TRY(expr)                            \
    do {                                          \
        rhmc_status s_ = (expr);                  \
        if (s_ != RHMC_OK) return s_;             \
    } while (0)

// ---------------------------------------------------------------- geometry
// Everything a kernel needs to locate a site and its eight neighbours.
struct Geom {
    int Lx, Ly, Lz, Lt;
    int hx;          // Lx / 2
    int Vh;          // sites per parity
    int sy, sz, st;  // eo strides of one step in y, z, t: hx, hx*Ly, hx*Ly*Lz
    int tbc;         // +1 or -1
};

constexpr int kBlock = 256;       // threads per block for every kernel
constexpr int kMaxSys = 8;        // right-hand sides per operator launch
constexpr int kMaxShift = 32;
constexpr int kMaxBlockLen = 50;  // iterations between shifted-solution updates

#if defined(__HIPCC__)
// Blocks of a launch are dispatched round-robin over the eight XCDs; give
// each XCD a contiguous range of sites so that neighbour reuse stays in its L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblk) {
    const int q = nblk >> 3, r = nblk & 7;
    const int xcd = bid & 7, local = bid >> 3;
    return (xcd < r) ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

// Coordinates of site eo of parity par.
__device__ __forceinline__ void site_coords(const Geom& g, int eo, int par, int& x, int& y,
                                            int& z, int& t) {
    const int xh = eo % g.hx;
    int r = eo / g.hx;
    y = r % g.Ly;
    r /= g.Ly;
    z = r % g.Lz;
    t = r / g.Lz;
    x = 2 * xh + ((par + y + z + t) & 1);
}

// Site visited by processing index p (0 <= p < Vh) of a hopping launch.
// Blocks give each XCD a contiguous range of p, so the order decides how far
// apart (in sites processed) the eight uses of an input site are:
//   0: the eo index itself (x fastest, then y, z, t)
//   1: x, y, t, z             (t neighbours one xy-plane apart)
//   2: x, y, z mod 4, t, z/4  (z-tiles of 4 planes, t inside the tile)
//   3: x, y, z mod 2, t, z/2  (z-tiles of 2 planes)
// Order 2 needs Lz % 4 == 0 (the launcher falls back to 1 otherwise).
__device__ __forceinline__ void process_site(const Geom& g, int p, int par, int order, int& eo,
                                             int& x, int& y, int& z, int& t) {
    if (order == 0) {
        eo = p;
        site_coords(g, eo, par, x, y, z, t);
        return;
    }
    const int xh = p % g.hx;
    int r = p / g.hx;
    y = r % g.Ly;
    r /= g.Ly;
    if (order == 1) {
        t = r % g.Lt;
        z = r / g.Lt;
    } else {
        const int T = order == 2 ? 4 : 2;
        const int tz = r % T;
        r /= T;
        t = r % g.Lt;
        z = (r / g.Lt) * T + tz;
    }
    eo = xh + g.hx * (y + g.Ly * (z + g.Lz * t));
    x = 2 * xh + ((par + y + z + t) & 1);
}

// The eight neighbours (eo index, opposite parity) of site eo with coordinates
// (x,y,z,t) and the real factor multiplying each hop of D (Eq. stag):
//   forward  hop mu: +1/2 * eta_mu(n) * bc,  acts with U_mu(n)
//   backward hop mu: -1/2 * eta_mu(n) * bc,  acts with U_mu(n-mu)^dagger
// eta_mu(n) = (-1)^(x + ... + n_{mu-1}); bc = t_bc on a hop that wraps in t.
struct Hops {
    int nb[8];      // 0..3 forward, 4..7 backward
    float coef[8];  // +-0.5 exactly
};

__device__ __forceinline__ Hops make_hops(const Geom& g, int eo, int x, int y, int z, int t) {
    Hops h;
    const int row = g.Lx * (y + g.Ly * (z + g.Lz * t));
    const int xp = (x + 1 == g.Lx) ? 0 : x + 1;
    const int xm = (x == 0) ? g.Lx - 1 : x - 1;
    h.nb[0] = (row + xp) >> 1;
    h.nb[4] = (row + xm) >> 1;
    h.nb[1] = (y + 1 == g.Ly) ? eo - (g.Ly - 1) * g.sy : eo + g.sy;
    h.nb[5] = (y == 0) ? eo + (g.Ly - 1) * g.sy : eo - g.sy;
    h.nb[2] = (z + 1 == g.Lz) ? eo - (g.Lz - 1) * g.sz : eo + g.sz;
    h.nb[6] = (z == 0) ? eo + (g.Lz - 1) * g.sz : eo - g.sz;
    h.nb[3] = (t + 1 == g.Lt) ? eo - (g.Lt - 1) * g.st : eo + g.st;
    h.nb[7] = (t == 0) ? eo + (g.Lt - 1) * g.st : eo - g.st;
    const float e1 = (x & 1) ? -0.5f : 0.5f;
    const float e2 = ((x + y) & 1) ? -0.5f : 0.5f;
    const float e3 = ((x + y + z) & 1) ? -0.5f : 0.5f;
    const float bf = (t + 1 == g.Lt) ? (float)g.tbc : 1.0f;
    const float bb = (t == 0) ? (float)g.tbc : 1.0f;
    h.coef[0] = 0.5f;
    h.coef[4] = -0.5f;
    h.coef[1] = e1;
    h.coef[5] = -e1;
    h.coef[2] = e2;
    h.coef[6] = -e2;
    h.coef[3] = e3 * bf;
    h.coef[7] = -e3 * bb;
    return h;
}
#endif  // __HIPCC__

}  // namespace rhmc

// ---------------------------------------------------------------- objects
struct rhmc_lattice {
    int32_t L[4];
    int32_t t_bc;
    int64_t V, Vh;
    rhmc::Geom geom;
};

namespace rhmc {
struct Workspace;  // solver workspace, defined in solver.hip
void workspace_destroy(Workspace* w);
void md_destroy(void* md);  // md.hip
}  // namespace rhmc

struct rhmc_gauge {
    rhmc_lattice lat;
    int device;
    double2* u64c; // FP64-12: [6][8*Vh], rows 1-2; row 3 rebuilt in FP64
    double2* u64;  // FP64-18: [9][8*Vh] entry-major, link k = (2*mu + parity)*Vh + eo
    float4* u32;   // FP32-12: [3][8*Vh], rows 1-2 as three float4 per link; with
                   // hilo, [6][8*Vh]: planes 3-5 hold the FP32 remainders (lo)
    float2* u32f;  // FP32-18: [9][8*Vh] entry-major (no reconstruction)
    int hilo;      // FP64 operator available from hi + lo (no u64 needed)
    void* tmp_odd;           // odd-parity temporary for rhmc_apply_mdagm
    size_t tmp_odd_bytes;
    double* partial;         // [kMaxSys][hopping grid] block sums of rhmc_apply_mdagm
    rhmc::Workspace* ws;     // solver workspace (lazily created)
    int hop_variant[2][4];   // launch variant per [RHMC_PREC_*][rhs class]
    int hop_tuned[2][4];     // 1 once the autotuner has timed that case
    void* md;                // molecular-dynamics buffers (md.hip, lazily created)
};

namespace rhmc {

// ---------------------------------------------------------------- launchers
// Operator modes of the hopping kernel.
enum DslashMode {
    kModeD = 0,      // out = D in
    kModeA = 1,      // out = c*self - D in; partial Re<self, out> per rhs
    kModeResid = 2   // out = rhs - c*self + D in (FP64); partial ||out||^2 per rhs
};

// Arguments of one hopping launch over up to kMaxSys right-hand sides.
template <typename VT>
struct DslashArgs {
    Geom g;
    int out_par;
    int nrhs;
    const VT* in[kMaxSys];        // input of the opposite parity
    VT* out[kMaxSys];             // may be null in kModeResid
    const VT* self[kMaxSys];      // kModeA: p; kModeResid: x (output parity)
    const double2* rhs[kMaxSys];  // kModeResid: b
    float2* out32[kMaxSys];       // kModeResid: optional FP32 copy of the result
    double c[kMaxSys];            // diagonal coefficient m^2 + sigma
    const int* skip;              // if non-null: skip[r*skip_stride] != 0 -> rhs r finished
    int skip_stride;
    const int* all_done;          // if non-null and set: the launch does nothing
    double* partial;              // [nrhs][nblocks] block sums (kModeA, kModeResid)
    int variant;                  // launch variant (HopVariant index)
};

// Launch variants of the hopping kernel, index = order | nt << 2 | batch << 3
// | occ << 5:
//   order  site processing order (process_site), 0..3
//   nt     non-temporal (streaming) loads of the links, which are read once
//          per application and need not displace neighbour vectors
//   batch  hops whose loads are issued together: 1, 2, 4 or 8 (bits 0..3)
//   occ    cap on resident workgroups per CU (none, 5, 4, 3), set through an
//          unused dynamic LDS allocation: fewer sites in flight per XCD keep
//          the neighbour vectors they share inside that XCD's L2
constexpr int kHopVariants = 128;
// dynamic LDS bytes per workgroup for occ = 0..3 (160 KB of LDS per CU)
constexpr int kOccLds[4] = {0, 32 * 1024, 40 * 1024, 53 * 1024};
// right-hand-side classes of the kernel templates: 1, 2, 4, 8
inline int nr_class(int nrhs) { return nrhs <= 1 ? 0 : nrhs <= 2 ? 1 : nrhs <= 4 ? 2 : 3; }
// measured defaults on MI355X (48^3 x 12), [precision][rhs class]
void default_hop_variants(int (&v)[2][4]);

// Geometry of a hopping launch.
int dslash_grid(int Vh);

hipError_t launch_pack_links(const rhmc_gauge* g, const double2* canon, hipStream_t s);
// Links of the FP64 operator rebuilt from the FP32 hi and lo planes.
struct HiLoLink {
    float4 v;
};
// FP64 links with the first two rows stored (12 reals).
struct Fp64x12Link {
    double2 v;
};
// FP32 links with all 18 reals stored.
struct Fp32x18Link {
    float2 v;
};
hipError_t launch_dslash64c(const Fp64x12Link* u, int nlinks, const DslashArgs<double2>& a,
                            int mode, hipStream_t s);
hipError_t launch_dslash64hl(const HiLoLink* u, int nlinks, const DslashArgs<double2>& a,
                             int mode, hipStream_t s);
hipError_t launch_dslash64(const double2* u64, int nlinks, const DslashArgs<double2>& a,
                           int mode, hipStream_t s);
hipError_t launch_dslash32(const float4* u32, int nlinks, const DslashArgs<float2>& a,
                           int mode, hipStream_t s);
hipError_t launch_dslash32f(const Fp32x18Link* u, int nlinks, const DslashArgs<float2>& a,
                            int mode, hipStream_t s);

// The FP32 operator of a gauge object: FP32-12 links if stored, else FP32-18.
inline hipError_t launch_fp32_op(const rhmc_gauge* g, const DslashArgs<float2>& a, int mode,
                                 hipStream_t s) {
    const int nlinks = (int)(4 * g->lat.V);
    if (g->u32) return launch_dslash32(g->u32, nlinks, a, mode, s);
    return launch_dslash32f(reinterpret_cast<const Fp32x18Link*>(g->u32f), nlinks, a, mode, s);
}
inline bool has_fp32_op(const rhmc_gauge* g) { return g->u32 || g->u32f; }
hipError_t launch_neighbors(const Geom& g, int par, int* nb, int* sign, hipStream_t s);

// The FP64 operator of a gauge object: FP64-12 links if stored, else FP64-18,
// else hi + lo.
inline hipError_t launch_fp64_op(const rhmc_gauge* g, const DslashArgs<double2>& a, int mode,
                                 hipStream_t s) {
    const int nlinks = (int)(4 * g->lat.V);
    if (g->u64c)
        return launch_dslash64c(reinterpret_cast<const Fp64x12Link*>(g->u64c), nlinks, a, mode, s);
    if (g->u64) return launch_dslash64(g->u64, nlinks, a, mode, s);
    return launch_dslash64hl(reinterpret_cast<const HiLoLink*>(g->u32), nlinks, a, mode, s);
}
inline bool has_fp64_op(const rhmc_gauge* g) {
    return g->u64c || g->u64 || (g->u32 && g->hilo);
}

// Pick the launch variant of the gauge object for this precision and nrhs.
template <typename VT>
inline void set_variant(DslashArgs<VT>& a, const rhmc_gauge* g) {
    a.variant = g->hop_variant[sizeof(VT) == 8 ? RHMC_PREC_FP32 : RHMC_PREC_FP64][nr_class(a.nrhs)];
}

// Time every launch variant of one hopping application (out_parity 1, plain D)
// on the given vectors and keep the fastest in the gauge object.
rhmc_status tune_hop(rhmc_gauge* g, rhmc_prec prec, int nrhs, const void* in, void* out,
                     hipStream_t s);

}  // namespace rhmc
