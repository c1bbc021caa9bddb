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
// Division of non-negative 32-bit integers by a divisor fixed at set-up:
// q = (t + ((n - t) >> s1)) >> s2 with t = mulhi(m, n), exact for every
// divisor d >= 1 and dividend n < 2^32 (round-up multiply-high method of
// Granlund and Montgomery, 1994).  Replaces the ~25-instruction integer
// division in the index arithmetic of every site.
struct FastDiv {
    uint32_t d, m, s1, s2;
};

inline FastDiv make_fastdiv(uint32_t d) {
    uint32_t l = 0;
    while (l < 32 && (uint64_t(1) << l) < d) ++l;
    FastDiv f;
    f.d = d;
    f.m = (uint32_t)(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
    f.s1 = l < 1 ? l : 1;
    f.s2 = l > 0 ? l - 1 : 0;
    return f;
}

// Everything a kernel needs to locate a site and its eight neighbours.
struct Geom {
    int Lx, Ly, Lz, Lt;
    int hx;          // Lx / 2
    int Vh;          // sites per parity
    int sy, sz, st;  // eo strides of one step in y, z, t: hx, hx*Ly, hx*Ly*Lz
    int tbc;         // +1 or -1
    FastDiv dhx, dLy, dLz, dLt;
};

// Fills the divisor tables of a geometry whose extents are set.
inline void geom_init_divs(Geom& g) {
    g.dhx = make_fastdiv((uint32_t)g.hx);
    g.dLy = make_fastdiv((uint32_t)g.Ly);
    g.dLz = make_fastdiv((uint32_t)g.Lz);
    g.dLt = make_fastdiv((uint32_t)g.Lt);
}

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

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
    const uint32_t t = __umulhi(f.m, n);
    return (t + ((n - t) >> f.s1)) >> f.s2;
}

// q = n / d and r = n % d
__device__ __forceinline__ void fdivmod(int n, const FastDiv& f, int& q, int& r) {
    q = (int)fdiv((uint32_t)n, f);
    r = n - q * (int)f.d;
}

// Coordinates of site eo of parity par.
__device__ __forceinline__ void site_coords(const Geom& g, int eo, int par, int& x, int& y,
                                            int& z, int& t) {
    int xh, r;
    fdivmod(eo, g.dhx, r, xh);
    fdivmod(r, g.dLy, r, y);
    fdivmod(r, g.dLz, t, z);
    x = 2 * xh + ((par + y + z + t) & 1);
}

// Site visited by processing index p (0 <= p < Vh) of a hopping launch.
// Blocks give each XCD a contiguous range of p, so the order decides how far
// apart (in sites processed) the eight uses of an input site are:
//   zt == 0: the eo index itself (x fastest, then y, z, t)
//   zt >= 1: x, y, z mod zt, t, z / zt: z-tiles of zt planes with t inside a
//            tile (zt == 1: x, y, t, z), so that the t neighbours of a wave's
//            sites are zt xy-planes away; zt must divide Lz
__device__ __forceinline__ void process_site(const Geom& g, int p, int par, const FastDiv& zt,
                                             int& eo, int& x, int& y, int& z, int& t) {
    if (zt.d == 0) {
        eo = p;
        site_coords(g, eo, par, x, y, z, t);
        return;
    }
    int xh, r, tz;
    fdivmod(p, g.dhx, r, xh);
    fdivmod(r, g.dLy, r, y);
    fdivmod(r, zt, r, tz);
    int zq;
    fdivmod(r, g.dLt, zq, t);
    z = zq * (int)zt.d + tz;
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
// The two hops of direction mu (0..3, may differ per lane) from site eo
// with coordinates (x,y,z,t) and row = Lx*(y + Ly*(z + Lz*t)): neighbour eo
// indices n +- mu and the factors of D on them (as in make_hops).
__device__ __forceinline__ void dir_hops(const Geom& g, int mu, int eo, int x, int y, int z,
                                         int t, int row, int& nbp, int& nbm, float& cp,
                                         float& cm) {
    // The extents and strides are uniform; reading them through readfirstlane
    // keeps a select between fields of g (mu differs per lane) from becoming
    // an indexed access to the kernel argument, which would be copied to scratch.
    const int Lx = __builtin_amdgcn_readfirstlane(g.Lx), Ly = __builtin_amdgcn_readfirstlane(g.Ly);
    const int Lz = __builtin_amdgcn_readfirstlane(g.Lz), Lt = __builtin_amdgcn_readfirstlane(g.Lt);
    const int sy = __builtin_amdgcn_readfirstlane(g.sy), sz = __builtin_amdgcn_readfirstlane(g.sz);
    const int st = __builtin_amdgcn_readfirstlane(g.st);
    const int c = mu == 0 ? x : mu == 1 ? y : mu == 2 ? z : t;
    const int L = mu == 0 ? Lx : mu == 1 ? Ly : mu == 2 ? Lz : Lt;
    const int stride = mu == 1 ? sy : mu == 2 ? sz : st;
    const bool fw = c + 1 == L, bw = c == 0;
    if (mu == 0) {
        nbp = (row + (fw ? 0 : x + 1)) >> 1;
        nbm = (row + (bw ? Lx - 1 : x - 1)) >> 1;
    } else {
        nbp = fw ? eo - (L - 1) * stride : eo + stride;
        nbm = bw ? eo + (L - 1) * stride : eo - stride;
    }
    const int par = mu == 0 ? 0 : mu == 1 ? x : mu == 2 ? x + y : x + y + z;
    const float eta = (par & 1) ? -0.5f : 0.5f;
    cp = (mu == 3 && fw) ? eta * (float)g.tbc : eta;
    cm = (mu == 3 && bw) ? -eta * (float)g.tbc : -eta;
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
    int solver_depth;        // solver calls in progress on this object (nested)
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

// FP32 vector sets of two or more right-hand sides are stored in pairs: pair
// q = (rhs 2q, rhs 2q + 1) is a [3][Vh] array of float4 (re, im of rhs 2q,
// re, im of rhs 2q + 1), so element (r, c, eo) of a set is the complex64 at
// ((r/2)*3*Vh + c*Vh + eo)*2 + r%2.  A set of an odd count holds a last pair
// with an unused second half.  One right-hand side alone is a plain [3][Vh]
// array (FP64 sets are always plain [nrhs][3][Vh]).
inline bool paired_f32(int nrhs) { return nrhs >= 2; }
// complex64 offset of element i (< 3*Vh) of rhs r in an FP32 set
__host__ __device__ inline size_t f32_offset(bool paired, int r, size_t i, size_t n) {
    return paired ? (((size_t)(r >> 1) * n + i) << 1) + (size_t)(r & 1) : (size_t)r * n + i;
}
// complex64 entries an FP32 set of nrhs vectors of n entries occupies
inline size_t f32_set_size(int nrhs, size_t n) {
    return (size_t)(paired_f32(nrhs) ? (nrhs + 1) / 2 * 2 : nrhs) * n;
}

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
    int out32_paired;             // 1: out32 is a paired FP32 set (element stride 2)
    int paired;                   // FP32: in/out/self are paired sets (f32_offset)
    double c[kMaxSys];            // diagonal coefficient m^2 + sigma
    const int* skip;              // if non-null: skip[r*skip_stride] != 0 -> rhs r finished
    int skip_stride;
    const int* all_done;          // if non-null and set: the launch does nothing
    double* partial;              // [nrhs][nblocks] block sums (kModeA, kModeResid)
    int variant;                  // launch variant (HopVariant index)
    FastDiv zt;                   // site order: z-tile planes (d == 0: eo order), set at launch
};

// Launch variants of the hopping kernel,
// index = order + 8 * batch + 24 * shape + 96 * tile:
//   order  site processing order (process_site): 0 the eo index; 1..7 z-tiles
//          of kZTile[order] planes with t inside a tile (a tile size that does
//          not divide Lz falls back to 1)
//   batch  hops whose loads are issued together: 1, 2 or 4
//   shape  block shape: 0 blocks of 256 sites; 1, 2 blocks of whole rows of
//          the xy-plane staged in LDS (the fewest, the most rows that fit;
//          stage_rows), so the +-x and +-y hops read LDS (falls back to 0
//          where no row count fits); 3 blocks of 128 sites
//   tile   right-hand sides per launch: 0 all of the launch's class; 1 half
//          of a class of four or eight, i.e. two launches (each link then read
//          twice, each launch holding half the rhs registers)
// Link loads are non-temporal (read once per application).  Every variant
// computes the same bits.
constexpr int kHopOrders = 8, kHopBatches = 3, kHopShapes = 4, kHopTiles = 2;
constexpr int kHopVariants = kHopOrders * kHopBatches * kHopShapes * kHopTiles;
constexpr int kZTile[kHopOrders] = {0, 1, 2, 4, 6, 8, 3, 12};
inline int hop_order(int v) { return v % kHopOrders; }
inline int hop_batch(int v) { return (v / kHopOrders) % kHopBatches; }
inline int hop_stage(int v) { return (v / (kHopOrders * kHopBatches)) % kHopShapes; }
inline int hop_tile(int v) { return v / (kHopOrders * kHopBatches * kHopShapes); }
// sites per block of an unstaged launch of this shape
inline int hop_block(int shape) { return shape == 3 ? 128 : kBlock; }
// rhs per launch of this variant in a launch class of nr rhs (tiles stay
// even, so FP32 pairs stay whole)
inline int hop_tile_nr(int variant, int nr) { return (hop_tile(variant) && nr >= 4) ? nr / 2 : nr; }
// right-hand-side classes of the kernel templates: 1, 2, 4, 8
inline int nr_class(int nrhs) { return nrhs <= 1 ? 0 : nrhs <= 2 ? 1 : nrhs <= 4 ? 2 : 3; }
inline int nr_of_class(int cls) { return 1 << cls; }
// measured defaults on MI355X (48^3 x 12), [precision][rhs class]
void default_hop_variants(int (&v)[2][4]);

// LDS budget of a staged block (three blocks fit a CU's 160 KB)
constexpr size_t kStageLdsMax = 48 * 1024;

// Rows per block of a staged launch (0: staging not possible): R divides Ly,
// the block of R * Lx/2 sites is a whole number of waves (64..512 sites), and
// the staged input [NR][3][R + 2][Lx/2] fits the LDS budget; stage 1 takes
// the smallest such R, stage 2 the largest; other shapes stage nothing.
inline int stage_rows(const Geom& g, int stage, int nr, int vt_bytes) {
    if (stage != 1 && stage != 2) return 0;
    int best = 0;
    for (int R = 1; R <= g.Ly; ++R) {
        const int B = R * g.hx;
        if (g.Ly % R || B % 64 || B > 512) continue;
        const size_t lds = (size_t)nr * 3 * (R + 2) * g.hx * vt_bytes;
        if (lds > kStageLdsMax) continue;
        if (stage == 1) return R;
        best = R;
    }
    return best;
}

// Blocks of a hopping launch of this variant (one partial sum per block and
// rhs in the reducing modes); at most max_hop_grid(Vh).
// (Both launches of a tiled variant have this grid.)
inline int hop_grid(const Geom& g, int variant, int nr, int vt_bytes) {
    nr = hop_tile_nr(variant, nr);
    const int R = stage_rows(g, hop_stage(variant), nr, vt_bytes);
    if (R) return g.Vh / (R * g.hx);
    const int B = hop_block(hop_stage(variant));
    return (g.Vh + B - 1) / B;
}
inline int max_hop_grid(int Vh) { return (Vh + 63) / 64; }

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

// Blocks of the hopping launch the gauge object makes for this precision and
// rhs count (the consumer of the partial sums needs their number).
inline int gauge_hop_grid(const rhmc_gauge* g, rhmc_prec prec, int nrhs) {
    const int cls = nr_class(nrhs);
    return hop_grid(g->lat.geom, g->hop_variant[prec][cls], nr_of_class(cls),
                    prec == RHMC_PREC_FP32 ? 8 : 16);
}

// Time every launch variant of one hopping application (out_parity 1, plain D)
// on the given vectors and keep the fastest in the gauge object.
rhmc_status tune_hop(rhmc_gauge* g, rhmc_prec prec, int nrhs, const void* in, void* out,
                     hipStream_t s);

}  // namespace rhmc
