// C ABI of librhmc (include/rhmc.h): argument validation, object lifetime and
// dispatch to the kernels and the solver driver.  No exception crosses the ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "common.h"
#include "gauge.h"
#include "md.h"
#include "solver.h"

namespace rhmc {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

static rhmc_status invalid(const std::string& msg) {
    set_error(msg);
    return RHMC_ERR_INVALID_ARG;
}

static rhmc_status use_device(int dev) {
    RHMC_HIP_TRY(hipSetDevice(dev));
    return RHMC_OK;
}

// ---------------------------------------------------------------- static scratch
// Device memory of rhmc_apply_mdagm_static: the odd-parity temporary and the
// block partial sums of A live in this array instead of buffers the gauge
// object allocates.  Each GPU holds its own copy for the life of the process;
// its address is looked up once per device, with that device current, and
// only that address is passed to kernels.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static void* g_scratch_addr[kMaxDevices] = {};

// Address of this device's scratch (the device must be current).
static rhmc_status scratch_address(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices) return invalid("device index out of range for the static scratch");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_addr[dev]) {
        void* p = nullptr;
        RHMC_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) {
            set_error("hipGetSymbolAddress returned no address for the static scratch");
            return RHMC_ERR_HIP;
        }
        g_scratch_addr[dev] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_addr[dev]);
    return RHMC_OK;
}

// Bytes of a vector set of nrhs vectors of one parity (FP32 sets of two or
// more are paired, with room for an even count).
static size_t vec_set_bytes(const rhmc_gauge* g, rhmc_prec prec, int nrhs) {
    const size_t n = (size_t)3 * g->lat.Vh;
    return prec == RHMC_PREC_FP64 ? sizeof(double2) * n * nrhs : sizeof(float2) * f32_set_size(nrhs, n);
}

// Bytes of scratch rhmc_apply_mdagm_static needs: the partial sums (rounded
// up to 256 bytes), then nrhs odd-parity vectors.
static size_t static_mdagm_bytes(const rhmc_gauge* g, rhmc_prec prec, int nrhs, size_t* part_bytes) {
    const size_t pb = sizeof(double) * kMaxSys * (size_t)max_hop_grid((int)g->lat.Vh);
    *part_bytes = (pb + 255) & ~size_t(255);
    return *part_bytes + vec_set_bytes(g, prec, nrhs);
}


// Odd-parity temporary of the gauge object, grown on demand.
static rhmc_status tmp_odd(rhmc_gauge* g, size_t bytes, void** out) {
    if (g->tmp_odd_bytes < bytes) {
        hipFree(g->tmp_odd);
        g->tmp_odd = nullptr;
        g->tmp_odd_bytes = 0;
        RHMC_HIP_TRY(hipMalloc(&g->tmp_odd, bytes));
        g->tmp_odd_bytes = bytes;
    }
    *out = g->tmp_odd;
    return RHMC_OK;
}

template <typename VT>
static rhmc_status hop(rhmc_gauge* g, int out_par, rhmc_prec prec, int nrhs, const void* in,
                       void* out, int mode, const void* self, double c, hipStream_t s,
                       double* partial_buf = nullptr) {
    const size_t n = (size_t)3 * g->lat.Vh;
    // kModeA partial sums nobody reads: [kMaxSys][max_hop_grid] doubles
    double* partial = partial_buf ? partial_buf : g->partial;
    // FP32 sets of two or more vectors are paired (f32_offset); launches
    // over kMaxSys (even) of them at a time start at a pair
    const bool pr = std::is_same<VT, float2>::value && paired_f32(nrhs);
    for (int r0 = 0; r0 < nrhs; r0 += kMaxSys) {
        const int cnt = nrhs - r0 < kMaxSys ? nrhs - r0 : kMaxSys;
        DslashArgs<VT> a{};
        a.g = g->lat.geom;
        a.out_par = out_par;
        a.nrhs = cnt;
        a.partial = partial;
        a.paired = pr;
        for (int k = 0; k < cnt; ++k) {
            const size_t o = f32_offset(pr, r0 + k, 0, n);
            a.in[k] = reinterpret_cast<const VT*>(in) + o;
            a.out[k] = reinterpret_cast<VT*>(out) + o;
            if (self) a.self[k] = reinterpret_cast<const VT*>(self) + o;
            a.c[k] = c;
        }
        set_variant(a, g);
        if constexpr (std::is_same<VT, double2>::value) {
            RHMC_HIP_TRY(launch_fp64_op(g, a, mode, s));
        } else {
            RHMC_HIP_TRY(launch_fp32_op(g, a, mode, s));
        }
    }
    (void)prec;
    return RHMC_OK;
}

static rhmc_status check_prec(const rhmc_gauge* g, rhmc_prec prec) {
    if (prec == RHMC_PREC_FP64 && !has_fp64_op(g))
        return invalid("gauge object has no FP64 operator (FP64-18 or hi/lo links)");
    if (prec == RHMC_PREC_FP32 && !has_fp32_op(g)) return invalid("gauge object has no FP32 links");
    if (prec != RHMC_PREC_FP64 && prec != RHMC_PREC_FP32) return invalid("unknown precision");
    return RHMC_OK;
}

static rhmc_status check_params(const rhmc_solver_params* p, const rhmc_gauge* g,
                                rhmc_solver_params* out) {
    rhmc_solver_params_default(out);
    if (p) *out = *p;
    if (!(out->tol > 0) || !std::isfinite(out->tol)) return invalid("tol must be positive");
    if (out->maxiter < 1) return invalid("maxiter must be >= 1");
    if (out->mode != RHMC_MODE_FP64 && out->mode != RHMC_MODE_MIXED) return invalid("unknown mode");
    if (out->block < 1 || out->block > kMaxBlockLen) return invalid("block must be in 1..50");
    if (out->reliable_every < 1) return invalid("reliable_every must be >= 1");
    if (std::isnan(out->fp64_head)) return invalid("fp64_head is NaN");
    if (out->two_pass && out->mode != RHMC_MODE_FP64) {
        set_error("two_pass needs mode FP64: a mixed solve needs its shifted solutions for refinement");
        return RHMC_ERR_UNSUPPORTED;
    }
    if (out->two_pass && out->per_shift) return invalid("two_pass and per_shift exclude each other");
    if (!has_fp64_op(g))
        return invalid("solvers need an FP64 operator (FP64-18 or hi/lo links): true residuals are FP64");
    if (out->mode == RHMC_MODE_MIXED && !has_fp32_op(g)) return invalid("MIXED mode needs FP32 links");
    return RHMC_OK;
}

}  // namespace rhmc

using namespace rhmc;

extern "C" {

void rhmc_solver_params_default(rhmc_solver_params* p) {
    if (!p) return;
    p->tol = 1e-10;
    p->maxiter = 100000;
    p->mode = RHMC_MODE_FP64;
    p->reliable_every = 50;
    p->refine = 1;
    p->block = 32;
    p->use_graph = 1;
    p->poll_every = 0;
    p->tune = 0;
    p->per_shift = 0;
    p->fp64_head = 0.0;
    p->two_pass = 0;
}

rhmc_status rhmc_lattice_create(const int32_t L[4], int32_t t_bc, rhmc_lattice** out) {
    if (!L || !out) return invalid("null argument");
    *out = nullptr;
    int64_t V = 1;
    for (int i = 0; i < 4; ++i) {
        if (L[i] < 2 || (L[i] & 1)) return invalid("every lattice extent must be even and >= 2");
        V *= L[i];
    }
    // 32-bit byte offsets within a link plane (8 * Vh entries of up to 16 B)
    if (V > (int64_t(1) << 26)) return invalid("lattice volume above 2^26 sites");
    if (t_bc != 1 && t_bc != -1) return invalid("t_bc must be +1 or -1");
    rhmc_lattice* lat = new (std::nothrow) rhmc_lattice();
    if (!lat) return RHMC_ERR_OOM;
    std::memcpy(lat->L, L, sizeof(lat->L));
    lat->t_bc = t_bc;
    lat->V = V;
    lat->Vh = V / 2;
    Geom& g = lat->geom;
    g.Lx = L[0];
    g.Ly = L[1];
    g.Lz = L[2];
    g.Lt = L[3];
    g.hx = L[0] / 2;
    g.Vh = (int)(V / 2);
    g.sy = g.hx;
    g.sz = g.hx * L[1];
    g.st = g.hx * L[1] * L[2];
    g.tbc = t_bc;
    geom_init_divs(g);
    *out = lat;
    return RHMC_OK;
}

void rhmc_lattice_destroy(rhmc_lattice* lat) { delete lat; }

rhmc_status rhmc_debug_neighbors(const rhmc_lattice* lat, int32_t parity, int32_t* out,
                                 int32_t* sign) {
    if (!lat || !out) return invalid("null argument");
    if (parity != 0 && parity != 1) return invalid("parity must be 0 or 1");
    const size_t cnt = (size_t)lat->Vh * 8;
    int *d_nb = nullptr, *d_sg = nullptr;
    RHMC_HIP_TRY(hipMalloc(&d_nb, cnt * sizeof(int)));
    hipError_t e = hipMalloc(&d_sg, cnt * sizeof(int));
    if (e == hipSuccess) e = launch_neighbors(lat->geom, parity, d_nb, d_sg, 0);
    if (e == hipSuccess) e = hipMemcpy(out, d_nb, cnt * sizeof(int), hipMemcpyDeviceToHost);
    if (e == hipSuccess && sign) e = hipMemcpy(sign, d_sg, cnt * sizeof(int), hipMemcpyDeviceToHost);
    hipFree(d_nb);
    hipFree(d_sg);
    RHMC_HIP_TRY(e);
    return RHMC_OK;
}

// Largest |U_3j - conj(row1 x row2)_j| over all links (host array, complex128
// [..][3][3]): how far row 3 is from what 12-real storage rebuilds.
static double su3_defect(const double* links, size_t nlinks) {
    double worst = 0.0;
    for (size_t k = 0; k < nlinks; ++k) {
        const double* u = links + k * 18;
        for (int j = 0; j < 3; ++j) {
            const int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            const double a1r = u[2 * j1], a1i = u[2 * j1 + 1], a2r = u[2 * j2], a2i = u[2 * j2 + 1];
            const double b1r = u[6 + 2 * j1], b1i = u[6 + 2 * j1 + 1];
            const double b2r = u[6 + 2 * j2], b2i = u[6 + 2 * j2 + 1];
            const double pr = a1r * b2r - a1i * b2i - (a2r * b1r - a2i * b1i);
            const double pi = a1r * b2i + a1i * b2r - (a2r * b1i + a2i * b1r);
            const double dr = u[12 + 2 * j] - pr, di = u[12 + 2 * j + 1] + pi;
            const double d = std::sqrt(dr * dr + di * di);
            if (!(d <= worst)) worst = d;   // also propagates NaN
        }
    }
    return worst;
}
constexpr double kFp64x12Defect = 1e-12;   // rebuilt row within 1e-12 of the stored one
constexpr double kFp32x12Defect = 1e-6;

rhmc_status rhmc_gauge_create(const rhmc_lattice* lat, const double* links, uint32_t flags,
                              hipStream_t stream, rhmc_gauge** out) {
    if (!lat || !links || !out) return invalid("null argument");
    *out = nullptr;
    const uint32_t known = RHMC_LINKS_FP64_18 | RHMC_LINKS_FP32_12 | RHMC_LINKS_HILO_12 |
                           RHMC_LINKS_FP64_12 | RHMC_LINKS_FP32_18;
    if (flags & ~known) return invalid("unknown link flags");
    // 12-real storage rebuilds row 3 as conj(row1 x row2), which needs det U = 1
    const double defect = su3_defect(links, (size_t)4 * lat->V);
    if (!std::isfinite(defect)) return invalid("links hold NaN or Inf");
    if (flags == 0) {
        flags = (defect <= kFp32x12Defect ? RHMC_LINKS_FP32_12 : RHMC_LINKS_FP32_18) |
                (defect <= kFp64x12Defect ? RHMC_LINKS_FP64_12 : RHMC_LINKS_FP64_18);
    }
    if ((flags & RHMC_LINKS_FP64_12) && defect > kFp64x12Defect)
        return invalid("FP64-12 links need SU(3) input to FP64 accuracy (row 3 = conj(row1 x row2))");
    if (flags & RHMC_LINKS_HILO_12) flags |= RHMC_LINKS_FP32_12;   // hi is the FP32-12 copy
    if ((flags & RHMC_LINKS_FP32_12) && defect > kFp32x12Defect)
        return invalid("12-real FP32 links need SU(3) input (row 3 = conj(row1 x row2))");
    rhmc_gauge* g = new (std::nothrow) rhmc_gauge();
    if (!g) return RHMC_ERR_OOM;
    g->lat = *lat;
    g->hilo = (flags & RHMC_LINKS_HILO_12) ? 1 : 0;
    default_hop_variants(g->hop_variant);
    hipError_t e = hipGetDevice(&g->device);
    const size_t nlinks = (size_t)4 * lat->V;
    double2* canon = nullptr;
    if (e == hipSuccess && (flags & RHMC_LINKS_FP64_18))
        e = hipMalloc(&g->u64, nlinks * 9 * sizeof(double2));
    if (e == hipSuccess && (flags & RHMC_LINKS_FP64_12))
        e = hipMalloc(&g->u64c, nlinks * 6 * sizeof(double2));
    if (e == hipSuccess && (flags & RHMC_LINKS_FP32_12))
        e = hipMalloc(&g->u32, nlinks * (g->hilo ? 6 : 3) * sizeof(float4));
    if (e == hipSuccess && (flags & RHMC_LINKS_FP32_18))
        e = hipMalloc(&g->u32f, nlinks * 9 * sizeof(float2));
    if (e == hipSuccess)
        e = hipMalloc(&g->partial, sizeof(double) * kMaxSys * (size_t)max_hop_grid((int)lat->Vh));
    if (e == hipSuccess) e = hipMalloc(&canon, nlinks * 9 * sizeof(double2));
    if (e == hipSuccess)
        e = hipMemcpyAsync(canon, links, nlinks * 9 * sizeof(double2), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = launch_pack_links(g, canon, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    hipFree(canon);
    if (e != hipSuccess) {
        set_error(std::string("rhmc_gauge_create: ") + hipGetErrorString(e));
        rhmc_gauge_destroy(g);
        return e == hipErrorOutOfMemory ? RHMC_ERR_OOM : RHMC_ERR_HIP;
    }
    *out = g;
    return RHMC_OK;
}

void rhmc_gauge_destroy(rhmc_gauge* g) {
    if (!g) return;
    hipSetDevice(g->device);
    workspace_destroy(g->ws);
    md_destroy(g->md);
    hipFree(g->u64);
    hipFree(g->u64c);
    hipFree(g->u32);
    hipFree(g->u32f);
    hipFree(g->tmp_odd);
    hipFree(g->partial);
    delete g;
}

rhmc_status rhmc_dslash_eo(const rhmc_gauge* gc, int32_t out_parity, rhmc_prec prec, int32_t nrhs,
                           const void* in, void* out, hipStream_t stream) {
    rhmc_gauge* g = const_cast<rhmc_gauge*>(gc);
    if (!g || !in || !out) return invalid("null argument");
    if (out_parity != 0 && out_parity != 1) return invalid("out_parity must be 0 or 1");
    if (nrhs < 1 || nrhs > 64) return invalid("nrhs must be in 1..64");
    if (in == out) return invalid("in and out must not overlap");
    RHMC_TRY(check_prec(g, prec));
    RHMC_TRY(use_device(g->device));
    if (prec == RHMC_PREC_FP64)
        return hop<double2>(g, out_parity, prec, nrhs, in, out, kModeD, nullptr, 0.0, stream);
    return hop<float2>(g, out_parity, prec, nrhs, in, out, kModeD, nullptr, 0.0, stream);
}

rhmc_status rhmc_apply_mdagm(const rhmc_gauge* gc, double m, rhmc_prec prec, int32_t nrhs,
                             const void* in, void* out, hipStream_t stream) {
    rhmc_gauge* g = const_cast<rhmc_gauge*>(gc);
    if (!g || !in || !out) return invalid("null argument");
    if (nrhs < 1 || nrhs > 64) return invalid("nrhs must be in 1..64");
    if (in == out) return invalid("in and out must not overlap");
    if (!std::isfinite(m)) return invalid("m must be finite");
    RHMC_TRY(check_prec(g, prec));
    RHMC_TRY(use_device(g->device));
    void* t = nullptr;
    RHMC_TRY(tmp_odd(g, vec_set_bytes(g, prec, nrhs), &t));
    if (prec == RHMC_PREC_FP64) {
        RHMC_TRY(hop<double2>(g, 1, prec, nrhs, in, t, kModeD, nullptr, 0.0, stream));
        return hop<double2>(g, 0, prec, nrhs, t, out, kModeA, in, m * m, stream);
    }
    RHMC_TRY(hop<float2>(g, 1, prec, nrhs, in, t, kModeD, nullptr, 0.0, stream));
    return hop<float2>(g, 0, prec, nrhs, t, out, kModeA, in, m * m, stream);
}

rhmc_status rhmc_apply_mdagm_static(const rhmc_gauge* gc, double m, rhmc_prec prec, int32_t nrhs,
                                    const void* in, void* out, hipStream_t stream) {
    rhmc_gauge* g = const_cast<rhmc_gauge*>(gc);
    if (!g || !in || !out) return invalid("null argument");
    if (nrhs < 1 || nrhs > 64) return invalid("nrhs must be in 1..64");
    if (in == out) return invalid("in and out must not overlap");
    if (!std::isfinite(m)) return invalid("m must be finite");
    RHMC_TRY(check_prec(g, prec));
    size_t part_bytes = 0;
    const size_t need = static_mdagm_bytes(g, prec, nrhs, &part_bytes);
    if (need > kScratchBytes)
        return invalid("rhmc_apply_mdagm_static needs " + std::to_string(need) +
                       " bytes of scratch (odd temporary and partial sums), above the " +
                       std::to_string(kScratchBytes) + " of the static array; use rhmc_apply_mdagm");
    RHMC_TRY(use_device(g->device));
    unsigned char* base = nullptr;
    RHMC_TRY(scratch_address(g->device, &base));
    double* partial = reinterpret_cast<double*>(base);
    void* t = base + part_bytes;
    // nothing in the scratch needs to start at zero: D_oe writes every site
    // of the temporary and the A launch writes every partial it owns
    if (prec == RHMC_PREC_FP64) {
        RHMC_TRY(hop<double2>(g, 1, prec, nrhs, in, t, kModeD, nullptr, 0.0, stream, partial));
        return hop<double2>(g, 0, prec, nrhs, t, out, kModeA, in, m * m, stream, partial);
    }
    RHMC_TRY(hop<float2>(g, 1, prec, nrhs, in, t, kModeD, nullptr, 0.0, stream, partial));
    return hop<float2>(g, 0, prec, nrhs, t, out, kModeA, in, m * m, stream, partial);
}

static rhmc_status check_shifts(double m, int nshift, const double* shifts) {
    if (nshift < 1 || nshift > kMaxShift) return invalid("nshift must be in 1..32");
    if (!shifts) return invalid("null shifts");
    for (int i = 0; i < nshift; ++i) {
        if (!std::isfinite(shifts[i]) || shifts[i] < 0) return invalid("shifts must be finite and >= 0");
        if (m * m + shifts[i] <= 0) return invalid("m^2 + shift must be > 0 (A + shift positive definite)");
    }
    return RHMC_OK;
}

rhmc_status rhmc_multishift_cg(const rhmc_gauge* gc, double m, int32_t nshift,
                               const double* shifts, int32_t nrhs, const void* b, void* x,
                               const rhmc_solver_params* params, rhmc_solver_stats* stats,
                               hipStream_t stream) {
    rhmc_gauge* g = const_cast<rhmc_gauge*>(gc);
    if (!g || !b || !x) return invalid("null argument");
    if (nrhs < 1 || nrhs > 64) return invalid("nrhs must be in 1..64");
    if (!std::isfinite(m)) return invalid("m must be finite");
    RHMC_TRY(check_shifts(m, nshift, shifts));
    rhmc_solver_params prm;
    RHMC_TRY(check_params(params, g, &prm));
    if (prm.two_pass) return invalid("two_pass forms no shifted solutions: use rhmc_rational_apply");
    RHMC_TRY(use_device(g->device));
    const size_t n = (size_t)3 * g->lat.Vh;
    return multishift(g, m, nshift, shifts, nrhs, reinterpret_cast<const double2*>(b),
                      reinterpret_cast<double2*>(x), (size_t)nshift * n, n, prm, stats, stream);
}

rhmc_status rhmc_rational_apply(const rhmc_gauge* gc, double m, const rhmc_rational* rat,
                                int32_t nrhs, const void* b, void* y,
                                const rhmc_solver_params* params, rhmc_solver_stats* stats,
                                hipStream_t stream) {
    rhmc_gauge* g = const_cast<rhmc_gauge*>(gc);
    if (!g || !rat || !b || !y) return invalid("null argument");
    if (b == y) return invalid("b and y must not overlap");
    if (nrhs < 1 || nrhs > 64) return invalid("nrhs must be in 1..64");
    if (!std::isfinite(m) || !std::isfinite(rat->alpha0)) return invalid("non-finite coefficient");
    if (rat->npole < 1 || !rat->alpha) return invalid("rational needs npole >= 1 and alpha");
    for (int i = 0; i < rat->npole; ++i)
        if (!std::isfinite(rat->alpha[i])) return invalid("non-finite coefficient");
    RHMC_TRY(check_shifts(m, rat->npole, rat->beta));
    rhmc_solver_params prm;
    RHMC_TRY(check_params(params, g, &prm));
    RHMC_TRY(use_device(g->device));
    if (stats) {
        stats->total_iterations = 0;
        stats->reliable_updates = 0;
        stats->refine_rounds = 0;
        stats->time_ms = 0;
        stats->max_true_residual = 0;
        stats->fp64_head_iterations = 0;
    }
    return rational(g, m, rat, nrhs, reinterpret_cast<const double2*>(b),
                    reinterpret_cast<double2*>(y), prm, stats, stream);
}

rhmc_status rhmc_pf_phi(const rhmc_gauge* gc, double m, int32_t nrhs, const void* r_even,
                        const void* r_odd, void* phi, hipStream_t stream) {
    rhmc_gauge* g = const_cast<rhmc_gauge*>(gc);
    if (!g || !r_even || !r_odd || !phi) return invalid("null argument");
    if (nrhs < 1 || nrhs > 64) return invalid("nrhs must be in 1..64");
    if (phi == r_even || phi == r_odd) return invalid("phi must not overlap R");
    if (!std::isfinite(m)) return invalid("m must be finite");
    RHMC_TRY(check_prec(g, RHMC_PREC_FP64));
    RHMC_TRY(use_device(g->device));
    // A-mode of the hopping kernel: out = c * self - D_eo in, with c = m
    return hop<double2>(g, 0, RHMC_PREC_FP64, nrhs, r_odd, phi, kModeA, r_even, m, stream);
}

rhmc_status rhmc_pf_action(const rhmc_gauge* gc, double m, const rhmc_rational* rat, int32_t nrhs,
                           const void* phi, double* S, const rhmc_solver_params* params,
                           rhmc_solver_stats* stats, hipStream_t stream) {
    rhmc_gauge* g = const_cast<rhmc_gauge*>(gc);
    if (!g || !rat || !phi || !S) return invalid("null argument");
    if (nrhs < 1 || nrhs > 64) return invalid("nrhs must be in 1..64");
    if (!std::isfinite(m) || !std::isfinite(rat->alpha0)) return invalid("non-finite coefficient");
    if (rat->npole < 1 || !rat->alpha) return invalid("rational needs npole >= 1 and alpha");
    for (int i = 0; i < rat->npole; ++i)
        if (!std::isfinite(rat->alpha[i])) return invalid("non-finite coefficient");
    RHMC_TRY(check_shifts(m, rat->npole, rat->beta));
    rhmc_solver_params prm;
    RHMC_TRY(check_params(params, g, &prm));
    RHMC_TRY(use_device(g->device));
    if (stats) {
        stats->total_iterations = 0;
        stats->reliable_updates = 0;
        stats->refine_rounds = 0;
        stats->time_ms = 0;
        stats->max_true_residual = 0;
        stats->fp64_head_iterations = 0;
    }
    return pf_action(g, m, rat, nrhs, reinterpret_cast<const double2*>(phi), S, prm, stats, stream);
}

rhmc_status rhmc_pf_force(const rhmc_gauge* gc, double m, const rhmc_rational* rat, int32_t nrhs,
                          const void* phi, void* force, const rhmc_solver_params* params,
                          rhmc_solver_stats* stats, hipStream_t stream) {
    rhmc_gauge* g = const_cast<rhmc_gauge*>(gc);
    if (!g || !rat || !phi || !force) return invalid("null argument");
    if (nrhs < 1 || nrhs > 64) return invalid("nrhs must be in 1..64");
    if (!std::isfinite(m) || !std::isfinite(rat->alpha0)) return invalid("non-finite coefficient");
    if (rat->npole < 1 || !rat->alpha) return invalid("rational needs npole >= 1 and alpha");
    for (int i = 0; i < rat->npole; ++i)
        if (!std::isfinite(rat->alpha[i])) return invalid("non-finite coefficient");
    RHMC_TRY(check_shifts(m, rat->npole, rat->beta));
    rhmc_solver_params prm;
    RHMC_TRY(check_params(params, g, &prm));
    if (prm.two_pass) return invalid("two_pass forms no shifted solutions: the force needs them");
    RHMC_TRY(use_device(g->device));
    if (stats) {
        stats->total_iterations = 0;
        stats->reliable_updates = 0;
        stats->refine_rounds = 0;
        stats->time_ms = 0;
        stats->max_true_residual = 0;
        stats->fp64_head_iterations = 0;
    }
    return pf_force(g, m, rat, nrhs, reinterpret_cast<const double2*>(phi),
                    reinterpret_cast<double2*>(force), nullptr, 0.0, prm, stats, stream);
}

rhmc_status rhmc_tune_dslash(rhmc_gauge* g, rhmc_prec prec, int32_t nrhs, const void* in,
                             void* out, hipStream_t stream) {
    if (!g || !in || !out) return invalid("null argument");
    if (nrhs < 1 || nrhs > kMaxSys) return invalid("nrhs must be in 1..8");
    if (in == out) return invalid("in and out must not overlap");
    RHMC_TRY(check_prec(g, prec));
    RHMC_TRY(use_device(g->device));
    return tune_hop(g, prec, nrhs, in, out, stream);
}

rhmc_status rhmc_dslash_variant(const rhmc_gauge* g, rhmc_prec prec, int32_t nrhs,
                                int32_t* variant) {
    if (!g || !variant) return invalid("null argument");
    if (nrhs < 1 || nrhs > 64) return invalid("nrhs must be in 1..64");
    RHMC_TRY(check_prec(g, prec));
    *variant = g->hop_variant[prec][nr_class(nrhs < kMaxSys ? nrhs : kMaxSys)];
    return RHMC_OK;
}

rhmc_status rhmc_set_dslash_variant(rhmc_gauge* g, rhmc_prec prec, int32_t nrhs,
                                    int32_t variant) {
    if (!g) return invalid("null argument");
    if (nrhs < 1 || nrhs > 64) return invalid("nrhs must be in 1..64");
    if (variant < 0 || variant >= kHopVariants) return invalid("variant must be in 0.." + std::to_string(kHopVariants - 1));
    RHMC_TRY(check_prec(g, prec));
    const int cls = nr_class(nrhs < kMaxSys ? nrhs : kMaxSys);
    g->hop_variant[prec][cls] = variant;
    g->hop_tuned[prec][cls] = 1;
    return RHMC_OK;
}

// ------------------------------------------------------------------ molecular dynamics
static rhmc_status need_fp64_links(const rhmc_gauge* g) {
    if (!has_fp64_op(g)) {
        set_error("molecular dynamics needs an FP64 link storage (FP64-12, FP64-18 or hi/lo)");
        return RHMC_ERR_UNSUPPORTED;
    }
    return RHMC_OK;
}

static rhmc_status check_rational(double m, const rhmc_rational* rat) {
    if (!rat) return invalid("null rational");
    if (!std::isfinite(m) || !std::isfinite(rat->alpha0)) return invalid("non-finite coefficient");
    if (rat->npole < 1 || !rat->alpha) return invalid("rational needs npole >= 1 and alpha");
    for (int i = 0; i < rat->npole; ++i)
        if (!std::isfinite(rat->alpha[i])) return invalid("non-finite coefficient");
    return check_shifts(m, rat->npole, rat->beta);
}

static rhmc_status check_md(const rhmc_gauge* g, const rhmc_md_params* p, rhmc_md_params* out) {
    if (!p) return invalid("null md params");
    *out = *p;
    if (!std::isfinite(p->beta) || !std::isfinite(p->mass)) return invalid("beta and mass must be finite");
    if (!std::isfinite(p->tau)) return invalid("tau must be finite");
    if (p->n_md < 1 || p->n_md > 1000000) return invalid("n_md must be in 1..1e6");
    if (p->gauge_steps < 2 || p->gauge_steps % 2 || p->gauge_steps > 100000)
        return invalid("gauge_steps must be even and in 2..1e5");
    if (!(p->lambda >= 0.0 && p->lambda <= 0.5)) return invalid("lambda must be in [0, 1/2]");
    RHMC_TRY(check_rational(p->mass, p->force_rational));
    if (p->solver.two_pass) return invalid("two_pass forms no shifted solutions: the force needs them");
    return check_params(&p->solver, g, &out->solver);
}

rhmc_status rhmc_gauge_action(const rhmc_gauge* gc, double beta, double* S, hipStream_t stream) {
    rhmc_gauge* g = const_cast<rhmc_gauge*>(gc);
    if (!g || !S) return invalid("null argument");
    if (!std::isfinite(beta)) return invalid("beta must be finite");
    RHMC_TRY(need_fp64_links(g));
    RHMC_TRY(use_device(g->device));
    return gauge_action(g, beta, S, stream);
}

rhmc_status rhmc_gauge_force_kick(const rhmc_gauge* g, double beta, double eps, double* mom,
                                  hipStream_t stream) {
    if (!g || !mom) return invalid("null argument");
    if (!std::isfinite(beta) || !std::isfinite(eps)) return invalid("beta and eps must be finite");
    RHMC_TRY(need_fp64_links(g));
    RHMC_TRY(use_device(g->device));
    RHMC_HIP_TRY(launch_gauge_force_mom(g, beta, eps, mom, stream));
    return RHMC_OK;
}

rhmc_status rhmc_pf_force_kick(const rhmc_gauge* gc, double m, const rhmc_rational* rat,
                               int32_t npf, const void* phi, double eps, double* mom,
                               const rhmc_solver_params* params, rhmc_solver_stats* stats,
                               hipStream_t stream) {
    rhmc_gauge* g = const_cast<rhmc_gauge*>(gc);
    if (!g || !phi || !mom) return invalid("null argument");
    if (npf < 1 || npf > 64) return invalid("npf must be in 1..64");
    if (!std::isfinite(eps)) return invalid("eps must be finite");
    RHMC_TRY(need_fp64_links(g));
    RHMC_TRY(check_rational(m, rat));
    rhmc_solver_params prm;
    RHMC_TRY(check_params(params, g, &prm));
    if (prm.two_pass) return invalid("two_pass forms no shifted solutions: the force needs them");
    RHMC_TRY(use_device(g->device));
    if (stats) {
        stats->total_iterations = 0;
        stats->reliable_updates = 0;
        stats->refine_rounds = 0;
        stats->time_ms = 0;
        stats->max_true_residual = 0;
        stats->fp64_head_iterations = 0;
    }
    return pf_force(g, m, rat, npf, reinterpret_cast<const double2*>(phi), nullptr, mom, eps, prm,
                    stats, stream);
}

rhmc_status rhmc_update_links(rhmc_gauge* g, double eps, const double* mom, hipStream_t stream) {
    if (!g || !mom) return invalid("null argument");
    if (!std::isfinite(eps)) return invalid("eps must be finite");
    RHMC_TRY(need_fp64_links(g));
    RHMC_TRY(use_device(g->device));
    RHMC_HIP_TRY(launch_update_links(g, eps, mom, stream));
    return RHMC_OK;
}

rhmc_status rhmc_kinetic(const rhmc_gauge* gc, const double* mom, double* K, hipStream_t stream) {
    rhmc_gauge* g = const_cast<rhmc_gauge*>(gc);
    if (!g || !mom || !K) return invalid("null argument");
    RHMC_TRY(use_device(g->device));
    return kinetic(g, mom, K, stream);
}

rhmc_status rhmc_gauge_links(const rhmc_gauge* g, void* links, hipStream_t stream) {
    if (!g || !links) return invalid("null argument");
    RHMC_TRY(need_fp64_links(g));
    RHMC_TRY(use_device(g->device));
    RHMC_HIP_TRY(launch_get_links(g, reinterpret_cast<double2*>(links), stream));
    return RHMC_OK;
}

void rhmc_md_params_default(rhmc_md_params* p) {
    if (!p) return;
    p->beta = 5.264;
    p->mass = 0.01335;
    p->tau = 1.0;
    p->n_md = 12;
    p->gauge_steps = 10;
    p->lambda = 0.1931833275037836;
    p->force_rational = nullptr;
    rhmc_solver_params_default(&p->solver);
}

rhmc_status rhmc_md_integrate(rhmc_gauge* g, const rhmc_md_params* params, int32_t npf,
                              const void* phi, double* mom, rhmc_md_stats* stats,
                              hipStream_t stream) {
    if (!g || !phi || !mom) return invalid("null argument");
    if (npf < 1 || npf > 64) return invalid("npf must be in 1..64");
    RHMC_TRY(need_fp64_links(g));
    rhmc_md_params p;
    RHMC_TRY(check_md(g, params, &p));
    RHMC_TRY(use_device(g->device));
    return md_integrate(g, p, npf, reinterpret_cast<const double2*>(phi), mom, stats, stream);
}

rhmc_status rhmc_trajectory(rhmc_gauge* g, const rhmc_hmc_params* params, int32_t npf,
                            const void* R, double* mom, double u, rhmc_trajectory_stats* stats,
                            hipStream_t stream) {
    if (!g || !params || !R || !mom || !stats) return invalid("null argument");
    if (npf < 1 || npf > 64) return invalid("npf must be in 1..64");
    if (!(u >= 0.0 && u <= 1.0)) return invalid("u must be in [0, 1]");
    RHMC_TRY(need_fp64_links(g));
    rhmc_hmc_params p = *params;
    RHMC_TRY(check_md(g, &params->md, &p.md));
    RHMC_TRY(check_rational(p.md.mass, p.heatbath_rational));
    RHMC_TRY(check_rational(p.md.mass, p.action_rational));
    RHMC_TRY(check_params(&params->metropolis_solver, g, &p.metropolis_solver));
    RHMC_TRY(use_device(g->device));
    *stats = rhmc_trajectory_stats{};
    return trajectory(g, p, npf, reinterpret_cast<const double2*>(R), mom, u, stats, stream);
}

const char* rhmc_status_string(rhmc_status s) {
    switch (s) {
        case RHMC_OK: return "ok";
        case RHMC_ERR_INVALID_ARG: return "invalid argument";
        case RHMC_ERR_NONFINITE: return "non-finite value";
        case RHMC_ERR_NOT_CONVERGED: return "not converged";
        case RHMC_ERR_HIP: return "HIP runtime error";
        case RHMC_ERR_OOM: return "out of device memory";
        case RHMC_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* rhmc_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
