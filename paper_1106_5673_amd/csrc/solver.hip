// Multi-shift CG driver (Sec. 4.3, Eq. shifted) for A = m^2 - D_eo D_oe.
//
// One CG iteration is four kernels on the caller's stream:
//   t  = D_oe p                                   (hopping, FP64 or FP32-12)
//   Ap = (m^2 + sigma_0) p - D_eo t, sum <p,Ap>   -> alpha, zeta_i, alpha_i
//   r' = r - alpha Ap, sum <r',r'>                -> beta, beta_i, convergence
//   p  = r' + beta p
// The scalar recurrences run in FP64 in the last workgroup of the reducing
// kernels, so the host only polls one flag.  The shifted solutions x_i and
// directions p_i are updated once per block of K iterations from the stored
// base residuals (state.h); a block is captured once as a hipGraph and
// replayed.  MIXED mode iterates in FP64 until every residual is below
// fp64_head ||b||, then in FP32 with 12-real links, and every
// `reliable_every` FP32 iterations replaces r by b - (A + sigma_0) x_0
// computed in FP64.  At the end every shift's true residual is recomputed in
// FP64, and a shift above tolerance gets a warm-started CG on its own system.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "blas.h"
#include "solver.h"
#include "force.h"
#include "state.h"

namespace rhmc {

using Clock = std::chrono::steady_clock;
// milliseconds since t; t moves to now
static double ms_since(Clock::time_point& t) {
    const auto now = Clock::now();
    const double d = std::chrono::duration<double, std::milli>(now - t).count();
    t = now;
    return d;
}

struct GraphKey {
    int nsys = 0, nshift = 0, K = 0, mode = -1, reliable = 0;
    const void* b[kMaxSys] = {};
    const void* x = nullptr;
    size_t x_sys = 0, x_shift = 0;
    double c[kMaxSys] = {};
    int base[kMaxSys] = {};
    int variants[2][4] = {};
    int two_pass = 0;
    const void* wacc = nullptr;
    const void* yacc = nullptr;
    size_t w_stride = 0;
    bool operator==(const GraphKey& o) const { return std::memcmp(this, &o, sizeof(*this)) == 0; }
};

constexpr int kGraphSlots = 12;

struct CachedGraph {
    GraphKey key;
    hipGraphExec_t exec = nullptr;
};

struct Workspace {
    int device = 0;
    size_t n = 0;          // complex numbers per vector (3*Vh)
    size_t vec_bytes = 0;  // bytes of one vector at FP64 width (both modes share buffers)
    // iteration vectors; they grow with the problem shape, never shrink
    void* ring = nullptr;  // [K+1][nsys] stored base residuals
    void* p = nullptr;     // [nsys]
    void* Ap = nullptr;    // [nsys]
    void* t = nullptr;     // [nsys] odd parity
    void* P = nullptr;     // [nsys][nshift] shifted directions
    size_t ring_cap = 0, p_cap = 0, Ap_cap = 0, t_cap = 0, P_cap = 0;  // bytes
    // fixed-size buffers, allocated once with the workspace
    double2* t64 = nullptr;    // [kMaxSys] odd parity, FP64
    double2* rb = nullptr;     // [kMaxSys] refinement right-hand sides
    double2* rx = nullptr;     // [kMaxSys] refinement corrections
    double* partial = nullptr;     // two regions of [kMaxSys][part_stride] block sums
    size_t part_stride = 0;
    double* sums = nullptr;        // [kMaxSys]
    SolverState* st = nullptr;     // device
    BlockCoef* coef = nullptr;     // device [kMaxSys][kMaxShift]
    SolverState* hst = nullptr;    // pinned host mirror
    int* flags_host = nullptr;     // pinned [2][2]: all_done, head_done per poll slot
    double* ratio_host = nullptr;  // pinned [2]: conv_ratio per poll slot
    double* sums_host = nullptr;   // pinned [kMaxSys]
    hipStream_t cap = nullptr;     // capture stream
    hipEvent_t ev[2] = {nullptr, nullptr};
    // rational apply: [nsys][npole] shifted solutions
    double2* xr = nullptr;
    size_t xr_cap = 0;
    // pseudofermion action: r(A) phi, [nrhs]
    double2* ya = nullptr;
    size_t ya_cap = 0;
    // pseudofermion force: D_oe x_i, [nsys][npole]
    double2* yf = nullptr;
    size_t yf_cap = 0;
    // two-pass rational apply: per-step scalars, coefficient scratch + weights
    double* hist = nullptr;
    size_t hist_cap = 0;
    double* tp = nullptr;
    size_t tp_cap = 0;
    // a MIXED call replays up to seven graphs (FP64 phase; FP32 with and
    // without replacement; the same two per refinement chunk of up to 8 systems)
    CachedGraph graphs[kGraphSlots];
    int graph_next = 0;
    // buffers replaced by grow() during a solver call, freed when the
    // outermost call returns (SolverCall)
    std::vector<void*> retired;
};

static void free_graphs(Workspace* w) {
    for (auto& g : w->graphs) {
        if (g.exec) hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
        g.key = GraphKey();
    }
}

void workspace_destroy(Workspace* w) {
    if (!w) return;
    free_graphs(w);
    for (void* p : w->retired) hipFree(p);
    for (void* p : {w->ring, w->p, w->Ap, w->t, w->P, (void*)w->t64, (void*)w->rb, (void*)w->rx,
                    (void*)w->xr, (void*)w->ya, (void*)w->yf, (void*)w->hist, (void*)w->tp,
                    (void*)w->partial, (void*)w->sums,
                    (void*)w->st, (void*)w->coef})
        hipFree(p);
    hipHostFree(w->hst);
    hipHostFree(w->flags_host);
    hipHostFree(w->ratio_host);
    hipHostFree(w->sums_host);
    if (w->cap) hipStreamDestroy(w->cap);
    for (auto& e : w->ev)
        if (e) hipEventDestroy(e);
    delete w;
}

static rhmc_status alloc(void** p, size_t bytes) {
    RHMC_HIP_TRY(hipMalloc(p, bytes));
    return RHMC_OK;
}

// Grow one buffer to at least `need` bytes.  Captured graphs hold the old
// address, so they are dropped.  The old buffer is retired, not freed: code
// of the same solver call may still hold pointers into it (or have kernels
// queued on it), so it stays allocated until the outermost call returns.
static rhmc_status grow(Workspace* w, void** buf, size_t* cap, size_t need) {
    if (*cap >= need) return RHMC_OK;
    free_graphs(w);
    if (*buf) w->retired.push_back(*buf);
    *buf = nullptr;
    *cap = 0;
    RHMC_TRY(alloc(buf, need));
    *cap = need;
    return RHMC_OK;
}

// Scope of one solver entry point (calls nest: a rational apply runs
// multi-shift solves).  When the outermost one returns, every result has
// been waited for, and the buffers grow() retired during it are freed.
struct SolverCall {
    rhmc_gauge* g;
    explicit SolverCall(rhmc_gauge* g_) : g(g_) { ++g->solver_depth; }
    ~SolverCall() {
        if (--g->solver_depth > 0 || !g->ws) return;
        for (void* p : g->ws->retired) hipFree(p);
        g->ws->retired.clear();
    }
    SolverCall(const SolverCall&) = delete;
    SolverCall& operator=(const SolverCall&) = delete;
};

// Ensure room for nsys systems x nshift shifts with blocks of K.  The
// workspace object and its fixed-size buffers are created once per gauge
// object and never freed before rhmc_gauge_destroy.
static rhmc_status ensure_workspace(rhmc_gauge* g, int nsys, int nshift, int K) {
    Workspace* w = g->ws;
    if (!w) {
        w = new Workspace();
        g->ws = w;
        w->device = g->device;
        w->n = (size_t)3 * g->lat.Vh;
        w->vec_bytes = w->n * sizeof(double2);
        const size_t vb = w->vec_bytes;
        RHMC_TRY(alloc((void**)&w->t64, vb * kMaxSys));
        RHMC_TRY(alloc((void**)&w->rb, vb * kMaxSys));
        RHMC_TRY(alloc((void**)&w->rx, vb * kMaxSys));
        w->part_stride = (size_t)max_hop_grid(g->lat.geom.Vh) + 2;
        RHMC_TRY(alloc((void**)&w->partial, sizeof(double) * 2 * kMaxSys * w->part_stride));
        RHMC_TRY(alloc((void**)&w->sums, sizeof(double) * kMaxSys));
        RHMC_TRY(alloc((void**)&w->st, sizeof(SolverState)));
        RHMC_TRY(alloc((void**)&w->coef, sizeof(BlockCoef) * kMaxSys * kMaxShift));
        RHMC_HIP_TRY(hipHostMalloc((void**)&w->hst, sizeof(SolverState), hipHostMallocDefault));
        RHMC_HIP_TRY(hipHostMalloc((void**)&w->flags_host, sizeof(int) * 4, hipHostMallocDefault));
        RHMC_HIP_TRY(hipHostMalloc((void**)&w->ratio_host, sizeof(double) * 2, hipHostMallocDefault));
        RHMC_HIP_TRY(hipHostMalloc((void**)&w->sums_host, sizeof(double) * kMaxSys, hipHostMallocDefault));
        RHMC_HIP_TRY(hipStreamCreateWithFlags(&w->cap, hipStreamNonBlocking));
        RHMC_HIP_TRY(hipEventCreateWithFlags(&w->ev[0], hipEventDisableTiming));
        RHMC_HIP_TRY(hipEventCreateWithFlags(&w->ev[1], hipEventDisableTiming));
    }
    const size_t vb = w->vec_bytes;
    RHMC_TRY(grow(w, &w->ring, &w->ring_cap, vb * (size_t)(K + 1) * nsys));
    RHMC_TRY(grow(w, &w->p, &w->p_cap, vb * nsys));
    RHMC_TRY(grow(w, &w->Ap, &w->Ap_cap, vb * nsys));
    RHMC_TRY(grow(w, &w->t, &w->t_cap, vb * nsys));
    RHMC_TRY(grow(w, &w->P, &w->P_cap, vb * (size_t)nsys * nshift));
    return RHMC_OK;
}

static rhmc_status ensure_rational_buffer(rhmc_gauge* g, size_t nvec, double2** out) {
    Workspace* w = g->ws;
    RHMC_TRY(grow(w, (void**)&w->xr, &w->xr_cap, w->vec_bytes * nvec));
    *out = w->xr;
    return RHMC_OK;
}

// ------------------------------------------------------------------ problem
struct Problem {
    int nsys, nshift;
    double m2;
    double sigma0[kMaxSys];
    double off[kMaxSys][kMaxShift];
    int base[kMaxSys];
    double tol[kMaxSys];          // relative tolerance per system
    const double2* b[kMaxSys];    // FP64 sources
    double2* X;                   // FP64 solutions
    size_t x_sys, x_shift;        // element strides
    int mode, K, reliable_blocks, maxiter;
    double head_rel;              // MIXED: FP64 iterations until ||r|| <= head_rel ||b|| (0: none)
    // two-pass rational apply: no shifted vectors (the flush only moves the
    // residual ring); the first pass records per-step scalars into hist, the
    // second adds w(k) r(k) into yacc
    bool two_pass;
    double* hist;
    int hist_cap;
    const double* wacc;
    size_t w_stride;
    double2* yacc;
    bool use_graph;
    bool tune;
    int poll_every;
};

template <typename VT>
static VT* vec(void* base, size_t n, size_t idx) {
    return reinterpret_cast<VT*>(base) + idx * n;
}

// Iteration vectors come in sets of ns systems: FP32 sets of two or more
// systems are paired (f32_offset), FP64 sets are plain [ns][n].  Both fit the
// buffers, which are sized for FP64 sets.
template <typename VT>
static bool set_paired(int ns) {
    return std::is_same<VT, float2>::value && paired_f32(ns);
}
template <typename VT>
static size_t set_len(int ns, size_t n) {
    return set_paired<VT>(ns) ? f32_set_size(ns, n) : (size_t)ns * n;
}
// system j of the set at `set`
template <typename VT>
static VT* sys_vec(void* set, size_t n, int ns, int j) {
    return reinterpret_cast<VT*>(set) + f32_offset(set_paired<VT>(ns), j, 0, n);
}
// system j of slot l of the residual ring (one set per slot)
template <typename VT>
static VT* ring_vec(void* ring, size_t n, int ns, int l, int j) {
    return sys_vec<VT>(reinterpret_cast<VT*>(ring) + (size_t)l * set_len<VT>(ns, n), n, ns, j);
}

// Enqueue one block of K iterations (+ flush, + optional reliable update).
template <typename VT>
static rhmc_status enqueue_block(const rhmc_gauge* g, Workspace* w, const Problem& pb,
                                 bool reliable, hipStream_t s) {
    const size_t n = w->n;
    const int ns = pb.nsys;
    const bool f32 = std::is_same<VT, float2>::value;

    DslashArgs<VT> d{};
    d.g = g->lat.geom;
    d.nrhs = ns;
    d.skip = &w->st->sys[0].done;
    d.skip_stride = (int)(sizeof(SysScalars) / sizeof(int));
    d.all_done = &w->st->all_done;
    d.partial = w->partial;
    DslashArgs<VT> a = d;
    d.out_par = 1;
    a.out_par = 0;
    // blocks of the A-mode launch (partials of <p, Ap>) and of the FP64
    // residual launch of a reliable update
    const int dgrid = gauge_hop_grid(g, f32 ? RHMC_PREC_FP32 : RHMC_PREC_FP64, ns);
    const int rgrid = gauge_hop_grid(g, RHMC_PREC_FP64, ns);
    const int vgrid = vec_blocks(n);
    const bool pr = set_paired<VT>(ns);
    d.paired = a.paired = pr;
    for (int j = 0; j < ns; ++j) {
        d.in[j] = sys_vec<VT>(w->p, n, ns, j);
        d.out[j] = sys_vec<VT>(w->t, n, ns, j);
        a.in[j] = sys_vec<VT>(w->t, n, ns, j);
        a.self[j] = sys_vec<VT>(w->p, n, ns, j);
        a.out[j] = sys_vec<VT>(w->Ap, n, ns, j);
        a.c[j] = pb.m2 + pb.sigma0[j];
    }
    set_variant(d, g);
    set_variant(a, g);
    for (int q = 0; q < pb.K; ++q) {
        if constexpr (std::is_same<VT, float2>::value) {
            RHMC_HIP_TRY(launch_fp32_op(g, d, kModeD, s));
            RHMC_HIP_TRY(launch_fp32_op(g, a, kModeA, s));
        } else {
            RHMC_HIP_TRY(launch_fp64_op(g, d, kModeD, s));
            RHMC_HIP_TRY(launch_fp64_op(g, a, kModeA, s));
        }
        // r' = r - alpha A p (alpha from the A-kernel sums) and its block sums
        double* partR = w->partial + kMaxSys * w->part_stride;
        VecArgs<VT> r{};
        r.state = w->st;
        r.n = n;
        r.partial = partR;
        r.nblk = vgrid;
        r.part2 = w->partial;
        r.nblk2 = dgrid;
        r.q = q;
        r.paired = pr;
        for (int j = 0; j < ns; ++j) {
            r.x[j] = ring_vec<VT>(w->ring, n, ns, q, j);
            r.y[j] = sys_vec<VT>(w->Ap, n, ns, j);
            r.z[j] = ring_vec<VT>(w->ring, n, ns, q + 1, j);
        }
        RHMC_HIP_TRY(launch_rupdate<VT>(r, ns, s));
        // p = r' + beta p, and the FP64 recurrences of this step
        VecArgs<VT> p = r;
        for (int j = 0; j < ns; ++j) {
            p.x[j] = ring_vec<VT>(w->ring, n, ns, q + 1, j);
            p.y[j] = sys_vec<VT>(w->p, n, ns, j);
            p.z[j] = nullptr;
        }
        RHMC_HIP_TRY(launch_pupdate<VT>(p, ns, s));
    }
    FlushArgs<VT> f{};
    f.state = w->st;
    f.coef = w->coef;
    f.n = n;
    f.nshift = pb.two_pass ? 0 : pb.nshift;
    f.nsys = ns;
    f.w = pb.wacc;
    f.w_stride = pb.w_stride;
    f.y = pb.yacc;
    f.ring = reinterpret_cast<VT*>(w->ring);
    f.ring_slot = set_len<VT>(ns, n);
    f.paired = pr;
    f.P = reinterpret_cast<double2*>(w->P);
    f.X = pb.X;
    f.x_sys = pb.x_sys;
    f.x_shift = pb.x_shift;
    RHMC_HIP_TRY(launch_flush<VT>(f, ns, pb.K, s));

    if (reliable) {
        // r = b - (m^2 + sigma_0) x_0 + D_eo D_oe x_0 in FP64, stored into r(k0)
        DslashArgs<double2> d64{};
        d64.g = g->lat.geom;
        d64.nrhs = ns;
        d64.skip = d.skip;
        d64.skip_stride = d.skip_stride;
        d64.all_done = d.all_done;
        d64.out_par = 1;
        DslashArgs<double2> r64 = d64;
        r64.out_par = 0;
        r64.partial = w->partial;
        for (int j = 0; j < ns; ++j) {
            const double2* x0 = pb.X + j * pb.x_sys + pb.base[j] * pb.x_shift;
            d64.in[j] = x0;
            d64.out[j] = w->t64 + (size_t)j * n;
            r64.in[j] = w->t64 + (size_t)j * n;
            r64.self[j] = x0;
            r64.rhs[j] = pb.b[j];
            r64.c[j] = pb.m2 + pb.sigma0[j];
            r64.out[j] = nullptr;
            if (f32) r64.out32[j] = reinterpret_cast<float2*>(ring_vec<VT>(w->ring, n, ns, 0, j));
        }
        r64.out32_paired = f32 && pr;
        if (!f32)
            for (int j = 0; j < ns; ++j) r64.out[j] = reinterpret_cast<double2*>(ring_vec<VT>(w->ring, n, ns, 0, j));
        set_variant(d64, g);
        set_variant(r64, g);
        RHMC_HIP_TRY(launch_fp64_op(g, d64, kModeD, s));
        RHMC_HIP_TRY(launch_fp64_op(g, r64, kModeResid, s));
        RHMC_HIP_TRY(launch_finalize(kFinReliable, w->st, w->partial, rgrid, ns, nullptr, s));
        if (f32) {
            // <r, p> with the replaced r: alpha of the next step (state.h)
            Dot32Args dp{};
            dp.n = n;
            dp.partial = w->partial + kMaxSys * w->part_stride;
            dp.paired = pr;
            for (int j = 0; j < ns; ++j) {
                dp.a[j] = reinterpret_cast<const float2*>(ring_vec<VT>(w->ring, n, ns, 0, j));
                dp.b[j] = reinterpret_cast<const float2*>(sys_vec<VT>(w->p, n, ns, j));
            }
            RHMC_HIP_TRY(launch_dot32(dp, ns, s));
            RHMC_HIP_TRY(launch_finalize(kFinReliableDot, w->st, dp.partial, vgrid, ns, nullptr, s));
        }
    }
    return RHMC_OK;
}

template <typename VT>
static rhmc_status get_graph(rhmc_gauge* g, Workspace* w, const Problem& pb, bool reliable,
                             hipGraphExec_t* out) {
    GraphKey k;
    std::memset(static_cast<void*>(&k), 0, sizeof(k));
    k.nsys = pb.nsys;
    k.nshift = pb.nshift;
    k.K = pb.K;
    k.mode = pb.mode;
    k.reliable = reliable;
    for (int j = 0; j < pb.nsys; ++j) {
        k.b[j] = pb.b[j];
        k.c[j] = pb.m2 + pb.sigma0[j];
        k.base[j] = pb.base[j];
    }
    std::memcpy(k.variants, g->hop_variant, sizeof(k.variants));
    k.x = pb.X;
    k.x_sys = pb.x_sys;
    k.x_shift = pb.x_shift;
    k.two_pass = pb.two_pass;
    k.wacc = pb.wacc;
    k.yacc = pb.yacc;
    k.w_stride = pb.w_stride;
    for (auto& cg : w->graphs)
        if (cg.exec && cg.key == k) {
            *out = cg.exec;
            return RHMC_OK;
        }
    CachedGraph& slot = w->graphs[w->graph_next];
    w->graph_next = (w->graph_next + 1) % kGraphSlots;
    if (slot.exec) hipGraphExecDestroy(slot.exec);
    slot.exec = nullptr;
    hipGraph_t graph = nullptr;
    RHMC_HIP_TRY(hipStreamBeginCapture(w->cap, hipStreamCaptureModeThreadLocal));
    rhmc_status st = enqueue_block<VT>(g, w, pb, reliable, w->cap);
    hipError_t e = hipStreamEndCapture(w->cap, &graph);
    if (st != RHMC_OK) {
        if (graph) hipGraphDestroy(graph);
        return st;
    }
    RHMC_HIP_TRY(e);
    e = hipGraphInstantiate(&slot.exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    RHMC_HIP_TRY(e);
    slot.key = k;
    *out = slot.exec;
    return RHMC_OK;
}

// Scalar state and r = p = b for a new shared solve whose first blocks
// iterate in VT.
template <typename VT>
static rhmc_status krylov_init(rhmc_gauge* g, const Problem& pb, hipStream_t s) {
    RHMC_TRY(ensure_workspace(g, pb.nsys, pb.nshift, pb.K));
    Workspace* w = g->ws;
    const size_t n = w->n;
    SolverState* h = w->hst;
    std::memset(h, 0, sizeof(SolverState));
    h->nsys = pb.nsys;
    h->nshift = pb.nshift;
    h->first_block = 1;
    h->maxiter = pb.maxiter;
    h->coef = w->coef;
    h->hist = pb.hist;
    h->hist_cap = pb.hist_cap;
    for (int j = 0; j < pb.nsys; ++j) {
        h->sys[j].tolb = pb.tol[j];
        h->sys[j].head_rr = pb.head_rel;
        h->sys[j].base = pb.base[j];
        for (int i = 0; i < pb.nshift; ++i) {
            ShiftScalars& q = h->sh[j][i];
            q.off = pb.off[j][i];
            q.zeta = q.zeta_prev = 1.0;
            q.active = q.block_active = 1;
        }
    }
    RHMC_HIP_TRY(hipMemcpyAsync(w->st, h, sizeof(SolverState), hipMemcpyHostToDevice, s));
    VecArgs<VT> st{};
    st.state = w->st;
    st.n = n;
    st.partial = w->partial;
    st.paired = set_paired<VT>(pb.nsys);
    for (int j = 0; j < pb.nsys; ++j) {
        st.b64[j] = pb.b[j];
        st.x[j] = ring_vec<VT>(w->ring, n, pb.nsys, 0, j);
        st.y[j] = sys_vec<VT>(w->p, n, pb.nsys, j);
    }
    RHMC_HIP_TRY(launch_start<VT>(st, pb.nsys, s));
    RHMC_HIP_TRY(launch_finalize(kFinInit, w->st, w->partial, vec_blocks(n), pb.nsys, nullptr, s));
    RHMC_HIP_TRY(hipMemcpyAsync(h, w->st, sizeof(SolverState), hipMemcpyDeviceToHost, s));
    RHMC_HIP_TRY(hipStreamSynchronize(s));
    for (int j = 0; j < pb.nsys; ++j) {
        const double bn = h->sys[j].bnorm;
        if (!std::isfinite(bn)) {
            set_error("source holds NaN or Inf");
            return RHMC_ERR_NONFINITE;
        }
        if (bn == 0.0 && pb.X)
            for (int i = 0; i < pb.nshift; ++i)
                RHMC_HIP_TRY(hipMemsetAsync(pb.X + j * pb.x_sys + i * pb.x_shift, 0,
                                            n * sizeof(double2), s));
    }
    return RHMC_OK;
}

// Replay blocks of K iterations in VT until every system is done or, with
// `head`, until every system is done or below its head threshold; at most
// enough blocks for the iterations maxiter leaves.  The host mirror holds the
// final state on return.
template <typename VT>
static rhmc_status krylov_loop(rhmc_gauge* g, const Problem& pb, bool head, hipStream_t s) {
    Workspace* w = g->ws;
    SolverState* h = w->hst;
    if (pb.tune) {
        const rhmc_prec pr = std::is_same<VT, float2>::value ? RHMC_PREC_FP32 : RHMC_PREC_FP64;
        if (!g->hop_tuned[pr][nr_class(pb.nsys)])
            RHMC_TRY(tune_hop(g, pr, pb.nsys, w->p, w->t, s));
    }
    hipGraphExec_t gb = nullptr, gr = nullptr;
    if (pb.use_graph) {
        RHMC_TRY(get_graph<VT>(g, w, pb, false, &gb));
        if (pb.mode == RHMC_MODE_MIXED) RHMC_TRY(get_graph<VT>(g, w, pb, true, &gr));
    }
    const int left = std::max(0, pb.maxiter - h->iter);
    const int max_blocks = (left + pb.K - 1) / pb.K + 1;
    int launched = 0;
    bool done = h->all_done != 0 || (head && h->head_done != 0);
    int pending = -1;         // poll slot whose flag copy is in flight
    double prev_ratio = -1.0; // conv_ratio at the previous poll read
    while (!done && launched < max_blocks) {
        const bool rel = pb.mode == RHMC_MODE_MIXED && ((launched + 1) % pb.reliable_blocks == 0);
        if (pb.use_graph) {
            RHMC_HIP_TRY(hipGraphLaunch(rel ? gr : gb, s));
        } else {
            RHMC_TRY(enqueue_block<VT>(g, w, pb, rel, s));
        }
        ++launched;
        if (launched % pb.poll_every == 0 || launched == max_blocks) {
            // all_done and head_done are adjacent in SolverState
            const int slot = (launched / pb.poll_every) & 1;
            RHMC_HIP_TRY(hipMemcpyAsync(&w->flags_host[2 * slot], &w->st->all_done,
                                        2 * sizeof(int), hipMemcpyDeviceToHost, s));
            RHMC_HIP_TRY(hipMemcpyAsync(&w->ratio_host[slot], &w->st->conv_ratio, sizeof(double),
                                        hipMemcpyDeviceToHost, s));
            RHMC_HIP_TRY(hipEventRecord(w->ev[slot], s));
            if (pending >= 0) {
                RHMC_HIP_TRY(hipEventSynchronize(w->ev[pending]));
                done = w->flags_host[2 * pending] != 0 ||
                       (head && w->flags_host[2 * pending + 1] != 0);
                const double ratio = w->ratio_host[pending];
                // With the residual falling by f per poll interval, the blocks
                // in flight reach tolerance when ratio * f <= 1: wait for them
                // rather than queue another block that would only early-exit.
                if (!done && !head && prev_ratio > 0.0 && ratio < prev_ratio &&
                    ratio * (ratio / prev_ratio) <= 1.0) {
                    RHMC_HIP_TRY(hipEventSynchronize(w->ev[slot]));
                    done = w->flags_host[2 * slot] != 0;
                    prev_ratio = w->ratio_host[slot];
                    pending = -1;
                    continue;
                }
                prev_ratio = ratio;
            }
            pending = slot;
        }
    }
    RHMC_HIP_TRY(hipMemcpyAsync(h, w->st, sizeof(SolverState), hipMemcpyDeviceToHost, s));
    RHMC_HIP_TRY(hipStreamSynchronize(s));
    return RHMC_OK;
}

// Shared Krylov solve in one precision; X receives every shifted solution.
template <typename VT>
static rhmc_status run_krylov(rhmc_gauge* g, const Problem& pb, hipStream_t s, int* iters_out,
                              int* reliable_out) {
    RHMC_TRY(krylov_init<VT>(g, pb, s));
    RHMC_TRY(krylov_loop<VT>(g, pb, false, s));
    *iters_out = g->ws->hst->iter;
    *reliable_out = g->ws->hst->reliable_count;
    return RHMC_OK;
}

// MIXED shared solve.  A shifted solution is never restarted, so the FP32
// rounding of the operator and of r made while ||r|| is still large stays in
// it (the reliable updates repair only the base system): with head_rel > 0
// the solve iterates in FP64 until every system has ||r|| <= head_rel ||b||,
// then rounds r and p to FP32 at that block boundary and goes on in FP32 with
// reliable updates from the same scalar state.  The first FP32 step takes the
// exact line search, as after a residual replacement.
static rhmc_status run_mixed(rhmc_gauge* g, const Problem& pb, hipStream_t s, int* iters_out,
                             int* reliable_out, int* head_out, double* head_ms) {
    *head_out = 0;
    *head_ms = 0.0;
    if (!(pb.head_rel > 0.0)) return run_krylov<float2>(g, pb, s, iters_out, reliable_out);
    auto th = Clock::now();
    Problem ph = pb;
    ph.mode = RHMC_MODE_FP64;
    RHMC_TRY(krylov_init<double2>(g, ph, s));
    RHMC_TRY(krylov_loop<double2>(g, ph, true, s));   // ends synchronised
    *head_ms = ms_since(th);
    Workspace* w = g->ws;
    const SolverState* h = w->hst;
    *head_out = h->iter;
    if (!h->all_done) {
        // r (ring slot j) and p to FP32, through the Ap and t buffers
        const size_t n = w->n;
        const int ns = pb.nsys;
        const bool pr = set_paired<float2>(ns);
        NarrowArgs nr{}, np{};
        nr.n = np.n = n;
        nr.paired = np.paired = pr;
        for (int j = 0; j < ns; ++j) {
            nr.x[j] = vec<double2>(w->ring, n, j);
            nr.y[j] = sys_vec<float2>(w->Ap, n, ns, j);
            np.x[j] = vec<double2>(w->p, n, j);
            np.y[j] = sys_vec<float2>(w->t, n, ns, j);
        }
        RHMC_HIP_TRY(launch_narrow(nr, ns, s));
        RHMC_HIP_TRY(launch_narrow(np, ns, s));
        const size_t set_bytes = set_len<float2>(ns, n) * sizeof(float2);
        RHMC_HIP_TRY(hipMemcpyAsync(w->ring, w->Ap, set_bytes, hipMemcpyDeviceToDevice, s));
        RHMC_HIP_TRY(hipMemcpyAsync(w->p, w->t, set_bytes, hipMemcpyDeviceToDevice, s));
        Dot32Args dp{};
        dp.n = n;
        dp.partial = w->partial + kMaxSys * w->part_stride;
        dp.paired = pr;
        for (int j = 0; j < ns; ++j) {
            dp.a[j] = ring_vec<float2>(w->ring, n, ns, 0, j);
            dp.b[j] = sys_vec<float2>(w->p, n, ns, j);
        }
        RHMC_HIP_TRY(launch_dot32(dp, ns, s));
        RHMC_HIP_TRY(launch_finalize(kFinReliableDot, w->st, dp.partial, vec_blocks(n), ns,
                                     nullptr, s));
        RHMC_TRY(krylov_loop<float2>(g, pb, false, s));
    }
    *iters_out = h->iter;
    *reliable_out = h->reliable_count;
    return RHMC_OK;
}

// FP64 true residuals ||b_j - (A + sigma_ji) x_ji||^2 for a list of (j, i);
// optionally stores the residual vectors (at most kMaxSys per call).
static rhmc_status true_residuals(rhmc_gauge* g, const Problem& pb, const std::vector<int>& list,
                                  double* out2, double2* store, hipStream_t s) {
    Workspace* w = g->ws;
    const size_t n = w->n;
    for (size_t c0 = 0; c0 < list.size(); c0 += kMaxSys) {
        const int cnt = (int)std::min<size_t>(kMaxSys, list.size() - c0);
        DslashArgs<double2> d{};
        d.g = g->lat.geom;
        d.nrhs = cnt;
        d.out_par = 1;
        DslashArgs<double2> r = d;
        r.out_par = 0;
        r.partial = w->partial;
        for (int k = 0; k < cnt; ++k) {
            const int p = list[c0 + k];
            const int j = p / pb.nshift, i = p % pb.nshift;
            const double2* x = pb.X + j * pb.x_sys + i * pb.x_shift;
            d.in[k] = x;
            d.out[k] = w->t64 + (size_t)k * n;
            r.in[k] = w->t64 + (size_t)k * n;
            r.self[k] = x;
            r.rhs[k] = pb.b[j];
            r.c[k] = pb.m2 + pb.sigma0[j] + pb.off[j][i];
            r.out[k] = store ? store + (size_t)k * n : nullptr;
        }
        set_variant(d, g);
        set_variant(r, g);
        RHMC_HIP_TRY(launch_fp64_op(g, d, kModeD, s));
        RHMC_HIP_TRY(launch_fp64_op(g, r, kModeResid, s));
        RHMC_HIP_TRY(launch_finalize(kFinNorms, nullptr, w->partial, gauge_hop_grid(g, RHMC_PREC_FP64, cnt), cnt,
                                     w->sums, s));
        RHMC_HIP_TRY(hipMemcpyAsync(w->sums_host, w->sums, sizeof(double) * cnt,
                                    hipMemcpyDeviceToHost, s));
        RHMC_HIP_TRY(hipStreamSynchronize(s));
        for (int k = 0; k < cnt; ++k) out2[c0 + k] = w->sums_host[k];
    }
    return RHMC_OK;
}

// The shared Krylov solve stops each shift at kKrylovMargin * tol of its
// recurrence residual, so that the FP64 true residual (which differs from it
// by rounding) still meets tol without a refinement round; a refinement
// solve aims at kRefineMargin * tol for the same reason.
constexpr double kKrylovMargin = 0.9;
constexpr double kRefineMargin = 0.8;

// Relative residual at which a MIXED shared solve leaves FP64 (0: no FP64
// phase).  Automatic: min(1, 1e3 sqrt(tol)), i.e. 1e-2 for tol 1e-10, where
// the FP32 rounding made after the switch keeps every shift within tol
// without refinement on rough fields at small mass; no FP64 phase for
// tol >= 1e-6.
static double mixed_head(const rhmc_solver_params& prm) {
    if (prm.mode != RHMC_MODE_MIXED || prm.per_shift) return 0.0;
    const double h = prm.fp64_head == 0.0 ? std::min(1.0, 1e3 * std::sqrt(prm.tol)) : prm.fp64_head;
    return (h > 0.0 && h < 1.0) ? h : 0.0;
}

static rhmc_status solve_impl(rhmc_gauge* g, Problem pb, const rhmc_solver_params& prm,
                              rhmc_solver_stats* stats, hipStream_t s) {
    const auto t0 = Clock::now();
    auto tp = t0;   // end of the previous phase
    double head_ms = 0.0, krylov_ms = 0.0, check_ms = 0.0, refine_ms = 0.0;
    int iters = 0, rel = 0, head = 0;
    const bool per_shift = prm.per_shift != 0;
    const int total = pb.nsys * pb.nshift;
    std::vector<int> conv(total), refine_it(total, 0);
    double bnorm[kMaxSys];
    std::vector<double> res(total), res2(total);
    if (!per_shift) {
        if (pb.mode == RHMC_MODE_MIXED)
            RHMC_TRY(run_mixed(g, pb, s, &iters, &rel, &head, &head_ms));
        else
            RHMC_TRY(run_krylov<double2>(g, pb, s, &iters, &rel));
        krylov_ms = ms_since(tp) - head_ms;
        const SolverState hs = *g->ws->hst;
        for (int j = 0; j < pb.nsys; ++j)
            for (int i = 0; i < pb.nshift; ++i) {
                const ShiftScalars& q = hs.sh[j][i];
                conv[j * pb.nshift + i] = q.active ? hs.sys[j].iters : q.conv_iter;
            }
        for (int j = 0; j < pb.nsys; ++j) bnorm[j] = hs.sys[j].bnorm;
        std::vector<int> all(total);
        for (int p = 0; p < total; ++p) all[p] = p;
        RHMC_TRY(true_residuals(g, pb, all, res2.data(), nullptr, s));
        for (int p = 0; p < total; ++p) {
            const int j = p / pb.nshift;
            res[p] = bnorm[j] > 0 ? std::sqrt(res2[p]) / bnorm[j] : 0.0;
        }
        check_ms += ms_since(tp);
    } else {
        // every shifted system from a zero start: the residual is b, and the
        // batched per-shift CG below (the refinement loop) solves each system
        RHMC_TRY(ensure_workspace(g, pb.nsys, pb.nshift, pb.K));
        Workspace* ws = g->ws;
        DotArgs d{};
        d.n = ws->n;
        d.partial = ws->partial;
        for (int j = 0; j < pb.nsys; ++j) d.a[j] = d.b[j] = pb.b[j];
        RHMC_HIP_TRY(launch_dot(d, pb.nsys, s));
        RHMC_HIP_TRY(launch_finalize(kFinNorms, nullptr, ws->partial, vec_blocks(ws->n), pb.nsys,
                                     ws->sums, s));
        RHMC_HIP_TRY(hipMemcpyAsync(ws->sums_host, ws->sums, sizeof(double) * pb.nsys,
                                    hipMemcpyDeviceToHost, s));
        for (int j = 0; j < pb.nsys; ++j)
            for (int i = 0; i < pb.nshift; ++i)
                RHMC_HIP_TRY(hipMemsetAsync(pb.X + j * pb.x_sys + i * pb.x_shift, 0,
                                            ws->n * sizeof(double2), s));
        RHMC_HIP_TRY(hipStreamSynchronize(s));
        for (int j = 0; j < pb.nsys; ++j) {
            bnorm[j] = std::sqrt(ws->sums_host[j]);
            if (!std::isfinite(bnorm[j])) {
                set_error("source holds NaN or Inf");
                return RHMC_ERR_NONFINITE;
            }
        }
        for (int p = 0; p < total; ++p) res[p] = bnorm[p / pb.nshift] > 0 ? 1.0 : 0.0;
    }
    Workspace* w = g->ws;

    int rounds = 0;
    const double tol = prm.tol;
    const int max_rounds = prm.refine ? 4 : (per_shift ? 1 : 0);
    while (rounds < max_rounds) {
        std::vector<int> bad;
        for (int p = 0; p < total; ++p)
            if (!(res[p] <= tol)) bad.push_back(p);
        if (bad.empty()) break;
        ++rounds;
        // batch systems of similar shift: they need similar iteration counts
        std::stable_sort(bad.begin(), bad.end(), [&](int p, int q) {
            return pb.sigma0[p / pb.nshift] + pb.off[p / pb.nshift][p % pb.nshift] <
                   pb.sigma0[q / pb.nshift] + pb.off[q / pb.nshift][q % pb.nshift];
        });
        for (size_t c0 = 0; c0 < bad.size(); c0 += kMaxSys) {
            const int cnt = (int)std::min<size_t>(kMaxSys, bad.size() - c0);
            std::vector<int> chunk(bad.begin() + c0, bad.begin() + c0 + cnt);
            std::vector<double> r2(cnt);
            RHMC_TRY(true_residuals(g, pb, chunk, r2.data(), w->rb, s));
            Problem rp = pb;
            rp.nsys = cnt;
            rp.nshift = 1;
            rp.X = w->rx;
            rp.x_sys = w->n;
            rp.x_shift = 0;
            rp.head_rel = 0.0;   // one system per shift: reliable updates suffice
            for (int k = 0; k < cnt; ++k) {
                const int p = chunk[k];
                const int j = p / pb.nshift, i = p % pb.nshift;
                rp.sigma0[k] = pb.sigma0[j] + pb.off[j][i];
                rp.off[k][0] = 0.0;
                rp.base[k] = 0;
                rp.b[k] = w->rb + (size_t)k * w->n;
                const double rn = std::sqrt(r2[k]);
                rp.tol[k] = rn > 0 ? std::min(0.5, kRefineMargin * tol * bnorm[j] / rn) : 0.5;
            }
            int it2 = 0, rel2 = 0;
            if (pb.mode == RHMC_MODE_MIXED)
                RHMC_TRY(run_krylov<float2>(g, rp, s, &it2, &rel2));
            else
                RHMC_TRY(run_krylov<double2>(g, rp, s, &it2, &rel2));
            rel += rel2;
            AddArgs ad{};
            ad.n = w->n;
            for (int k = 0; k < cnt; ++k) {
                const int p = chunk[k];
                const int j = p / pb.nshift, i = p % pb.nshift;
                ad.x[k] = w->rx + (size_t)k * w->n;
                ad.y[k] = pb.X + j * pb.x_sys + i * pb.x_shift;
                refine_it[p] += w->hst->sys[k].iters;
            }
            RHMC_HIP_TRY(launch_add(ad, cnt, s));
        }
        RHMC_HIP_TRY(hipStreamSynchronize(s));
        refine_ms += ms_since(tp);
        RHMC_TRY(true_residuals(g, pb, bad, res2.data(), nullptr, s));
        for (size_t k = 0; k < bad.size(); ++k) {
            const int p = bad[k];
            const int j = p / pb.nshift;
            res[p] = bnorm[j] > 0 ? std::sqrt(res2[k]) / bnorm[j] : 0.0;
        }
        check_ms += ms_since(tp);
    }
    RHMC_HIP_TRY(hipStreamSynchronize(s));
    const auto t1 = Clock::now();

    double worst = 0.0;
    bool ok = true;
    for (int p = 0; p < total; ++p) {
        worst = std::max(worst, res[p]);
        if (!(res[p] <= tol)) ok = false;
    }
    if (per_shift) {
        // each system's own iterations; the shared count is the largest
        for (int p = 0; p < total; ++p) {
            conv[p] = refine_it[p];
            iters = std::max(iters, refine_it[p]);
        }
    }
    if (stats) {
        for (int p = 0; p < total; ++p) {
            if (stats->iterations) stats->iterations[p] = conv[p];
            if (stats->true_residual) stats->true_residual[p] = res[p];
            if (stats->refine_iterations) stats->refine_iterations[p] = refine_it[p];
        }
        stats->total_iterations = iters;
        stats->reliable_updates = rel;
        stats->refine_rounds = rounds;
        stats->fp64_head_iterations = head;
        stats->time_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        stats->max_true_residual = worst;
        stats->head_ms = head_ms;
        stats->krylov_ms = krylov_ms;
        stats->check_ms = check_ms;
        stats->refine_ms = refine_ms;
    }
    for (int p = 0; p < total; ++p)
        if (!std::isfinite(res[p])) {
            set_error("solution is not finite");
            return RHMC_ERR_NONFINITE;
        }
    if (!ok) {
        set_error("some shift did not reach the requested tolerance");
        return RHMC_ERR_NOT_CONVERGED;
    }
    return RHMC_OK;
}

// Iterations per block.  A residual replacement (MIXED) needs the shifted
// solutions flushed, i.e. a block boundary, so in MIXED mode the block length
// is the divisor of reliable_every nearest to the requested one (at most
// kMaxBlockLen, at least half the request): the replacements then fall exactly
// every reliable_every iterations (50 -> blocks of 25 for the default 32).
// Without such a divisor the request is kept and the cadence rounds up.
static int block_length(const rhmc_solver_params& prm) {
    const int want = std::max(1, std::min(kMaxBlockLen, prm.block));
    if (prm.mode != RHMC_MODE_MIXED || prm.reliable_every <= 0) return want;
    int best = 0;
    for (int d = std::max(1, want / 2); d <= kMaxBlockLen; ++d) {
        if (prm.reliable_every % d) continue;
        if (!best || std::abs(d - want) < std::abs(best - want) ||
            (std::abs(d - want) == std::abs(best - want) && d > best))
            best = d;
    }
    return best ? best : want;
}

// The shared solve of nrhs <= kMaxSys right-hand sides b[j] (stride n) for
// the shifts, from the Krylov space of the smallest one.
static Problem make_problem(const rhmc_gauge* g, double m, int nshift, const double* shifts,
                            int nrhs, const double2* b, double2* x, size_t x_sys, size_t x_shift,
                            const rhmc_solver_params& prm) {
    const size_t n = (size_t)3 * g->lat.Vh;
    double smin = shifts[0];
    int base = 0;
    for (int i = 1; i < nshift; ++i)
        if (shifts[i] < smin) {
            smin = shifts[i];
            base = i;
        }
    const int K = block_length(prm);
    Problem pb{};
    pb.nsys = nrhs;
    pb.nshift = nshift;
    pb.m2 = m * m;
    for (int j = 0; j < nrhs; ++j) {
        pb.sigma0[j] = smin;
        pb.base[j] = base;
        pb.tol[j] = kKrylovMargin * prm.tol;
        pb.b[j] = b + (size_t)j * n;
        for (int i = 0; i < nshift; ++i) pb.off[j][i] = shifts[i] - smin;
    }
    pb.X = x;
    pb.x_sys = x_sys;
    pb.x_shift = x_shift;
    pb.mode = prm.mode;
    pb.K = K;
    pb.reliable_blocks = std::max(1, (prm.reliable_every + K - 1) / K);   // exact when K divides it
    pb.maxiter = prm.maxiter;
    pb.head_rel = mixed_head(prm);
    pb.use_graph = prm.use_graph != 0;
    pb.tune = prm.tune != 0;
    pb.poll_every = prm.poll_every > 0 ? prm.poll_every : 1;
    return pb;
}

rhmc_status multishift(rhmc_gauge* g, double m, int nshift, const double* shifts, int nrhs,
                       const double2* b, double2* x, size_t x_sys, size_t x_shift,
                       const rhmc_solver_params& prm, rhmc_solver_stats* stats, hipStream_t s) {
    SolverCall scope(g);
    const size_t n = (size_t)3 * g->lat.Vh;
    rhmc_solver_stats acc{};
    // process the right-hand sides in groups of kMaxSys; a group that ends
    // NOT_CONVERGED keeps its last iterates and the later groups are still
    // solved, so every output and every stat is written (worst status returned)
    rhmc_status worst = RHMC_OK;
    for (int r0 = 0; r0 < nrhs; r0 += kMaxSys) {
        const int cnt = std::min(kMaxSys, nrhs - r0);
        const Problem pb = make_problem(g, m, nshift, shifts, cnt, b + (size_t)r0 * n,
                                        x + (size_t)r0 * x_sys, x_sys, x_shift, prm);
        rhmc_solver_stats st{};
        if (stats) {
            st.iterations = stats->iterations ? stats->iterations + (size_t)r0 * nshift : nullptr;
            st.true_residual = stats->true_residual ? stats->true_residual + (size_t)r0 * nshift : nullptr;
            st.refine_iterations =
                stats->refine_iterations ? stats->refine_iterations + (size_t)r0 * nshift : nullptr;
        }
        const rhmc_status rs = solve_impl(g, pb, prm, &st, s);
        acc.total_iterations = std::max(acc.total_iterations, st.total_iterations);
        acc.reliable_updates += st.reliable_updates;
        acc.refine_rounds = std::max(acc.refine_rounds, st.refine_rounds);
        acc.fp64_head_iterations = std::max(acc.fp64_head_iterations, st.fp64_head_iterations);
        acc.time_ms += st.time_ms;
        acc.max_true_residual = std::max(acc.max_true_residual, st.max_true_residual);
        acc.head_ms += st.head_ms;
        acc.krylov_ms += st.krylov_ms;
        acc.check_ms += st.check_ms;
        acc.refine_ms += st.refine_ms;
        if (stats) {
            stats->head_ms = acc.head_ms;
            stats->krylov_ms = acc.krylov_ms;
            stats->check_ms = acc.check_ms;
            stats->refine_ms = acc.refine_ms;
            stats->total_iterations = acc.total_iterations;
            stats->reliable_updates = acc.reliable_updates;
            stats->refine_rounds = acc.refine_rounds;
            stats->fp64_head_iterations = acc.fp64_head_iterations;
            stats->time_ms = acc.time_ms;
            stats->max_true_residual = acc.max_true_residual;
        }
        if (rs == RHMC_ERR_NOT_CONVERGED)
            worst = rs;
        else if (rs != RHMC_OK)
            return rs;
    }
    if (worst != RHMC_OK) set_error("some shift did not reach the requested tolerance");
    return worst;
}

// Two-pass rational apply (FP64), a variant of the shared Krylov solve of
// Sec. 4.3 that the paper does not describe: y = alpha0 b + sum_i alpha_i x_i
// (Eq. system_r) with no x_i formed.
// Pass 1 runs the shared Krylov solve with no shifted vectors and records
// every step's alpha and beta; with x_i = sum_k c_i(k) r(k) the weights
// w(k) = sum_i alpha_i c_i(k) follow from those scalars alone
// (k_two_pass_coef).  Pass 2 repeats the identical iteration (every
// reduction is deterministic, so the residuals are the same bits) and adds
// w(k) r(k) to y from the residual ring at each block boundary.  Twice the
// operator work of the one-pass solve, none of its per-shift vector traffic
// or memory.  Stats: the per-shift residual is the recurrence's
// |zeta_i| ||r|| / ||b|| at the shift's last step (no x_i exists to check).
constexpr int kTwoPassMaxIter = 1 << 22;   // 24 B of history per step and system

static rhmc_status rational_two_pass(rhmc_gauge* g, double m, const rhmc_rational* rat, int nrhs,
                                     const double2* b, double2* y, const rhmc_solver_params& prm,
                                     rhmc_solver_stats* stats, hipStream_t s) {
    const size_t n = (size_t)3 * g->lat.Vh;
    const int np = rat->npole;
    bool converged = true;
    for (int r0 = 0; r0 < nrhs; r0 += kMaxSys) {
        const auto t0 = std::chrono::steady_clock::now();
        const int cnt = std::min(kMaxSys, nrhs - r0);
        Problem pb = make_problem(g, m, np, rat->beta, cnt, b + (size_t)r0 * n, nullptr, 0, 0, prm);
        pb.two_pass = true;
        pb.maxiter = std::min(pb.maxiter, kTwoPassMaxIter);   // bounds the step history
        RHMC_TRY(ensure_workspace(g, cnt, np, pb.K));
        Workspace* w = g->ws;
        const int cap = pb.maxiter + 1;
        RHMC_TRY(grow(w, (void**)&w->hist, &w->hist_cap, sizeof(double) * 3 * (size_t)cap * cnt));
        pb.hist = w->hist;
        pb.hist_cap = cap;
        RHMC_TRY(krylov_init<double2>(g, pb, s));
        RHMC_TRY(krylov_loop<double2>(g, pb, false, s));
        const SolverState s1 = *w->hst;
        int nmax = 1;
        for (int j = 0; j < cnt; ++j) nmax = std::max(nmax, s1.sys[j].iters);
        const size_t coef_n = (size_t)cnt * np * 3 * nmax;
        RHMC_TRY(grow(w, (void**)&w->tp, &w->tp_cap, sizeof(double) * (coef_n + (size_t)cnt * nmax)));
        TwoPassArgs ta{};
        ta.state = w->st;
        ta.hist = w->hist;
        ta.hist_cap = cap;
        ta.coef = w->tp;
        ta.nmax = nmax;
        for (int i = 0; i < np; ++i) ta.alpha[i] = rat->alpha[i];
        ta.w = w->tp + coef_n;
        RHMC_HIP_TRY(launch_two_pass_weights(ta, cnt, np, s));
        CombineArgs c{};   // y = alpha0 b
        c.n = n;
        c.nterm = 0;
        c.alpha0 = rat->alpha0;
        for (int j = 0; j < cnt; ++j) {
            c.b[j] = b + (size_t)(r0 + j) * n;
            c.y[j] = y + (size_t)(r0 + j) * n;
        }
        RHMC_HIP_TRY(launch_combine(c, cnt, s));
        Problem p2 = pb;
        p2.hist = nullptr;
        p2.hist_cap = 0;
        p2.wacc = ta.w;
        p2.w_stride = (size_t)nmax;
        p2.yacc = y + (size_t)r0 * n;
        RHMC_TRY(krylov_init<double2>(g, p2, s));
        RHMC_TRY(krylov_loop<double2>(g, p2, false, s));
        for (int j = 0; j < cnt; ++j)
            if (w->hst->sys[j].iters != s1.sys[j].iters) {
                set_error("two-pass rational apply: the second pass did not repeat the first");
                return RHMC_ERR_HIP;
            }
        // recurrence residual of each shift at its last step
        std::vector<double> hist((size_t)cnt * nmax * 3);   // [j][nmax][3]
        RHMC_HIP_TRY(hipMemcpy2DAsync(hist.data(), sizeof(double) * 3 * nmax, w->hist,
                                      sizeof(double) * 3 * (size_t)cap, sizeof(double) * 3 * nmax,
                                      cnt, hipMemcpyDeviceToHost, s));
        RHMC_HIP_TRY(hipStreamSynchronize(s));
        const auto t1 = std::chrono::steady_clock::now();
        double worst = 0.0;
        int iters = 0;
        for (int j = 0; j < cnt; ++j) {
            iters = std::max(iters, s1.sys[j].iters);
            for (int i = 0; i < np; ++i) {
                const ShiftScalars& q = s1.sh[j][i];
                const int N = q.active ? s1.sys[j].iters : q.conv_iter;
                const double bn = s1.sys[j].bnorm;
                double res = 0.0;
                if (N > 0 && bn > 0)
                    res = std::fabs(q.zeta) * std::sqrt(hist[((size_t)j * nmax + N - 1) * 3 + 2]) / bn;
                if (!(res <= prm.tol)) converged = false;
                worst = std::max(worst, res);
                const size_t p = (size_t)(r0 + j) * np + i;
                if (stats && stats->iterations) stats->iterations[p] = N;
                if (stats && stats->true_residual) stats->true_residual[p] = res;
                if (stats && stats->refine_iterations) stats->refine_iterations[p] = 0;
            }
        }
        if (stats) {
            stats->total_iterations = std::max(stats->total_iterations, iters);
            stats->time_ms += std::chrono::duration<double, std::milli>(t1 - t0).count();
            stats->max_true_residual = std::max(stats->max_true_residual, worst);
        }
        if (!std::isfinite(worst)) {
            set_error("solution is not finite");
            return RHMC_ERR_NONFINITE;
        }
    }
    if (!converged) {
        set_error("some shift did not reach the requested tolerance");
        return RHMC_ERR_NOT_CONVERGED;
    }
    return RHMC_OK;
}

rhmc_status rational(rhmc_gauge* g, double m, const rhmc_rational* rat, int nrhs,
                     const double2* b, double2* y, const rhmc_solver_params& prm,
                     rhmc_solver_stats* stats, hipStream_t s) {
    SolverCall scope(g);
    if (prm.two_pass) return rational_two_pass(g, m, rat, nrhs, b, y, prm, stats, s);
    const size_t n = (size_t)3 * g->lat.Vh;
    const int np = rat->npole;
    const int K = block_length(prm);
    RHMC_TRY(ensure_workspace(g, std::min(nrhs, kMaxSys), np, K));
    double2* xr = nullptr;
    RHMC_TRY(ensure_rational_buffer(g, (size_t)std::min(nrhs, kMaxSys) * np, &xr));
    rhmc_status worst = RHMC_OK;   // every group is solved and combined
    for (int r0 = 0; r0 < nrhs; r0 += kMaxSys) {
        const int cnt = std::min(kMaxSys, nrhs - r0);
        rhmc_solver_stats st{};
        if (stats) {
            st.iterations = stats->iterations ? stats->iterations + (size_t)r0 * np : nullptr;
            st.true_residual = stats->true_residual ? stats->true_residual + (size_t)r0 * np : nullptr;
            st.refine_iterations =
                stats->refine_iterations ? stats->refine_iterations + (size_t)r0 * np : nullptr;
        }
        const rhmc_status rs = multishift(g, m, np, rat->beta, cnt, b + (size_t)r0 * n, xr,
                                          (size_t)np * n, n, prm, &st, s);
        if (stats) {
            stats->total_iterations = std::max(stats->total_iterations, st.total_iterations);
            stats->reliable_updates += st.reliable_updates;
            stats->refine_rounds = std::max(stats->refine_rounds, st.refine_rounds);
            stats->fp64_head_iterations =
                std::max(stats->fp64_head_iterations, st.fp64_head_iterations);
            stats->time_ms += st.time_ms;
            stats->max_true_residual = std::max(stats->max_true_residual, st.max_true_residual);
            stats->head_ms += st.head_ms;
            stats->krylov_ms += st.krylov_ms;
            stats->check_ms += st.check_ms;
            stats->refine_ms += st.refine_ms;
        }
        if (rs != RHMC_OK && rs != RHMC_ERR_NOT_CONVERGED) return rs;
        CombineArgs c{};
        c.n = n;
        c.nterm = np;
        c.alpha0 = rat->alpha0;
        for (int i = 0; i < np; ++i) c.alpha[i] = rat->alpha[i];
        c.x_stride = n;
        for (int j = 0; j < cnt; ++j) {
            c.b[j] = b + (size_t)(r0 + j) * n;
            c.x[j] = xr + (size_t)j * np * n;
            c.y[j] = y + (size_t)(r0 + j) * n;
        }
        RHMC_HIP_TRY(launch_combine(c, cnt, s));
        if (rs != RHMC_OK) worst = rs;
    }
    RHMC_HIP_TRY(hipStreamSynchronize(s));
    if (worst != RHMC_OK) set_error("some shift did not reach the requested tolerance");
    return worst;
}

rhmc_status pf_action(rhmc_gauge* g, double m, const rhmc_rational* rat, int nrhs,
                      const double2* phi, double* S, const rhmc_solver_params& prm,
                      rhmc_solver_stats* stats, hipStream_t s) {
    SolverCall scope(g);
    const size_t n = (size_t)3 * g->lat.Vh;
    const int K = block_length(prm);
    RHMC_TRY(ensure_workspace(g, std::min(nrhs, kMaxSys), rat->npole, K));
    Workspace* w = g->ws;
    RHMC_TRY(grow(w, (void**)&w->ya, &w->ya_cap, w->vec_bytes * (size_t)nrhs));
    const rhmc_status rs = rational(g, m, rat, nrhs, phi, w->ya, prm, stats, s);
    if (rs != RHMC_OK && rs != RHMC_ERR_NOT_CONVERGED) return rs;
    for (int r0 = 0; r0 < nrhs; r0 += kMaxSys) {
        const int cnt = std::min(kMaxSys, nrhs - r0);
        DotArgs d{};
        d.n = n;
        d.partial = w->partial;
        for (int k = 0; k < cnt; ++k) {
            d.a[k] = phi + (size_t)(r0 + k) * n;
            d.b[k] = w->ya + (size_t)(r0 + k) * n;
        }
        RHMC_HIP_TRY(launch_dot(d, cnt, s));
        RHMC_HIP_TRY(launch_finalize(kFinNorms, nullptr, w->partial, vec_blocks(n), cnt, w->sums, s));
        RHMC_HIP_TRY(hipMemcpyAsync(w->sums_host, w->sums, sizeof(double) * cnt,
                                    hipMemcpyDeviceToHost, s));
        RHMC_HIP_TRY(hipStreamSynchronize(s));
        for (int k = 0; k < cnt; ++k) S[r0 + k] = w->sums_host[k];
    }
    return rs;
}

rhmc_status pf_force(rhmc_gauge* g, double m, const rhmc_rational* rat, int nrhs,
                     const double2* phi, double2* force, double* mom, double eps,
                     const rhmc_solver_params& prm, rhmc_solver_stats* stats, hipStream_t s) {
    SolverCall scope(g);
    const size_t n = (size_t)3 * g->lat.Vh;
    const int np = rat->npole;
    const int grp = std::min(nrhs, kMaxSys);
    const int K = block_length(prm);
    RHMC_TRY(ensure_workspace(g, grp, np, K));
    Workspace* w = g->ws;
    double2* xr = nullptr;
    RHMC_TRY(ensure_rational_buffer(g, (size_t)grp * np, &xr));
    RHMC_TRY(grow(w, (void**)&w->yf, &w->yf_cap, w->vec_bytes * (size_t)grp * np));
    rhmc_status worst = RHMC_OK;
    for (int r0 = 0; r0 < nrhs; r0 += kMaxSys) {
        const int cnt = std::min(kMaxSys, nrhs - r0);
        rhmc_solver_stats st{};
        if (stats) {
            st.iterations = stats->iterations ? stats->iterations + (size_t)r0 * np : nullptr;
            st.true_residual = stats->true_residual ? stats->true_residual + (size_t)r0 * np : nullptr;
            st.refine_iterations =
                stats->refine_iterations ? stats->refine_iterations + (size_t)r0 * np : nullptr;
        }
        // x_i = (A + beta_i)^-1 phi for every pole
        const rhmc_status rs = multishift(g, m, np, rat->beta, cnt, phi + (size_t)r0 * n, xr,
                                          (size_t)np * n, n, prm, &st, s);
        if (stats) {
            stats->total_iterations = std::max(stats->total_iterations, st.total_iterations);
            stats->reliable_updates += st.reliable_updates;
            stats->refine_rounds = std::max(stats->refine_rounds, st.refine_rounds);
            stats->fp64_head_iterations =
                std::max(stats->fp64_head_iterations, st.fp64_head_iterations);
            stats->time_ms += st.time_ms;
            stats->max_true_residual = std::max(stats->max_true_residual, st.max_true_residual);
        }
        if (rs != RHMC_OK && rs != RHMC_ERR_NOT_CONVERGED) return rs;
        if (rs != RHMC_OK) worst = rs;
        // y_i = D_oe x_i with the FP64 operator, kMaxSys vectors per launch
        const int nvec = cnt * np;
        for (int v0 = 0; v0 < nvec; v0 += kMaxSys) {
            DslashArgs<double2> d{};
            d.g = g->lat.geom;
            d.out_par = 1;
            d.nrhs = std::min(kMaxSys, nvec - v0);
            for (int k = 0; k < d.nrhs; ++k) {
                d.in[k] = xr + (size_t)(v0 + k) * n;
                d.out[k] = w->yf + (size_t)(v0 + k) * n;
            }
            set_variant(d, g);
            RHMC_HIP_TRY(launch_fp64_op(g, d, kModeD, s));
        }
        ForceArgs f{};
        f.g = g->lat.geom;
        f.x = xr;
        f.y = w->yf;
        f.nrhs = cnt;
        f.npole = np;
        for (int i = 0; i < np; ++i) f.alpha[i] = rat->alpha[i];
        f.out = force;
        f.accumulate = r0 > 0;
        f.mom = mom;
        f.eps = eps;
        RHMC_HIP_TRY(launch_force(g, f, s));
    }
    RHMC_HIP_TRY(hipStreamSynchronize(s));
    return worst;
}

}  // namespace rhmc
