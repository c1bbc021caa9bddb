// Molecular dynamics of the Phi algorithm (Sec. 2.1): the multi-step
// second-order minimum-norm integrator, the Hamiltonian and one trajectory
// with its Metropolis test.  The host only sequences kernels: every kick,
// link update and reduction runs on the device, and the host reads back one
// scalar per reduction.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <new>

#include "blas.h"
#include "gauge.h"
#include "md.h"
#include "solver.h"
#include "state.h"

namespace rhmc {

namespace {

struct MdWork {
    double* red = nullptr;        // block partial sums of a reduction
    double* sums = nullptr;       // device result of a reduction
    double* sums_host = nullptr;  // pinned copy
    double2* phi = nullptr;       // pseudofermions of a trajectory
    size_t phi_bytes = 0;
    char* backup = nullptr;       // link storages at the start of a trajectory
    size_t backup_bytes = 0;
};

constexpr int kRedSlots = 2048;

rhmc_status md_work(rhmc_gauge* g, MdWork** out) {
    if (!g->md) {
        MdWork* w = new (std::nothrow) MdWork();
        if (!w) return RHMC_ERR_OOM;
        hipError_t e = hipMalloc(&w->red, sizeof(double) * kRedSlots);
        if (e == hipSuccess) e = hipMalloc(&w->sums, sizeof(double) * 8);
        if (e == hipSuccess) e = hipHostMalloc(&w->sums_host, sizeof(double) * 8);
        if (e != hipSuccess) {
            md_destroy(w);
            set_error(std::string("molecular-dynamics buffers: ") + hipGetErrorString(e));
            return e == hipErrorOutOfMemory ? RHMC_ERR_OOM : RHMC_ERR_HIP;
        }
        g->md = w;
    }
    *out = static_cast<MdWork*>(g->md);
    return RHMC_OK;
}

rhmc_status ensure(void** buf, size_t* cap, size_t need) {
    if (*cap >= need) return RHMC_OK;
    hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
    RHMC_HIP_TRY(hipMalloc(buf, need));
    *cap = need;
    return RHMC_OK;
}

// (pointer, bytes) of each link storage of g
struct Storage {
    void* p[4];
    size_t bytes[4];
};
Storage storages(const rhmc_gauge* g) {
    const size_t nl = (size_t)4 * g->lat.V;
    Storage st{};
    st.p[0] = g->u64;
    st.bytes[0] = g->u64 ? nl * 9 * sizeof(double2) : 0;
    st.p[1] = g->u64c;
    st.bytes[1] = g->u64c ? nl * 6 * sizeof(double2) : 0;
    st.p[2] = g->u32;
    st.bytes[2] = g->u32 ? nl * (g->hilo ? 6 : 3) * sizeof(float4) : 0;
    st.p[3] = g->u32f;
    st.bytes[3] = g->u32f ? nl * 9 * sizeof(float2) : 0;
    return st;
}

rhmc_status copy_links(rhmc_gauge* g, MdWork* w, bool save, hipStream_t s) {
    const Storage st = storages(g);
    size_t total = st.bytes[0] + st.bytes[1] + st.bytes[2] + st.bytes[3];
    if (save) RHMC_TRY(ensure((void**)&w->backup, &w->backup_bytes, total));
    size_t off = 0;
    for (int i = 0; i < 4; ++i) {
        if (!st.bytes[i]) continue;
        if (save)
            RHMC_HIP_TRY(hipMemcpyAsync(w->backup + off, st.p[i], st.bytes[i],
                                        hipMemcpyDeviceToDevice, s));
        else
            RHMC_HIP_TRY(hipMemcpyAsync(st.p[i], w->backup + off, st.bytes[i],
                                        hipMemcpyDeviceToDevice, s));
        off += st.bytes[i];
    }
    return RHMC_OK;
}

rhmc_status read_sum(MdWork* w, int nblk, double* out, hipStream_t s) {
    RHMC_HIP_TRY(launch_finalize(kFinNorms, nullptr, w->red, nblk, 1, w->sums, s));
    RHMC_HIP_TRY(hipMemcpyAsync(w->sums_host, w->sums, sizeof(double), hipMemcpyDeviceToHost, s));
    RHMC_HIP_TRY(hipStreamSynchronize(s));
    *out = w->sums_host[0];
    return RHMC_OK;
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

void merge(rhmc_md_stats* st, const rhmc_solver_stats& ss) {
    st->cg_iterations += ss.total_iterations;
    st->max_true_residual = std::fmax(st->max_true_residual, ss.max_true_residual);
}

}  // namespace

void md_destroy(void* p) {
    MdWork* w = static_cast<MdWork*>(p);
    if (!w) return;
    hipFree(w->red);
    hipFree(w->sums);
    hipHostFree(w->sums_host);
    hipFree(w->phi);
    hipFree(w->backup);
    delete w;
}

rhmc_status gauge_action(rhmc_gauge* g, double beta, double* S, hipStream_t s) {
    MdWork* w = nullptr;
    RHMC_TRY(md_work(g, &w));
    const int nblk = plaquette_blocks(g);
    RHMC_HIP_TRY(launch_plaquette(g, w->red, s));
    double sum = 0.0;
    RHMC_TRY(read_sum(w, nblk, &sum, s));
    *S = beta * sum;
    return RHMC_OK;
}

rhmc_status kinetic(rhmc_gauge* g, const double* mom, double* K, hipStream_t s) {
    MdWork* w = nullptr;
    RHMC_TRY(md_work(g, &w));
    DotArgs d{};
    d.n = (size_t)4 * 4 * g->lat.V;   // 8 doubles per link as 4 complex numbers
    d.a[0] = d.b[0] = reinterpret_cast<const double2*>(mom);
    d.partial = w->red;
    RHMC_HIP_TRY(launch_dot(d, 1, s));
    double sum = 0.0;
    RHMC_TRY(read_sum(w, vec_blocks(d.n), &sum, s));
    *K = 0.5 * sum;
    return RHMC_OK;
}

// Multi-step 2MN scheme.  Kicks are collected until the next link update
// (they all act on the same links) and then applied once per force.
rhmc_status md_integrate(rhmc_gauge* g, const rhmc_md_params& p, int npf, const double2* phi,
                         double* mom, rhmc_md_stats* stats, hipStream_t s) {
    const double t0 = now_ms();
    rhmc_md_stats st{};
    rhmc_status worst = RHMC_OK;
    double pend_f = 0.0, pend_g = 0.0;
    auto flush = [&]() -> rhmc_status {
        if (pend_f != 0.0) {
            rhmc_solver_stats ss{};
            const rhmc_status r = pf_force(g, p.mass, p.force_rational, npf, phi, nullptr, mom,
                                           pend_f, p.solver, &ss, s);
            if (r != RHMC_OK && r != RHMC_ERR_NOT_CONVERGED) return r;
            if (r != RHMC_OK) worst = r;
            merge(&st, ss);
            ++st.fermion_forces;
        }
        if (pend_g != 0.0) {
            RHMC_HIP_TRY(launch_gauge_force_mom(g, p.beta, pend_g, mom, s));
            ++st.gauge_forces;
        }
        pend_f = pend_g = 0.0;
        return RHMC_OK;
    };
    auto drift = [&](double c) -> rhmc_status {
        RHMC_TRY(flush());
        RHMC_HIP_TRY(launch_update_links(g, c, mom, s));
        ++st.link_updates;
        return RHMC_OK;
    };
    const double lam = p.lambda;
    const double delta = p.tau / p.n_md;
    const double h = delta / p.gauge_steps;
    auto inner = [&]() -> rhmc_status {
        for (int j = 0; j < p.gauge_steps / 2; ++j) {
            pend_g += lam * h;
            RHMC_TRY(drift(0.5 * h));
            pend_g += (1.0 - 2.0 * lam) * h;
            RHMC_TRY(drift(0.5 * h));
            pend_g += lam * h;
        }
        return RHMC_OK;
    };
    for (int i = 0; i < p.n_md; ++i) {
        pend_f += lam * delta;
        RHMC_TRY(inner());
        pend_f += (1.0 - 2.0 * lam) * delta;
        RHMC_TRY(inner());
        pend_f += lam * delta;
    }
    RHMC_TRY(flush());
    RHMC_HIP_TRY(hipStreamSynchronize(s));
    st.time_ms = now_ms() - t0;
    if (stats) *stats = st;
    return worst;
}

rhmc_status trajectory(rhmc_gauge* g, const rhmc_hmc_params& p, int npf, const double2* R,
                       double* mom, double u, rhmc_trajectory_stats* stats, hipStream_t s) {
    const double t0 = now_ms();
    MdWork* w = nullptr;
    RHMC_TRY(md_work(g, &w));
    const size_t n = (size_t)3 * g->lat.Vh;
    RHMC_TRY(ensure((void**)&w->phi, &w->phi_bytes, sizeof(double2) * n * npf));
    rhmc_status worst = RHMC_OK;
    auto keep = [&](rhmc_status r) -> bool {
        if (r == RHMC_ERR_NOT_CONVERGED) worst = r;
        return r == RHMC_OK || r == RHMC_ERR_NOT_CONVERGED;
    };
    // heat bath phi = r_hb(A) R
    rhmc_status r = rational(g, p.md.mass, p.heatbath_rational, npf, R, w->phi,
                             p.metropolis_solver, nullptr, s);
    if (!keep(r)) return r;
    double Sf[64];
    auto fermion_action = [&](double* out) -> rhmc_status {
        const rhmc_status q = pf_action(g, p.md.mass, p.action_rational, npf, w->phi, Sf,
                                        p.metropolis_solver, nullptr, s);
        if (!keep(q)) return q;
        double sum = 0.0;
        for (int k = 0; k < npf; ++k) sum += Sf[k];
        *out = sum;
        return RHMC_OK;
    };
    RHMC_TRY(kinetic(g, mom, &stats->kinetic[0], s));
    RHMC_TRY(gauge_action(g, p.md.beta, &stats->gauge_action[0], s));
    RHMC_TRY(fermion_action(&stats->pf_action[0]));
    RHMC_TRY(copy_links(g, w, true, s));
    // from here on a failure leaves the links as they were at the start
    auto fail = [&](rhmc_status q) -> rhmc_status {
        copy_links(g, w, false, s);
        hipStreamSynchronize(s);
        return q;
    };
    r = md_integrate(g, p.md, npf, w->phi, mom, &stats->md, s);
    if (!keep(r)) return fail(r);
    if ((r = kinetic(g, mom, &stats->kinetic[1], s)) != RHMC_OK) return fail(r);
    if ((r = gauge_action(g, p.md.beta, &stats->gauge_action[1], s)) != RHMC_OK) return fail(r);
    if ((r = fermion_action(&stats->pf_action[1])) != RHMC_OK) return fail(r);
    stats->dH = (stats->kinetic[1] - stats->kinetic[0]) +
                (stats->gauge_action[1] - stats->gauge_action[0]) +
                (stats->pf_action[1] - stats->pf_action[0]);
    stats->accepted = (u < std::exp(-stats->dH)) ? 1 : 0;
    if (!stats->accepted) RHMC_TRY(copy_links(g, w, false, s));
    RHMC_HIP_TRY(hipStreamSynchronize(s));
    stats->time_ms = now_ms() - t0;
    return worst;
}

}  // namespace rhmc
