/* The C ABI of librhmc used from plain C with HIP device buffers (no Python,
 * no torch).  On unit links a point source at one odd site of colour c gives
 * D_eo exactly +-1/2 at its eight even neighbours (sign eta_mu(n) times the
 * boundary sign, + for the forward hop out of n, - for the backward one) and
 * 0 elsewhere (Eq. stag); the multi-shift solve is then checked by its own
 * FP64 residual through rhmc_apply_mdagm; a rational apply agrees with its
 * two-pass form; a short trajectory of the Phi algorithm runs to a finite,
 * small energy change.  Prints "abi ok" and exits 0. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "rhmc.h"

#define CHECK(x)                                                                        \
    do {                                                                                \
        rhmc_status s_ = (x);                                                           \
        if (s_ != RHMC_OK) {                                                            \
            fprintf(stderr, "%s failed: %s (%s)\n", #x, rhmc_status_string(s_),         \
                    rhmc_last_error());                                                 \
            return 1;                                                                   \
        }                                                                               \
    } while (0)
#define HCHECK(x)                                                                       \
    do {                                                                                \
        if ((x) != hipSuccess) {                                                        \
            fprintf(stderr, "%s failed\n", #x);                                         \
            return 1;                                                                   \
        }                                                                               \
    } while (0)

static int lex(const int L[4], int x, int y, int z, int t) {
    return x + L[0] * (y + L[1] * (z + L[2] * t));
}

int main(void) {
    const int L[4] = {6, 4, 4, 8};
    const int V = L[0] * L[1] * L[2] * L[3], Vh = V / 2;
    rhmc_lattice* lat = NULL;
    CHECK(rhmc_lattice_create(L, -1, &lat));

    /* unit links, host complex128 [Lt][Lz][Ly][Lx][4][3][3] */
    double* links = (double*)calloc((size_t)V * 4 * 9 * 2, sizeof(double));
    for (int s = 0; s < V * 4; ++s)
        for (int i = 0; i < 3; ++i) links[((size_t)s * 9 + 4 * i) * 2] = 1.0;
    rhmc_gauge* g = NULL;
    CHECK(rhmc_gauge_create(lat, links, 0, 0, &g));

    /* point source at the odd site (1,2,3,5), colour 1 */
    const int src[4] = {1, 2, 3, 5}, colour = 1;
    const int src_eo = lex(L, src[0], src[1], src[2], src[3]) >> 1;
    const size_t nvec = (size_t)3 * Vh;
    double* h_in = (double*)calloc(nvec * 2, sizeof(double));
    double* h_out = (double*)calloc(nvec * 2, sizeof(double));
    h_in[((size_t)colour * Vh + src_eo) * 2] = 1.0;
    void *d_in, *d_out;
    HCHECK(hipMalloc(&d_in, nvec * 16));
    HCHECK(hipMalloc(&d_out, nvec * 16));
    HCHECK(hipMemcpy(d_in, h_in, nvec * 16, hipMemcpyHostToDevice));
    CHECK(rhmc_dslash_eo(g, 0, RHMC_PREC_FP64, 1, d_in, d_out, 0));
    HCHECK(hipMemcpy(h_out, d_out, nvec * 16, hipMemcpyDeviceToHost));

    /* expected: output at n = src -+ mu is the hop of n towards src */
    double* want = (double*)calloc(nvec * 2, sizeof(double));
    for (int mu = 0; mu < 4; ++mu)
        for (int dir = -1; dir <= 1; dir += 2) {
            int n[4] = {src[0], src[1], src[2], src[3]};
            n[mu] = (n[mu] - dir + L[mu]) % L[mu];   /* n + dir*mu = src */
            int eta = 1;
            for (int nu = 0; nu < mu; ++nu) eta *= (n[nu] & 1) ? -1 : 1;
            int bc = 1;
            if (mu == 3 && dir == +1 && n[3] == L[3] - 1) bc = -1;
            if (mu == 3 && dir == -1 && n[3] == 0) bc = -1;
            const int eo = lex(L, n[0], n[1], n[2], n[3]) >> 1;
            want[((size_t)colour * Vh + eo) * 2] += 0.5 * dir * eta * bc;
        }
    for (size_t i = 0; i < nvec * 2; ++i)
        if (h_out[i] != want[i]) {
            fprintf(stderr, "point source mismatch at %zu: %g vs %g\n", i, h_out[i], want[i]);
            return 1;
        }

    /* multi-shift solve on a smooth source, checked by its FP64 residual */
    for (size_t i = 0; i < nvec; ++i) {
        h_in[2 * i] = cos(0.37 * (double)i);
        h_in[2 * i + 1] = sin(0.11 * (double)i);
    }
    HCHECK(hipMemcpy(d_in, h_in, nvec * 16, hipMemcpyHostToDevice));
    const double shifts[3] = {0.0, 0.05, 1.0};
    const double m = 0.1;
    void* d_x;
    HCHECK(hipMalloc(&d_x, 3 * nvec * 16));
    rhmc_solver_params prm;
    rhmc_solver_params_default(&prm);
    prm.mode = RHMC_MODE_MIXED;
    rhmc_solver_stats st;
    memset(&st, 0, sizeof(st));
    CHECK(rhmc_multishift_cg(g, m, 3, shifts, 1, d_in, d_x, &prm, &st, 0));
    double bn = 0.0;
    for (size_t i = 0; i < nvec * 2; ++i) bn += h_in[i] * h_in[i];
    for (int k = 0; k < 3; ++k) {
        double* xk = (double*)malloc(nvec * 16);
        HCHECK(hipMemcpy(xk, (char*)d_x + (size_t)k * nvec * 16, nvec * 16, hipMemcpyDeviceToHost));
        CHECK(rhmc_apply_mdagm(g, m, RHMC_PREC_FP64, 1, (char*)d_x + (size_t)k * nvec * 16, d_out, 0));
        HCHECK(hipMemcpy(h_out, d_out, nvec * 16, hipMemcpyDeviceToHost));
        double r2 = 0.0;
        for (size_t i = 0; i < nvec * 2; ++i) {
            const double r = h_in[i] - h_out[i] - shifts[k] * xk[i];
            r2 += r * r;
        }
        free(xk);
        if (!(sqrt(r2 / bn) <= 1e-10)) {
            fprintf(stderr, "shift %g: residual %g\n", shifts[k], sqrt(r2 / bn));
            return 1;
        }
    }

    /* rational apply, one pass against the two-pass form (FP64) */
    const double ra[3] = {0.3, 0.2, 0.1}, rbeta[3] = {0.05, 0.5, 2.0};
    rhmc_rational rat = {0.5, 3, ra, rbeta};
    void *d_y1, *d_y2;
    HCHECK(hipMalloc(&d_y1, nvec * 16));
    HCHECK(hipMalloc(&d_y2, nvec * 16));
    rhmc_solver_params p64;
    rhmc_solver_params_default(&p64);
    CHECK(rhmc_rational_apply(g, m, &rat, 1, d_in, d_y1, &p64, NULL, 0));
    p64.two_pass = 1;
    CHECK(rhmc_rational_apply(g, m, &rat, 1, d_in, d_y2, &p64, NULL, 0));
    double* y1 = (double*)malloc(nvec * 16);
    double* y2 = (double*)malloc(nvec * 16);
    HCHECK(hipMemcpy(y1, d_y1, nvec * 16, hipMemcpyDeviceToHost));
    HCHECK(hipMemcpy(y2, d_y2, nvec * 16, hipMemcpyDeviceToHost));
    double dn = 0.0, yn = 0.0;
    for (size_t i = 0; i < nvec * 2; ++i) {
        dn += (y1[i] - y2[i]) * (y1[i] - y2[i]);
        yn += y1[i] * y1[i];
    }
    if (!(sqrt(dn / yn) <= 1e-11)) {
        fprintf(stderr, "two-pass rational apply differs: %g\n", sqrt(dn / yn));
        return 1;
    }

    /* a short trajectory (tau 0.1, one fermion step of two gauge steps) with
     * one rational for heat bath, action and force */
    rhmc_hmc_params hp;
    memset(&hp, 0, sizeof(hp));
    rhmc_md_params_default(&hp.md);
    hp.md.mass = m;
    hp.md.tau = 0.1;
    hp.md.n_md = 1;
    hp.md.gauge_steps = 2;
    hp.md.force_rational = &rat;
    hp.heatbath_rational = &rat;
    hp.action_rational = &rat;
    rhmc_solver_params_default(&hp.metropolis_solver);
    const size_t nmom = (size_t)8 * 4 * 2 * Vh;
    double* mom = (double*)malloc(nmom * sizeof(double));
    for (size_t i = 0; i < nmom; ++i) mom[i] = sin(1.7 * (double)i) * 1.2;
    void* d_mom;
    HCHECK(hipMalloc(&d_mom, nmom * sizeof(double)));
    HCHECK(hipMemcpy(d_mom, mom, nmom * sizeof(double), hipMemcpyHostToDevice));
    for (size_t i = 0; i < nvec; ++i) {
        h_in[2 * i] = 0.7 * cos(0.23 * (double)i);
        h_in[2 * i + 1] = 0.7 * sin(0.61 * (double)i);
    }
    HCHECK(hipMemcpy(d_in, h_in, nvec * 16, hipMemcpyHostToDevice));
    rhmc_trajectory_stats ts;
    memset(&ts, 0, sizeof(ts));
    CHECK(rhmc_trajectory(g, &hp, 1, d_in, (double*)d_mom, 0.5, &ts, 0));
    /* measured 0.084; a wrong force sign or scale gives order 1 and more */
    if (!(fabs(ts.dH) < 0.5)) {
        fprintf(stderr, "trajectory dH = %g\n", ts.dH);
        return 1;
    }
    printf("abi ok: %d iterations, max true residual %.2e, two-pass difference %.1e, "
           "trajectory dH %.2e (%d fermion forces)\n", st.total_iterations, st.max_true_residual,
           sqrt(dn / yn), ts.dH, ts.md.fermion_forces);
    hipFree(d_y1);
    hipFree(d_y2);
    hipFree(d_mom);
    free(y1);
    free(y2);
    free(mom);
    hipFree(d_in);
    hipFree(d_out);
    hipFree(d_x);
    free(links);
    free(h_in);
    free(h_out);
    free(want);
    rhmc_gauge_destroy(g);
    rhmc_lattice_destroy(lat);
    return 0;
}
