/* Size and field offsets of every struct of include/rhmc.h as the C compiler
 * lays them out, one "struct size" line and one "struct.field offset" line
 * each.  Runs without a GPU (no library call). */
#include <stddef.h>
#include <stdio.h>

#include "rhmc.h"

#define SIZE(T) printf(#T " %zu\n", sizeof(T))
#define FIELD(T, f) printf(#T "." #f " %zu\n", offsetof(T, f))

int main(void) {
    SIZE(rhmc_solver_params);
    FIELD(rhmc_solver_params, tol);
    FIELD(rhmc_solver_params, maxiter);
    FIELD(rhmc_solver_params, mode);
    FIELD(rhmc_solver_params, reliable_every);
    FIELD(rhmc_solver_params, refine);
    FIELD(rhmc_solver_params, block);
    FIELD(rhmc_solver_params, use_graph);
    FIELD(rhmc_solver_params, poll_every);
    FIELD(rhmc_solver_params, tune);
    FIELD(rhmc_solver_params, per_shift);
    FIELD(rhmc_solver_params, fp64_head);
    FIELD(rhmc_solver_params, two_pass);

    SIZE(rhmc_solver_stats);
    FIELD(rhmc_solver_stats, iterations);
    FIELD(rhmc_solver_stats, true_residual);
    FIELD(rhmc_solver_stats, refine_iterations);
    FIELD(rhmc_solver_stats, total_iterations);
    FIELD(rhmc_solver_stats, reliable_updates);
    FIELD(rhmc_solver_stats, refine_rounds);
    FIELD(rhmc_solver_stats, time_ms);
    FIELD(rhmc_solver_stats, max_true_residual);
    FIELD(rhmc_solver_stats, fp64_head_iterations);
    FIELD(rhmc_solver_stats, head_ms);
    FIELD(rhmc_solver_stats, krylov_ms);
    FIELD(rhmc_solver_stats, check_ms);
    FIELD(rhmc_solver_stats, refine_ms);

    SIZE(rhmc_rational);
    FIELD(rhmc_rational, alpha0);
    FIELD(rhmc_rational, npole);
    FIELD(rhmc_rational, alpha);
    FIELD(rhmc_rational, beta);

    SIZE(rhmc_md_params);
    FIELD(rhmc_md_params, beta);
    FIELD(rhmc_md_params, mass);
    FIELD(rhmc_md_params, tau);
    FIELD(rhmc_md_params, n_md);
    FIELD(rhmc_md_params, gauge_steps);
    FIELD(rhmc_md_params, lambda);
    FIELD(rhmc_md_params, force_rational);
    FIELD(rhmc_md_params, solver);

    SIZE(rhmc_md_stats);
    FIELD(rhmc_md_stats, fermion_forces);
    FIELD(rhmc_md_stats, gauge_forces);
    FIELD(rhmc_md_stats, link_updates);
    FIELD(rhmc_md_stats, cg_iterations);
    FIELD(rhmc_md_stats, max_true_residual);
    FIELD(rhmc_md_stats, time_ms);

    SIZE(rhmc_hmc_params);
    FIELD(rhmc_hmc_params, md);
    FIELD(rhmc_hmc_params, heatbath_rational);
    FIELD(rhmc_hmc_params, action_rational);
    FIELD(rhmc_hmc_params, metropolis_solver);

    SIZE(rhmc_trajectory_stats);
    FIELD(rhmc_trajectory_stats, kinetic);
    FIELD(rhmc_trajectory_stats, gauge_action);
    FIELD(rhmc_trajectory_stats, pf_action);
    FIELD(rhmc_trajectory_stats, dH);
    FIELD(rhmc_trajectory_stats, accepted);
    FIELD(rhmc_trajectory_stats, md);
    FIELD(rhmc_trajectory_stats, time_ms);
    return 0;
}
