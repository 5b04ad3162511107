/* Prints the size and field offsets of the C ABI's structs as the C compiler
 * lays them out, one "struct field offset" line each, for the binding's
 * layout test.  Usage: abi_layout; exit 0. */
#include <stddef.h>
#include <stdio.h>

#include "gspm.h"

#define F(S, f) printf(#S " " #f " %zu\n", offsetof(S, f))
#define Z(S) printf(#S " sizeof %zu\n", sizeof(S))

int main(void) {
    Z(gspm_create_opts);
    F(gspm_create_opts, device); F(gspm_create_opts, precision); F(gspm_create_opts, block_nodes);
    F(gspm_create_opts, profile); F(gspm_create_opts, stream); F(gspm_create_opts, reorder);
    F(gspm_create_opts, dev_alloc); F(gspm_create_opts, dev_free); F(gspm_create_opts, alloc_user);
    F(gspm_create_opts, deterministic);
    Z(gspm_params);
    F(gspm_params, Ms); F(gspm_params, A); F(gspm_params, K1); F(gspm_params, lambda100); F(gspm_params, lambda111);
    F(gspm_params, c11); F(gspm_params, c12); F(gspm_params, c44); F(gspm_params, alpha); F(gspm_params, mu0);
    F(gspm_params, gamma0); F(gspm_params, Nd); F(gspm_params, hext); F(gspm_params, sigma_ext);
    F(gspm_params, cg_tol); F(gspm_params, cg_maxit); F(gspm_params, precession); F(gspm_params, local_demag);
    F(gspm_params, crystal_rot); F(gspm_params, elastic_precond); F(gspm_params, gs_precond); F(gspm_params, ms_tol);
    Z(gspm_step_stats);
    F(gspm_step_stats, steps_done); F(gspm_step_stats, failed_step); F(gspm_step_stats, mech_iters);
    F(gspm_step_stats, gs_iters); F(gspm_step_stats, gs_iters_stage); F(gspm_step_stats, dm_avg);
    F(gspm_step_stats, elapsed_ms); F(gspm_step_stats, matvec_ms); F(gspm_step_stats, matvec_launches);
    F(gspm_step_stats, refinements); F(gspm_step_stats, learned_starts); F(gspm_step_stats, minres_starts);
    F(gspm_step_stats, warm_coef); F(gspm_step_stats, ms_iters); F(gspm_step_stats, mech_refinements);
    F(gspm_step_stats, gs_matvec_ms); F(gspm_step_stats, gs_matvec_launches); F(gspm_step_stats, phase_ms);
    F(gspm_step_stats, final_residual);
    return 0;
}
