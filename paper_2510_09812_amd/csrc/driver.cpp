// Relaxation and field/stress sweeps (Sec. 3.3): GSPM steps at a fixed
// applied field and stress until the mean per-node change of m over one step,
// <|m^n - m^{n-1}|> on the magnetic nodes (the convergence measure of
// Sec. 3.2 and 3.3), falls below a threshold; a sweep repeats that for a list
// of applied fields and stresses and records the cell-averaged magnetisation
// after each.  Host loops over the device step; every step runs in the
// library's kernels.
#include <cmath>
#include <cstring>

#include "context.h"

using namespace gspm;

namespace {

void add_stats(gspm_step_stats &acc, const gspm_step_stats &s) {
    acc.mech_iters += s.mech_iters;
    acc.gs_iters += s.gs_iters;
    for (int q = 0; q < 8; ++q) acc.gs_iters_stage[q] += s.gs_iters_stage[q];
    acc.elapsed_ms += s.elapsed_ms;
    acc.refinements += s.refinements;
    acc.mech_refinements += s.mech_refinements;
    acc.learned_starts += s.learned_starts;
    acc.minres_starts += s.minres_starts;
    acc.ms_iters += s.ms_iters;
    acc.dm_avg = s.dm_avg;
    acc.warm_coef[0] = s.warm_coef[0];
    acc.warm_coef[1] = s.warm_coef[1];
}

// Steps until dm_avg < dm_tol (the converging step included), at most
// max_steps.  st accumulates over the steps taken; steps_done counts them.
int relax(gspm_ctx *c, double dt, double dm_tol, int32_t max_steps, gspm_step_stats *st) {
    std::memset(st, 0, sizeof *st);
    st->failed_step = -1;
    for (int32_t k = 0; k < max_steps; ++k) {
        gspm_step_stats one;
        const int rc = run_steps(c, dt, 1, &one);
        add_stats(*st, one);
        if (rc) {
            st->failed_step = k;
            return rc;
        }
        st->steps_done = k + 1;
        if (one.dm_avg < dm_tol) return GSPM_OK;
    }
    c->err = "relax: <|dm|> did not fall below dm_tol within max_steps";
    return GSPM_E_NOCONV;
}

}  // namespace

extern "C" {

gspm_status gspm_relax(gspm_ctx *c, double dt, double dm_tol, int32_t max_steps, gspm_step_stats *stats) {
    if (!c) return GSPM_E_ARG;
    if (!c->have_mesh || !c->have_params || !c->have_m) {
        c->err = "relax needs upload_mesh, set_params and set_field(M) first";
        return GSPM_E_STATE;
    }
    if (!(dt > 0) || !std::isfinite(dt) || !(dm_tol > 0) || !std::isfinite(dm_tol) || max_steps <= 0) {
        c->err = "relax: dt and dm_tol must be positive and finite, max_steps positive";
        return GSPM_E_ARG;
    }
    hipSetDevice(c->device);
    gspm_step_stats local;
    return static_cast<gspm_status>(relax(c, dt, dm_tol, max_steps, stats ? stats : &local));
}

gspm_status gspm_sweep(gspm_ctx *c, double dt, double dm_tol, int32_t max_steps, int32_t n_points,
                       const double *hext, const double *sigma_ext, uint32_t flags, double *mbar,
                       int32_t *steps, int32_t *converged, int32_t *points_done) {
    if (!c) return GSPM_E_ARG;
    if (points_done) *points_done = 0;
    if (!hext || !mbar || !steps || n_points <= 0) {
        c->err = "sweep: hext, mbar and steps are required and n_points must be positive";
        return GSPM_E_ARG;
    }
    if (flags & ~(GSPM_SWEEP_STOP_ON_REVERSAL | GSPM_SWEEP_CONTINUE)) {
        c->err = "sweep: unknown flag";
        return GSPM_E_ARG;
    }
    if (!c->have_mesh || !c->have_params || !c->have_m) {
        c->err = "sweep needs upload_mesh, set_params and set_field(M) first";
        return GSPM_E_STATE;
    }
    if (!(dt > 0) || !std::isfinite(dt) || !(dm_tol > 0) || !std::isfinite(dm_tol) || max_steps <= 0) {
        c->err = "sweep: dt and dm_tol must be positive and finite, max_steps positive";
        return GSPM_E_ARG;
    }
    const bool stop_on_reversal = flags & GSPM_SWEEP_STOP_ON_REVERSAL, keep_going = flags & GSPM_SWEEP_CONTINUE;
    // the reversal test looks along the first point's field
    double dir[3] = {hext[0], hext[1], hext[2]};
    const double dn = std::sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    if (stop_on_reversal && !(dn > 0)) {
        c->err = "sweep: stop_on_reversal needs a nonzero first field";
        return GSPM_E_ARG;
    }
    for (int32_t k = 0; k < n_points; ++k) {
        gspm_params p = c->p;
        for (int a = 0; a < 3; ++a) p.hext[a] = hext[3 * k + a];
        if (sigma_ext)
            for (int a = 0; a < 6; ++a) p.sigma_ext[a] = sigma_ext[6 * k + a];
        gspm_status rc = gspm_set_params(c, &p);
        if (rc) return rc;
        gspm_step_stats st;
        rc = gspm_relax(c, dt, dm_tol, max_steps, &st);
        steps[k] = st.steps_done;
        if (converged) converged[k] = rc == GSPM_OK;
        // a point that ran out of steps is recorded and the sweep goes on only
        // when asked to; a failing step (failed_step set) always ends it
        if (rc && !(rc == GSPM_E_NOCONV && keep_going && st.failed_step < 0)) return rc;
        double eb[6];
        gspm_status ra = gspm_averages(c, mbar + 3 * k, eb);
        if (ra) return ra;
        if (points_done) *points_done = k + 1;
        const double along = mbar[3 * k] * dir[0] + mbar[3 * k + 1] * dir[1] + mbar[3 * k + 2] * dir[2];
        if (stop_on_reversal && along <= 0.0) break;
    }
    return GSPM_OK;
}

}  // extern "C"
