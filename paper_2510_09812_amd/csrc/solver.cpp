// CG driver and the GSPM step sequence (host side; all arithmetic runs in
// the kernels).
//
// CG runs without a host round trip per iteration.  Each iteration is two
// launches: the matvec, whose staging forms the new direction
// p_k = r_k + beta_k p_{k-1} after testing ||r_k|| on the device, with p.Ap
// fused into its epilogue; and the x/r update with r.r fused.  Directions are
// double-buffered (a block reads the previous direction at its halo nodes
// while other blocks write the new one).  Convergence is decided on the device
// and a converged solve turns the remaining launches into immediate exits.  The host
// enqueues iterations in batches and reads the convergence flags of the
// previous batch while the next one runs, so the device never waits for it.
#include <algorithm>
#include <cstring>

#include "context.h"

namespace gspm {

int hip_check(gspm_ctx *c, hipError_t e, const char *what) {
    if (e == hipSuccess) return GSPM_OK;
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? GSPM_E_OOM : GSPM_E_DEVICE;
}

void cg_prepare(gspm_ctx *c, int ns) {
    launch_fill(c->d.cg_bb, kMaxComp * kShards, 0.0, c->stream);
    launch_fill_i32(c->d.cg_flags, 2 * kMaxComp, 0, c->stream);
    launch_zero_ring(c->cg, ns, 0, 1, 0, 0, c->stream);
}

namespace {

template <class Apply>
CgResult cg_run(gspm_ctx *c, int nc, bool joint, double *x, const double *b, double tol, int maxit, SolveKind kind,
                Apply apply) {
    hipStream_t s = c->stream;
    const int ns = joint ? 1 : nc, n = c->n;
    CgResult res;
    apply(MV_RESID, x, nullptr, b, c->d.r, nullptr, 0);
    launch_cg_start(n, nc, joint, x, c->cg, tol, s);
    double *P[2] = {c->d.p, c->d.p2};

    const int cap = c->cg.ring - 2;
    const int first = std::min(std::max(c->predict[kind] + 1, 2), cap);
    const int later = std::min(std::max(c->predict[kind] / 32, 4), std::min(cap, 32));
    int k = 0;
    auto enqueue = [&](int cnt) {
        const int k1 = std::min(k + cnt, maxit);
        launch_zero_ring(c->cg, ns, k + 1, k1 + 1, k, k1, s);
        for (int it = k; it < k1; ++it) {
            double *pold = P[it & 1], *pnew = P[(it + 1) & 1];
            apply(MV_ITER, pold, c->d.q, nullptr, c->d.r, pnew, it);
            launch_cg_update(n, nc, joint, x, c->d.r, pnew, c->d.q, c->cg, it, s);
        }
        if (k1 == maxit) launch_cg_check(nc, joint, c->cg, maxit, tol, s);
        k = k1;
    };
    auto post = [&](int slot) {
        hipMemcpyAsync(c->h_flags + 2 * kMaxComp * slot, c->d.cg_flags, sizeof(int32_t) * 2 * kMaxComp,
                       hipMemcpyDeviceToHost, s);
        hipEventRecord(c->ev[slot], s);
    };
    enqueue(first);
    post(0);
    int pending = 0, next = 1;
    for (;;) {
        const bool more = k < maxit;
        if (more) {
            enqueue(later);
            post(next);
        }
        hipError_t e = hipEventSynchronize(c->ev[pending]);
        if (e != hipSuccess) {
            res.status = hip_check(c, e, "CG");
            return res;
        }
        const int32_t *f = c->h_flags + 2 * kMaxComp * pending;
        bool all = true, broke = false;
        for (int q = 0; q < ns; ++q) {
            all &= f[q] != 0;
            broke |= f[q] == 2;
        }
        if (all) {
            int mx = 0;
            for (int q = 0; q < ns; ++q) {
                res.iters[q] = f[kMaxComp + q];
                mx = std::max(mx, res.iters[q]);
            }
            if (broke) {
                res.status = GSPM_E_NONFINITE;
                c->err = "non-finite CG residual";
            }
            c->predict[kind] = mx;
            return res;
        }
        if (!more) {
            res.status = GSPM_E_NOCONV;
            c->err = "CG did not converge within cg_maxit iterations";
            for (int q = 0; q < ns; ++q) res.iters[q] = f[q] ? f[kMaxComp + q] : maxit;
            return res;
        }
        pending = next;
        next ^= 1;
    }
}

// Profile mode: an event pair around every elastic matvec of an iteration;
// pairs of launches issued after convergence (immediate exits) are dropped.
void prof_begin(gspm_ctx *c, int k) {
    if (!c->profile) return;
    if (c->prof_used + 2 > c->prof_ev.size()) {
        for (int i = 0; i < 256; ++i) {
            hipEvent_t e;
            hipEventCreate(&e);
            c->prof_ev.push_back(e);
        }
    }
    c->prof_iter.resize(c->prof_ev.size() / 2);
    c->prof_iter[c->prof_used / 2] = k;
    hipEventRecord(c->prof_ev[c->prof_used], c->stream);
}

void prof_end(gspm_ctx *c) {
    if (!c->profile) return;
    hipEventRecord(c->prof_ev[c->prof_used + 1], c->stream);
    c->prof_used += 2;
}

}  // namespace

CgResult cg_elastic(gspm_ctx *c, double *x, const double *b, double tol, int maxit, SolveKind kind) {
    const size_t first_pair = c->prof_used / 2;
    CgResult r = cg_run(c, 3, true, x, b, tol, maxit, kind,
                        [&](MatvecMode mode, const double *in, double *out, const double *bb, double *rr, double *p,
                            int k) {
                            const bool timed = mode == MV_ITER;
                            if (timed) prof_begin(c, k);
                            launch_elastic_matvec(c->mv, c->mat, mode, in, out, bb, rr, p, c->cg, k, tol, c->stream);
                            if (timed) prof_end(c);
                        });
    if (c->profile)
        for (size_t i = first_pair; i < c->prof_used / 2; ++i)
            if (c->prof_iter[i] >= r.iters[0]) c->prof_iter[i] = -1;
    return r;
}

CgResult cg_gs(gspm_ctx *c, int nc, double eps, double *x, const double *b, double tol, int maxit, SolveKind kind) {
    return cg_run(c, nc, false, x, b, tol, maxit, kind,
                  [&](MatvecMode mode, const double *in, double *out, const double *bb, double *r, double *p, int k) {
                      launch_gs_matvec(c->mv, nc, eps, 1.0, mode, in, out, bb, r, p, c->cg, k, tol, c->stream);
                  });
}

namespace {

// One step of Algorithm B.1 (App. B) in the finite-element form of Eq.
// (weak_GS); (1 - eps lap)^-1 [y + c h] is the solution g of
// (eps K + M) g = M y + c M h with eps = l_ex^2 dtau.  Rows 1 and 2 of Step 2
// use m^n and g^n as printed, row 3 uses m* and g*; g* uses h[m^n];
// elasticity is solved once per step at m^n and held for h[m*].
int one_step(gspm_ctx *c, double dtau, double eps1, double eps3, gspm_step_stats *st) {
    auto &d = c->d;
    hipStream_t s = c->stream;
    const int n = c->n;
    const size_t bytes3 = sizeof(double) * 3 * static_cast<size_t>(n);
    const double tol = c->p.cg_tol;
    const int maxit = c->p.cg_maxit;
    const double l100 = c->mat.l100, l111 = c->mat.l111;

    // volume averages at m^n: far field and homogeneous strain
    launch_avg_sums(n, d.w, d.m, l100, l111, d.sums, s);
    launch_derive(d.sums, c->dargs, &d.der[0], s);

    // mechanical equilibrium at m^n, warm start from u^{n-1}
    hipMemcpyAsync(d.unext, d.u, bytes3, hipMemcpyDeviceToDevice, s);
    cg_prepare(c, 1);
    launch_elastic_rhs(c->mv, c->mat, d.m, d.b, d.unext, c->cg.bb, s);
    CgResult r = cg_elastic(c, d.unext, d.b, tol, maxit, SK_MECH);
    st->mech_iters += r.iters[0];
    if (r.status) return r.status;

    if (c->p.precession) {
        // Step 1: g^n, three components
        cg_prepare(c, 3);
        launch_field_rhs(c->mv, c->mat, d.m, d.unext, &d.der[0], dtau, d.b, d.g, d.ch2, c->cg.bb, kShards, s);
        r = cg_gs(c, 3, eps1, d.g, d.b, tol, maxit, SK_GS1);
        for (int q = 0; q < 3; ++q) st->gs_iters_stage[q] += r.iters[q];
        if (r.status) return r.status;
        // Step 2, rows 1 and 2
        launch_update_m12(n, d.m, d.g, d.ms, s);
        // Step 1: g* for components 1 and 2 with h[m^n]
        cg_prepare(c, 2);
        launch_mass_rhs(c->mv, d.ms, d.ch2, d.b, d.gs, c->cg.bb, kShards, s);
        r = cg_gs(c, 2, eps1, d.gs, d.b, tol, maxit, SK_GS2);
        for (int q = 0; q < 2; ++q) st->gs_iters_stage[3 + q] += r.iters[q];
        if (r.status) return r.status;
        // Step 2, row 3
        launch_update_m3(n, d.m, d.gs, d.ms, s);
    } else {
        hipMemcpyAsync(d.ms, d.m, bytes3, hipMemcpyDeviceToDevice, s);
    }

    // Step 3: damped solve with h[m*], averages re-evaluated at m*
    launch_avg_sums(n, d.w, d.ms, l100, l111, d.sums, s);
    launch_derive(d.sums, c->dargs, &d.der[1], s);
    cg_prepare(c, 3);
    launch_field_rhs(c->mv, c->mat, d.ms, d.unext, &d.der[1], c->p.alpha * dtau, d.b, d.g, nullptr, c->cg.bb,
                     kShards, s);
    r = cg_gs(c, 3, eps3, d.g, d.b, tol, maxit, SK_GS3);
    for (int q = 0; q < 3; ++q) st->gs_iters_stage[5 + q] += r.iters[q];
    if (r.status) return r.status;

    // Step 4: unit length
    launch_fill(d.dm, kShards, 0.0, s);
    launch_fill_i32(d.bad, 1, 0, s);
    launch_normalize(n, d.w, d.g, d.m, d.mnext, d.dm, d.bad, s);
    double dmh[kShards];
    int32_t badh = 0;
    hipMemcpyAsync(dmh, d.dm, sizeof dmh, hipMemcpyDeviceToHost, s);
    hipMemcpyAsync(&badh, d.bad, sizeof badh, hipMemcpyDeviceToHost, s);
    int rc = hip_check(c, hipStreamSynchronize(s), "step");
    if (rc) return rc;
    if (badh) {
        c->err = "zero or non-finite magnetisation after the damped solve";
        return GSPM_E_NONFINITE;
    }
    double dsum = 0.0;
    for (int k = 0; k < kShards; ++k) dsum += dmh[k];
    st->dm_avg = c->nmag > 0 ? dsum / c->nmag : 0.0;
    std::swap(d.m, d.mnext);
    std::swap(d.u, d.unext);
    return GSPM_OK;
}

}  // namespace

int run_steps(gspm_ctx *c, double dt, int nsteps, gspm_step_stats *st) {
    std::memset(st, 0, sizeof *st);
    st->failed_step = -1;
    const double dtau = c->p.gamma0 * c->p.Ms * dt;
    const double lex2 = 2.0 * c->p.A / (c->p.mu0 * c->p.Ms * c->p.Ms);
    const double eps1 = lex2 * dtau, eps3 = c->p.alpha * eps1;
    c->prof_used = 0;
    hipEventRecord(c->t0, c->stream);
    int rc = GSPM_OK;
    for (int step = 0; step < nsteps; ++step) {
        rc = one_step(c, dtau, eps1, eps3, st);
        if (rc) {
            st->failed_step = step;
            break;
        }
        st->steps_done = step + 1;
    }
    hipEventRecord(c->t1, c->stream);
    int rc2 = hip_check(c, hipStreamSynchronize(c->stream), "step");
    if (!rc) rc = rc2;
    float ms = 0.0f;
    hipEventElapsedTime(&ms, c->t0, c->t1);
    st->elapsed_ms = ms;
    for (int q = 0; q < 8; ++q) st->gs_iters += st->gs_iters_stage[q];
    if (c->profile) {
        double tot = 0.0;
        int64_t cnt = 0;
        for (size_t i = 0; i + 1 < c->prof_used; i += 2) {
            if (c->prof_iter[i / 2] < 0) continue;
            float e = 0.0f;
            hipEventElapsedTime(&e, c->prof_ev[i], c->prof_ev[i + 1]);
            tot += e;
            ++cnt;
        }
        st->matvec_ms = tot;
        st->matvec_launches = cnt;
    }
    return rc;
}

}  // namespace gspm
