// CG driver and the GSPM step sequence (host side; all arithmetic runs in
// the kernels).
//
// CG runs without a host round trip per iteration.  The elastic solve, the GS
// solves and the step's magnetostatic solve run single-reduction CG: one
// fused launch per iteration, which completes the previous iteration (its
// scalars summed in the prologue), forms r, p and x in the staging and writes
// p and q = A p with the next iteration's dot products in the epilogue.
// Multi-component magnetostatic solves (and the preconditioned elastic solve)
// take separate launches: the matvec, whose staging forms the new direction
// p_k = z_k + beta_k p_{k-1} after testing ||r_k|| on the device, with p.Ap
// fused into its epilogue; and the x/r update with r.r fused.  Vectors that
// other workgroups read as halo while a launch writes their successors are
// double-buffered.  Convergence is decided on the device and a converged
// solve turns the remaining launches into immediate exits.  The host
// enqueues iterations in batches sized by the last solve of the same kind and
// reads the convergence flags of the previous batch while the next one runs;
// solves whose iterations carry library FFTs (the preconditioned elastic
// solve) wait for the flags instead of queueing ahead (cg_iterate).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "context.h"

namespace gspm {

int hip_check(gspm_ctx *c, hipError_t e, const char *what) {
    if (e == hipSuccess) return GSPM_OK;
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? GSPM_E_OOM : GSPM_E_DEVICE;
}

void cg_prepare(gspm_ctx *c, int ns) { launch_cg_reset(c->cg, ns, c->stream); }

namespace {

// Batched CG iterations with device-side convergence.  iter(k, false)
// enqueues iteration k on the scalar set `cg`; iter(maxit, true) the launch
// after the last permitted iteration, which tests (and, for single-reduction
// CG, completes) it.  Returns when every component of `cg` has converged (or
// broken down), or after maxit iterations.
template <class Iter>
CgResult cg_iterate(gspm_ctx *c, const CGScalars &cg, int nc, bool joint, int maxit, SolveKind kind, Iter iter) {
    hipStream_t s = c->stream;
    const int ns = joint ? 1 : nc;
    CgResult res;
    const int cap = cg.ring - 2;
    int &pred = c->predict[kind][c->refine_slot];
    // fused launches test an iteration's residual in the next launch (hence
    // pred + 1); the preconditioned iteration tests it at the end of its own
    // launch group when it closes a batch
    const int first = c->heavy_iter ? std::min(std::max(pred, 1), cap) : std::min(std::max(pred + 1, 2), cap);
    // Costly iterations are not queued ahead: each launch group that runs
    // past convergence still costs its library FFTs (about 80 us, a third of
    // a working iteration), more than the device idles while the host reads
    // the flags.  Their solves enqueue the predicted count (the batch's last
    // iteration tests its residual and leaves the next preconditioner
    // application to the next batch), wait, and go on one iteration at a
    // time.
    const bool ahead = !c->heavy_iter;
    const int later = c->heavy_iter ? 1 : std::min(std::max(pred / 32, 4), std::min(cap, 32));
    int k = 0;
    auto enqueue = [&](int cnt) {
        const int k1 = std::min(k + cnt, maxit);
        c->batch_last = k1 - 1;
        launch_zero_ring(cg, ns, k + 1, k1 + 1, k, k1, s);
        for (int it = k; it < k1; ++it) iter(it, false);
        if (k1 == maxit) iter(maxit, true);
        k = k1;
    };
    auto post = [&](int slot) {
        launch_i32_to_host(cg.done, 2 * kMaxComp, c->h_flags + 2 * kMaxComp * slot, s);
        hipEventRecord(c->ev[slot], s);
    };
    enqueue(first);
    post(0);
    int pending = 0, next = 1;
    for (;;) {
        const bool more = k < maxit;
        if (more && ahead) {
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
            pred = mx;
            return res;
        }
        if (!more) {
            res.status = GSPM_E_NOCONV;
            c->err = "CG did not converge within cg_maxit iterations";
            for (int q = 0; q < ns; ++q) res.iters[q] = f[q] ? f[kMaxComp + q] : maxit;
            return res;
        }
        if (!ahead) {
            // the flags just read are consumed: their slot takes the next batch
            enqueue(later);
            post(pending);
            continue;
        }
        pending = next;
        next ^= 1;
    }
}

// Profile mode: an event pair that the runtime records at the start and end of
// every elastic matvec kernel of an iteration (the kernel alone, as a kernel
// trace times it); pairs of launches issued after convergence (immediate
// exits) are dropped.  Returns the pair to launch with, or null.
const hipEvent_t *prof_begin(gspm_ctx *c, int k) {
    if (!c->profile || c->prof_list < 0) return nullptr;
    auto &pl = c->prof[c->prof_list];
    if (pl.used + 2 > pl.ev.size()) {
        for (int i = 0; i < 256; ++i) {
            hipEvent_t e;
            hipEventCreate(&e);
            pl.ev.push_back(e);
        }
    }
    pl.iter.resize(pl.ev.size() / 2);
    pl.iter[pl.used / 2] = k;
    return &pl.ev[pl.used];
}

void prof_end(gspm_ctx *c) {
    if (c->profile && c->prof_list >= 0) c->prof[c->prof_list].used += 2;
}

size_t prof_mark(const gspm_ctx *c) { return c->prof_list >= 0 ? c->prof[c->prof_list].used / 2 : 0; }

void prof_drop_after(gspm_ctx *c, size_t first_pair, int iters) {
    if (!c->profile || c->prof_list < 0) return;
    auto &pl = c->prof[c->prof_list];
    for (size_t i = first_pair; i < pl.used / 2; ++i)
        if (pl.iter[i] >= iters) pl.iter[i] = -1;
}

// Plain FP64 CG from the initial guess x (Sec. 2.5): residual, start test,
// iterations.  resid() writes r = b - A x and rr[0]; iter(k) one iteration.
// The relative residual at which a solve stopped (the largest over its scalar
// sets): |r|^2 of the recorded iteration (the slot every form leaves it in)
// over |b|^2; kept for the statistics of the call's last step.
void record_residual(gspm_ctx *c, const CGScalars &cg, int ns, const CgResult &r, SolveKind kind) {
    if (!c->want_res || r.status) return;
    ShardSources src{};
    for (int q = 0; q < ns; ++q) {
        src.p[q] = cg.rr_at(q, r.iters[q]);
        src.p[ns + q] = cg.bb_at(q);
    }
    double *h = c->h_step + 8;
    launch_totals_to_host(src, 2 * ns, h, c->stream);
    if (hip_check(c, hipStreamSynchronize(c->stream), "CG residual")) return;
    double worst = 0.0;
    for (int q = 0; q < ns; ++q)
        if (h[ns + q] > 0.0) worst = std::max(worst, std::sqrt(std::max(h[q], 0.0) / h[ns + q]));
    c->last_res[kind] = worst;
}

template <class Resid, class Iter>
CgResult cg_fp64(gspm_ctx *c, int nc, bool joint, double *x, double tol, int maxit, SolveKind kind, Resid resid,
                 Iter iter) {
    resid();
    launch_cg_start<double>(c->n, nc, joint, x, c->cg, tol, c->stream);
    CgResult r = cg_iterate(c, c->cg, nc, joint, maxit, kind, iter);
    record_residual(c, c->cg, joint ? 1 : nc, r, kind);
    return r;
}

// Mixed form: FP64 iterative refinement around FP32 CG.  Each outer step
// computes the true residual r = b - A x with the FP64 operator and stops
// when ||r|| <= tol ||b|| for every component (the same criterion as the
// plain path, on the true residual); otherwise an inner CG in FP32 vectors
// and FP32 element arithmetic (FP64 dot products) reduces the residual of
// A d = r by eta = max(tol ||b|| / (2 ||r||), kInnerFloor), and x += d.
// `scale` maps the FP64 residual to the right-hand side of the FP32 inner
// operator A' = scale A (the non-dimensional form the FP32 kernels use).
template <class Resid, class Iter32>
CgResult cg_mixed(gspm_ctx *c, int nc, bool joint, double *x, double tol, int maxit, SolveKind kind, double scale,
                  Resid resid, Iter32 iter32) {
    constexpr double kInnerFloor = 1e-6;
    hipStream_t s = c->stream;
    const int ns = joint ? 1 : nc, n = c->n;
    const size_t n3 = 3 * static_cast<size_t>(n);
    CgResult res;
    int total[kMaxComp] = {0, 0, 0};
    double *hs = c->h_mixed;   // pinned: the totals rr[ns] | bb[ns] of the outer residual
    for (int outer = 0;; ++outer) {
        launch_zero_ring(c->cg, ns, 0, 1, 0, 0, s);
        launch_zero_ring(c->cg_in, ns, 0, 1, 0, 0, s);   // slot 0 of an inner solve that may follow
        resid();
        ShardSources src{};
        for (int q = 0; q < ns; ++q) {
            src.p[q] = c->cg.rr_at(q, 0);
            src.p[ns + q] = c->cg.bb_at(q);
        }
        launch_totals_to_host(src, 2 * ns, hs, s);
        int rc = hip_check(c, hipStreamSynchronize(s), "CG");
        if (rc) {
            res.status = rc;
            return res;
        }
        double rr[kMaxComp] = {0, 0, 0}, bb[kMaxComp] = {0, 0, 0};
        bool conv[kMaxComp] = {true, true, true}, all = true;
        for (int q = 0; q < ns; ++q) {
            rr[q] = hs[q];
            bb[q] = hs[ns + q];
            if (!std::isfinite(rr[q])) {
                res.status = GSPM_E_NONFINITE;
                c->err = "non-finite residual";
                return res;
            }
            if (bb[q] == 0.0) {
                for (int cc = 0; cc < nc; ++cc)
                    if ((joint ? 0 : cc) == q) launch_fill(x + static_cast<size_t>(cc) * n, n, 0.0, s);
            }
            conv[q] = bb[q] == 0.0 || rr[q] <= tol * tol * bb[q];
            all &= conv[q];
        }
        if (all) {
            double worst = 0.0;
            for (int q = 0; q < ns; ++q)
                if (bb[q] > 0.0) worst = std::max(worst, std::sqrt(std::max(rr[q], 0.0) / bb[q]));
            c->last_res[kind] = worst;
            break;
        }
        int used = 0;
        for (int q = 0; q < ns; ++q) used = std::max(used, total[q]);
        if (used >= maxit) {
            res.status = GSPM_E_NOCONV;
            c->err = "CG did not converge within cg_maxit iterations";
            break;
        }
        // inner FP32 solve: per-component stopping folded into bb_in = eta^2 rr
        InnerStart ist{};
        for (int q = 0; q < kMaxComp; ++q) ist.done[q] = (q < ns && !conv[q]) ? 0 : 1;
        for (int q = 0; q < ns; ++q) {
            if (conv[q]) continue;
            const double eta = std::max(0.5 * tol * std::sqrt(bb[q] / rr[q]), kInnerFloor);
            ist.bb[q] = eta * eta * rr[q] * scale * scale;
        }
        const CGScalars &ci = c->cg_in;
        launch_inner_start(n, nc, joint, c->d.r, scale, c->d.r32, c->d.x32, static_cast<int64_t>(n3), ci, ist, s);
        const int budget = maxit - used;
        const size_t first_pair = prof_mark(c);
        c->refine_slot = outer > 0 ? 1 : 0;
        CgResult in = cg_iterate(c, ci, nc, joint, budget, kind, iter32);
        c->refine_slot = 0;
        prof_drop_after(c, first_pair, std::max(in.iters[0], std::max(in.iters[1], in.iters[2])));
        if (in.status == GSPM_E_NONFINITE || in.status == GSPM_E_DEVICE || in.status == GSPM_E_OOM) {
            res.status = in.status;
            return res;
        }
        for (int q = 0; q < ns; ++q)
            if (!conv[q]) total[q] += in.iters[q];
        launch_add_f32(static_cast<int64_t>(nc) * n, x, c->d.x32, s);
        ++c->refinements;
        if (kind == SK_MECH) ++c->mech_refinements;
    }
    for (int q = 0; q < ns; ++q) res.iters[q] = total[q];
    return res;
}

}  // namespace

// Iteration k of CG preconditioned by B on the periodic elastic system (no
// pinned node).  At k = 0 the preconditioner first forms z_0 = B r_0 (and
// r_0 . z_0).  Then: the matvec forms p_k = z_k + beta p_{k-1} and q = K p_k
// with p_k . q; the update takes x += alpha p_k, r -= alpha q with |r|^2; the
// preconditioner tests |r_{k+1}| (recording convergence as iteration k + 1)
// and forms z_{k+1} = B r_{k+1} with r_{k+1} . z_{k+1}: restriction to the
// grid, forward FFT, the symbol inverse mode by mode, inverse FFT,
// prolongation with the diagonal term.  p alternates between two buffers
// (other workgroups read p_{k-1} as halo while p_k is written).
// The last iteration of a batch only tests |r_{k+1}| and leaves z_{k+1} to
// the next batch, which the host enqueues after reading the flags: a solve
// that converged there skips the preconditioner's FFTs.
template <class T>
auto pcg_iteration(gspm_ctx *c, const MeshView &mvu, T *x, T *r, T *z, T *pa, T *pb, T *q, const CGScalars &cg,
                   double tol, int *fft_rc) {
    return [=](int k, bool last) {
        if (last) return;                  // |r| of the last iteration was tested by its own preconditioner pass
        hipStream_t s = c->stream;
        const GreenView &gv = c->pc.gv;
        auto precond = [&](int test_k) {
            launch_pc_restrict<T>(gv, c->n, r, cg, test_k, tol, s);
            int rc = green_fft(c, true);
            launch_pc_modes<T>(gv, cg, s);
            rc = rc ? rc : green_fft(c, false);
            launch_pc_prolong<T>(gv, c->mv, r, z, pcg_rz_at(cg, test_k), cg, s);
            if (rc && !*fft_rc) *fft_rc = rc;
        };
        if (k == 0 || c->pc_owed) {
            precond(k);
            c->pc_owed = false;
        }
        T *pin = (k & 1) ? pa : pb, *pout = (k & 1) ? pb : pa;
        launch_elastic_pcg<T>(mvu, c->mat, k, z, pin, pout, q, cg, s, prof_begin(c, k));
        prof_end(c);
        launch_pcg_update<T>(c->n, x, r, pout, q, cg, k, s);
        if (k == c->batch_last) {
            launch_cg_check(3, true, cg, k + 1, tol, s);
            c->pc_owed = true;
        } else {
            precond(k + 1);
        }
    };
}

// The elastic solve with the Green's-operator preconditioner (elastic_precond):
// b (the periodic right-hand side) loses its mean and |b| is recomputed, CG
// runs with B on the periodic system (FP64, or FP64 refinement around FP32
// inner iterations in the mixed form), and x is pinned at p0 by a translation.
CgResult cg_elastic_green(gspm_ctx *c, double *x, double *b, double tol, int maxit, SolveKind kind) {
    hipStream_t s = c->stream;
    MeshView mvu = c->mv;
    mvu.p0 = -1;
    launch_remove_mean3(c->n, b, c->pc.aux, c->cg.bb_at(0), s, c->mv.det);
    auto resid = [&]() {
        launch_elastic_matvec<double>(mvu, c->mat, MV_RESID, x, nullptr, b, c->d.r, nullptr, c->cg, 0, tol, s);
    };
    auto &d = c->d;
    int fft_rc = 0;
    CgResult r;
    c->heavy_iter = true;
    if (c->precision == GSPM_MIXED) {
        const double scale = 1.0 / (c->mv.len_scale * c->mat.c11);
        r = cg_mixed(c, 3, true, x, tol, maxit, kind, scale, resid,
                     pcg_iteration<float>(c, mvu, d.x32, d.r32, d.r32b, d.p32, d.p32b, d.q32, c->cg_in, 1.0, &fft_rc));
    } else {
        const size_t first_pair = prof_mark(c);
        r = cg_fp64(c, 3, true, x, tol, maxit, kind, resid,
                    pcg_iteration<double>(c, mvu, x, d.r, d.r2, d.p, d.p2, d.q, c->cg, tol, &fft_rc));
        prof_drop_after(c, first_pair, r.iters[0]);
    }
    c->heavy_iter = false;
    if (fft_rc && r.status == GSPM_OK) r.status = fft_rc;
    launch_pin_shift(c->n, x, c->p0, c->pc.aux + 3 * kShards, s);
    return r;
}

// The elastic solve runs single-reduction CG: one fused launch per iteration
// (launch_elastic_cg), r, p and q alternating between two buffers.
CgResult cg_elastic(gspm_ctx *c, double *x, const double *b, double tol, int maxit, SolveKind kind) {
    c->prof_list = 0;
    if (c->p.elastic_precond == GSPM_PRECOND_GREEN) {
        CgResult r = cg_elastic_green(c, x, const_cast<double *>(b), tol, maxit, kind);
        c->prof_list = -1;
        return r;
    }
    const size_t first_pair = prof_mark(c);
    hipStream_t s = c->stream;
    auto resid = [&]() {
        launch_elastic_matvec<double>(c->mv, c->mat, MV_RESID, x, nullptr, b, c->d.r, nullptr, c->cg, 0, tol, s);
    };
    // iteration k reads the buffers of iteration k-1 and writes those of k
    auto fused = [&](auto *R0, auto *R1, auto *P0, auto *P1, auto *Q0, auto *Q1, auto *xv, const CGScalars &cg,
                     double t) {
        return [=](int k, bool last) {
            auto *R = k & 1 ? R1 : R0, *P = k & 1 ? P1 : P0, *Q = k & 1 ? Q1 : Q0;
            auto *Rp = k & 1 ? R0 : R1, *Pp = k & 1 ? P0 : P1, *Qp = k & 1 ? Q0 : Q1;
            if (k == 0) Rp = R0;
            const hipEvent_t *ev = last ? nullptr : prof_begin(c, k);
            launch_elastic_cg(c->mv, c->mat, k, last, Rp, Pp, Qp, R, P, Q, xv, cg, t, s, ev);
            if (!last) prof_end(c);
        };
    };
    CgResult r;
    if (c->precision == GSPM_MIXED) {
        auto &d = c->d;
        const double scale = 1.0 / (c->mv.len_scale * c->mat.c11);
        r = cg_mixed(c, 3, true, x, tol, maxit, kind, scale, resid,
                     fused(d.r32, d.r32b, d.p32, d.p32b, d.q32, d.q32b, d.x32, c->cg_in, 1.0));
    } else {
        auto &d = c->d;
        r = cg_fp64(c, 3, true, x, tol, maxit, kind, resid, fused(d.r, d.r2, d.p, d.p2, d.q, d.q2, x, c->cg, tol));
        prof_drop_after(c, first_pair, r.iters[0]);
    }
    c->prof_list = -1;
    return r;
}

CgResult cg_gs_run(gspm_ctx *c, int nc, double eps, double *x, const double *b, double tol, int maxit,
                   SolveKind kind);

// The GS solves; with gs_precond = GSPM_PRECOND_JACOBI, CG preconditioned by
// the operator's diagonal D = eps K_ii + M_ii (the same stopping rule on |r|).
CgResult cg_gs(gspm_ctx *c, int nc, double eps, double *x, const double *b, double tol, int maxit, SolveKind kind) {
    c->prof_list = nc == 3 ? 1 : -1;
    CgResult r = cg_gs_run(c, nc, eps, x, b, tol, maxit, kind);
    c->prof_list = -1;
    return r;
}

GsRowsView gs_rows(gspm_ctx *c, double eps, double mass, bool fp32) {
    auto &d = c->d;
    int k = -1;
    for (int j = 0; j < 2; ++j)
        if (c->gs_slot[j].valid && c->gs_slot[j].eps == eps && c->gs_slot[j].mass == mass) k = j;
    if (k < 0) {
        k = !c->gs_slot[0].valid ? 0 : !c->gs_slot[1].valid ? 1 : (c->gs_slot[0].used <= c->gs_slot[1].used ? 0 : 1);
        const int n = c->n;
        launch_gs_combine<double>(c->gs_nent, d.gs_kv, d.gs_mv, eps, mass, 1.0, d.gs_a64[k], c->stream);
        launch_gs_combine<double>(n, d.gs_kd, d.gs_md, eps, mass, 1.0, d.gs_d64[k], c->stream);
        if (c->precision == GSPM_MIXED) {
            // the FP32 operators' scaling: A' = A / len_scale^3
            const double ls = c->mv.len_scale, sc = 1.0 / (ls * ls * ls);
            launch_gs_combine<float>(c->gs_nent, d.gs_kv, d.gs_mv, eps, mass, sc, d.gs_a32[k], c->stream);
            launch_gs_combine<float>(n, d.gs_kd, d.gs_md, eps, mass, sc, d.gs_d32[k], c->stream);
        }
        c->gs_slot[k].valid = true;
        c->gs_slot[k].eps = eps;
        c->gs_slot[k].mass = mass;
    }
    c->gs_slot[k].used = ++c->gs_tick;
    GsRowsView v{d.gs_off, d.gs_col, nullptr, nullptr};
    if (fp32) {
        v.a = d.gs_a32[k];
        v.d = d.gs_d32[k];
    } else {
        v.a = d.gs_a64[k];
        v.d = d.gs_d64[k];
    }
    return v;
}

// The GS solves run single-reduction CG in row form (launch_gs_rows_cg): one
// launch per iteration, r, p and q alternating between two buffers.
CgResult cg_gs_run(gspm_ctx *c, int nc, double eps, double *x, const double *b, double tol, int maxit,
                   SolveKind kind) {
    hipStream_t s = c->stream;
    const bool jac = c->p.gs_precond == GSPM_PRECOND_JACOBI;
    const GsRowsView r64 = gs_rows(c, eps, 1.0, false);
    auto resid = [&]() {
        launch_gs_rows<double>(c->mv_rows, r64, nc, MV_RESID, x, nullptr, b, c->d.r, c->cg, s);
    };
    // iteration k reads the buffers of iteration k-1 and writes those of k
    auto fused = [&](const GsRowsView &rv, auto *R0, auto *R1, auto *P0, auto *P1, auto *Q0, auto *Q1, auto *xv,
                     const CGScalars &cg, double t) {
        return [=](int k, bool last) {
            auto *R = k & 1 ? R1 : R0, *P = k & 1 ? P1 : P0, *Q = k & 1 ? Q1 : Q0;
            auto *Rp = k & 1 ? R0 : R1, *Pp = k & 1 ? P0 : P1, *Qp = k & 1 ? Q0 : Q1;
            if (k == 0) Rp = R0;
            const hipEvent_t *ev = last ? nullptr : prof_begin(c, k);
            launch_gs_rows_cg(c->mv_rows, rv, nc, k, last, Rp, Pp, Qp, R, P, Q, xv, cg, t, jac, s, ev);
            if (!last) prof_end(c);
        };
    };
    auto &d = c->d;
    if (c->precision == GSPM_MIXED) {
        const double ls = c->mv.len_scale, scale = 1.0 / (ls * ls * ls);
        const GsRowsView r32 = gs_rows(c, eps, 1.0, true);
        return cg_mixed(c, nc, false, x, tol, maxit, kind, scale, resid,
                        fused(r32, d.r32, d.r32b, d.p32, d.p32b, d.q32, d.q32b, d.x32, c->cg_in, 1.0));
    }
    const size_t first_pair = prof_mark(c);
    CgResult res = cg_fp64(c, nc, false, x, tol, maxit, kind, resid,
                           fused(r64, d.r, d.r2, d.p, d.p2, d.q, d.q2, x, c->cg, tol));
    prof_drop_after(c, first_pair, std::max(res.iters[0], std::max(res.iters[1], res.iters[2])));
    return res;
}

// K^ms x = b (Eq. weak_demag) on the pinned all-element Laplacian.  The
// pinned node has b = 0 and x = 0, and its rows of K^ms are zero, so it stays
// zero.  One component (the step's solve) runs single-reduction CG, one fused
// launch per iteration as the elastic solve; several (gspm_solve) run the GS
// solves' two-launch form with per-component scalars.
CgResult cg_ms(gspm_ctx *c, int nc, double *x, const double *b, double tol, int maxit, SolveKind kind) {
    hipStream_t s = c->stream;
    auto resid = [&]() {
        launch_ms_matvec<double>(c->mv, nc, MV_RESID, x, nullptr, b, c->d.r, nullptr, c->cg, 0, tol, s);
    };
    if (nc == 1) {
        auto fused = [&](auto *R0, auto *R1, auto *P0, auto *P1, auto *Q0, auto *Q1, auto *xv, const CGScalars &cg,
                         double t) {
            return [=](int k, bool last) {
                auto *R = k & 1 ? R1 : R0, *P = k & 1 ? P1 : P0, *Q = k & 1 ? Q1 : Q0;
                auto *Rp = k & 1 ? R0 : R1, *Pp = k & 1 ? P0 : P1, *Qp = k & 1 ? Q0 : Q1;
                if (k == 0) Rp = R0;
                launch_ms_cg(c->mv, k, last, Rp, Pp, Qp, R, P, Q, xv, cg, t, s);
            };
        };
        auto &d = c->d;
        if (c->precision == GSPM_MIXED) {
            const double ls = c->mv.len_scale;
            return cg_mixed(c, 1, false, x, tol, maxit, kind, 1.0 / (ls * ls * ls), resid,
                            fused(d.r32, d.r32b, d.p32, d.p32b, d.q32, d.q32b, d.x32, c->cg_in, 1.0));
        }
        return cg_fp64(c, 1, false, x, tol, maxit, kind, resid, fused(d.r, d.r2, d.p, d.p2, d.q, d.q2, x, c->cg, tol));
    }
    if (c->precision == GSPM_MIXED) {
        float *P[2] = {c->d.p32, c->d.p32b};
        const double ls = c->mv.len_scale, scale = 1.0 / (ls * ls * ls);
        return cg_mixed(c, nc, false, x, tol, maxit, kind, scale, resid, [&](int k, bool last) {
            if (last) {
                launch_cg_check(nc, false, c->cg_in, k, 1.0, s);
                return;
            }
            launch_ms_matvec<float>(c->mv, nc, MV_ITER, P[k & 1], c->d.q32, nullptr, c->d.r32, P[(k + 1) & 1],
                                    c->cg_in, k, 1.0, s);
            launch_cg_update<float>(c->n, nc, false, c->d.x32, c->d.r32, P[(k + 1) & 1], c->d.q32, c->cg_in, k, s);
        });
    }
    double *P[2] = {c->d.p, c->d.p2};
    return cg_fp64(c, nc, false, x, tol, maxit, kind, resid, [&](int k, bool last) {
        if (last) {
            launch_cg_check(nc, false, c->cg, k, tol, s);
            return;
        }
        launch_ms_matvec<double>(c->mv, nc, MV_ITER, P[k & 1], c->d.q, nullptr, c->d.r, P[(k + 1) & 1], c->cg, k,
                                 tol, s);
        launch_cg_update<double>(c->n, nc, false, x, c->d.r, P[(k + 1) & 1], c->d.q, c->cg, k, s);
    });
}

namespace {

// One step of Algorithm B.1 (App. B) in the finite-element form of Eq.
// (weak_GS); (1 - eps lap)^-1 [y + c h] is the solution g of
// (eps K + M) g = M y + c M h with eps = l_ex^2 dtau.  Rows 1 and 2 of Step 2
// use m^n and g^n as printed, row 3 uses m* and g*; g* uses h[m^n];
// elasticity (and, with local_demag, the local magnetostatic potential of
// Eq. weak_demag) is solved once per step at m^n and held for h[m*].
int one_step(gspm_ctx *c, double dtau, double eps1, double eps3, gspm_step_stats *st) {
    auto &d = c->d;
    hipStream_t s = c->stream;
    const int n = c->n;
    const size_t bytes3 = sizeof(double) * 3 * static_cast<size_t>(n);
    const double tol = c->p.cg_tol;
    const int maxit = c->p.cg_maxit;
    // profile mode: event at each phase boundary (phase_ms of the statistics)
    auto mark = [&](int b) {
        if (c->profile) hipEventRecord(c->phase_ev[b], s);
    };
    mark(0);

    // volume averages at m^n: far field and homogeneous strain
    launch_avg_sums(n, d.w, d.m, c->mat, d.sums, s, c->mv.det);
    launch_derive(d.sums, c->dargs, &d.der[0], s);
    mark(1);

    // mechanical equilibrium at m^n, warm start from u^{n-1}
    hipMemcpyAsync(d.unext, d.u, bytes3, hipMemcpyDeviceToDevice, s);
    cg_prepare(c, 1);
    if (c->p.elastic_precond == GSPM_PRECOND_GREEN) {
        // the periodic system's right-hand side: nothing pinned
        MeshView mvu = c->mv;
        mvu.p0 = -1;
        launch_elastic_rhs(mvu, c->mat, d.m, d.b, d.unext, c->cg.bb, s);
    } else {
        launch_elastic_rhs(c->mv, c->mat, d.m, d.b, d.unext, c->cg.bb, s);
    }
    {
        const bool net = c->warm_mode == GSPM_WARM_LEARNED && c->have_prev;
        const bool extrap = c->warm_mode != GSPM_WARM_PREVIOUS && c->commits >= 2;
        if (net || extrap) {
            minres_start(c, d.m, net ? d.mprev : nullptr, extrap ? d.uprev : nullptr, d.unext, d.b);
            st->learned_starts += net;
            ++st->minres_starts;
        }
    }
    CgResult r = cg_elastic(c, d.unext, d.b, tol, maxit, SK_MECH);
    st->mech_iters += r.iters[0];
    if (r.status) return r.status;
    mark(2);

    // local magnetostatics at m^n, warm start from the previous potential
    const double *ud = nullptr;
    if (c->p.local_demag) {
        hipMemcpyAsync(d.udnext, d.ud, sizeof(double) * static_cast<size_t>(n), hipMemcpyDeviceToDevice, s);
        cg_prepare(c, 1);
        launch_ms_rhs(c->mv, c->p.Ms, d.m, d.b, d.udnext, c->cg.bb, s);
        r = cg_ms(c, 1, d.udnext, d.b, c->p.ms_tol > 0.0 ? c->p.ms_tol : std::max(1e-3 * tol, 1e-12), maxit, SK_MS);
        st->ms_iters += r.iters[0];
        if (r.status) return r.status;
        ud = d.udnext;
    }
    mark(3);
    const double inv_ms = 1.0 / c->p.Ms;

    // GS starts: the lumped solution the right-hand side kernels write, plus,
    // with the corrected start, the same stage's correction of the last step
    const bool corrected = c->gs_start == GSPM_GS_START_CORRECTED;
    auto gs_begin = [&](double *x, int nc, int stage) {
        if (!corrected) return;
        launch_gs_start(static_cast<int64_t>(nc) * n, x, d.gcorr + kGcorrOff[stage] * static_cast<int64_t>(n),
                        d.gstart, (c->gcorr_ok >> stage) & 1u, s);
    };
    auto gs_end = [&](const double *x, int nc, int stage, const CgResult &res) {
        if (!corrected) return;
        if (res.status) {
            c->gcorr_ok &= ~(1u << stage);
            return;
        }
        launch_gs_correction(static_cast<int64_t>(nc) * n, x, d.gstart,
                             d.gcorr + kGcorrOff[stage] * static_cast<int64_t>(n), (c->gcorr_ok >> stage) & 1u, s);
        c->gcorr_ok |= 1u << stage;
    };

    if (c->p.precession) {
        // Step 1: g^n, three components
        cg_prepare(c, 3);
        launch_field_rhs(c->mv, c->mat, d.m, d.unext, &d.der[0], dtau, d.b, d.g, d.ch2, c->cg.bb, kShards, ud,
                         inv_ms, s);
        gs_begin(d.g, 3, 0);
        r = cg_gs(c, 3, eps1, d.g, d.b, tol, maxit, SK_GS1);
        gs_end(d.g, 3, 0, r);
        for (int q = 0; q < 3; ++q) st->gs_iters_stage[q] += r.iters[q];
        if (r.status) return r.status;
        mark(4);
        // Step 2, rows 1 and 2
        launch_update_m12(n, d.m, d.g, d.ms, s);
        // Step 1: g* for components 1 and 2 with h[m^n]
        cg_prepare(c, 2);
        launch_mass_rhs(c->mv, d.ms, d.ch2, d.b, d.gs, c->cg.bb, kShards, s);
        gs_begin(d.gs, 2, 1);
        r = cg_gs(c, 2, eps1, d.gs, d.b, tol, maxit, SK_GS2);
        gs_end(d.gs, 2, 1, r);
        for (int q = 0; q < 2; ++q) st->gs_iters_stage[3 + q] += r.iters[q];
        if (r.status) return r.status;
        // Step 2, row 3
        launch_update_m3(n, d.m, d.gs, d.ms, s);
    } else {
        mark(4);
        hipMemcpyAsync(d.ms, d.m, bytes3, hipMemcpyDeviceToDevice, s);
    }
    mark(5);

    // Step 3: damped solve with h[m*], averages re-evaluated at m*
    launch_avg_sums(n, d.w, d.ms, c->mat, d.sums, s, c->mv.det);
    launch_derive(d.sums, c->dargs, &d.der[1], s);
    mark(6);
    cg_prepare(c, 3);
    launch_field_rhs(c->mv, c->mat, d.ms, d.unext, &d.der[1], c->p.alpha * dtau, d.b, d.g, nullptr, c->cg.bb,
                     kShards, ud, inv_ms, s);
    gs_begin(d.g, 3, 2);
    r = cg_gs(c, 3, eps3, d.g, d.b, tol, maxit, SK_GS3);
    gs_end(d.g, 3, 2, r);
    for (int q = 0; q < 3; ++q) st->gs_iters_stage[5 + q] += r.iters[q];
    if (r.status) return r.status;
    mark(7);

    // Step 4: unit length; the host reads the sum of |dm| and the failure flag
    launch_fill(d.dm, kShards, 0.0, s);
    launch_fill_i32(d.bad, 1, 0, s);
    launch_normalize(n, d.w, d.g, d.m, d.mnext, d.dm, d.bad, s, c->mv.det);
    ShardSources dms{};
    dms.p[0] = d.dm;
    launch_totals_to_host(dms, 1, c->h_step, s);
    launch_i32_to_host(d.bad, 1, reinterpret_cast<int32_t *>(c->h_step + 1), s);
    mark(8);
    int rc = hip_check(c, hipStreamSynchronize(s), "step");
    if (rc) return rc;
    if (c->profile) {
        for (int b = 0; b < 8; ++b) {
            float e = 0.0f;
            hipEventElapsedTime(&e, c->phase_ev[b], c->phase_ev[b + 1]);
            st->phase_ms[b] += e;
        }
    }
    if (*reinterpret_cast<const int32_t *>(c->h_step + 1)) {
        c->err = "zero or non-finite magnetisation after the damped solve";
        return GSPM_E_NONFINITE;
    }
    st->dm_avg = c->nmag > 0 ? c->h_step[0] / c->nmag : 0.0;
    // m^{n-1} <- m^n <- m^{n+1} and u^{n-2} <- u^{n-1} <- u^n: the old
    // buffers keep the previous states
    std::swap(d.mprev, d.m);
    std::swap(d.m, d.mnext);
    std::swap(d.uprev, d.u);
    std::swap(d.u, d.unext);
    if (ud) std::swap(d.ud, d.udnext);
    c->have_prev = true;
    ++c->commits;
    return GSPM_OK;
}

}  // namespace

int run_steps(gspm_ctx *c, double dt, int nsteps, gspm_step_stats *st) {
    std::memset(st, 0, sizeof *st);
    st->failed_step = -1;
    const double dtau = c->p.gamma0 * c->p.Ms * dt;
    const double lex2 = 2.0 * c->p.A / (c->p.mu0 * c->p.Ms * c->p.Ms);
    const double eps1 = lex2 * dtau, eps3 = c->p.alpha * eps1;
    for (auto &pl : c->prof) pl.used = 0;
    const int64_t ref0 = c->refinements, mref0 = c->mech_refinements;
    hipEventRecord(c->t0, c->stream);
    int rc = GSPM_OK;
    for (auto &v : c->last_res) v = 0.0;
    for (int step = 0; step < nsteps; ++step) {
        c->want_res = step == nsteps - 1;
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
    c->want_res = false;
    const SolveKind res_kind[5] = {SK_MECH, SK_GS1, SK_GS2, SK_GS3, SK_MS};
    for (int q = 0; q < 5; ++q) st->final_residual[q] = c->last_res[res_kind[q]];
    for (int q = 0; q < 8; ++q) st->gs_iters += st->gs_iters_stage[q];
    st->refinements = c->refinements - ref0;
    st->mech_refinements = c->mech_refinements - mref0;
    if (st->minres_starts > 0) hipMemcpy(st->warm_coef, c->d.wcoef, 2 * sizeof(double), hipMemcpyDeviceToHost);
    if (c->profile) {
        for (int li = 0; li < 2; ++li) {
            double tot = 0.0;
            int64_t cnt = 0;
            const auto &pl = c->prof[li];
            for (size_t i = 0; i + 1 < pl.used; i += 2) {
                if (pl.iter[i / 2] < 0) continue;
                float e = 0.0f;
                hipEventElapsedTime(&e, pl.ev[i], pl.ev[i + 1]);
                tot += e;
                ++cnt;
            }
            if (li == 0) {
                st->matvec_ms = tot;
                st->matvec_launches = cnt;
            } else {
                st->gs_matvec_ms = tot;
                st->gs_matvec_launches = cnt;
            }
        }
    }
    return rc;
}

}  // namespace gspm
