// The GS operator eps K + mass M (Eq. weak_GS, magnetic elements) in row form.
//
// One 256-thread workgroup per owner block, one thread per owned row (a
// wavefront covers one 64-row slice).
//   1. Staging: the block's node set (owned range, then halo list) is copied
//      into LDS as one short vector per node holding the NC components of the
//      operand; in a CG iteration the operand is the new direction
//      p_k = z_k + beta p_{k-1}, formed here for owned and halo nodes alike
//      from the previous iteration's r, p and q.
//   2. Rows: each thread walks its row's entries (column index and
//      coefficient, coalesced across the wavefront by the entry-major slice
//      layout), reads the staged vector of the column and accumulates in
//      registers.  The order of the sum is fixed by the layout, so the result
//      does not depend on scheduling.
//   3. Epilogue: the fused work (residuals, CG vectors and dot products),
//      written once per owned node, coalesced.
// The coefficients are the assembled P1 element matrices (Sec. 2.3) of the
// host's upload pass; a slot caches A = eps K + mass M for each (eps, mass)
// in use, rebuilt on the device when the pair changes.
#include <hip/hip_ext.h>

#include "device_common.h"

namespace gspm {

// the staged vector of a node: NC components, padded to 4 for NC = 3 so one
// wide LDS read fetches it
template <class T, int NC>
struct RowVec {
    static constexpr int kPad = NC == 3 ? 4 : NC;
    T v[kPad];
};

template <class T, int NC>
struct GsRowArgs {
    const T *in;
    T *out;
    const T *b;
    T *r;
    CGScalars cg;
    int mode, n;
};

// APPLY: out = A in.  RESID: r = b - A in on the components not yet
// converged, with r.r into slot 0 of the r.r ring.
template <class T, int NC>
__global__ void __launch_bounds__(kThreads) k_gs_rows(const MeshView mv, const GsRowsView rv, const GsRowArgs<T, NC> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    using V = RowVec<T, NC>;
    V *f = reinterpret_cast<V *>(smem_raw);
    const int b = xcd_block(blockIdx.x, gridDim.x);
    int live[NC];
    bool any = false;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        live[c] = (a.mode == MV_APPLY) ? 1 : (a.cg.done[c] == 0);
        any |= live[c] != 0;
    }
    if (!any) return;
    const T *A = static_cast<const T *>(rv.a), *D = static_cast<const T *>(rv.d);
    const int nb = mv.nb, n0 = b * nb, cnt = min(nb, mv.n - n0), n = a.n;
    const int hbeg = mv.halo_ptr[b], nloc = nb + (mv.halo_ptr[b + 1] - hbeg);
    // staging, four nodes per thread at a time (index loads, then data loads,
    // then LDS stores) to keep the halo's dependent loads in flight
    constexpr int kU = 4;
    for (int l0 = threadIdx.x; l0 < nloc; l0 += kU * kThreads) {
        int ls[kU], gs[kU];
        bool ok[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            ls[u] = l0 + u * kThreads;
            ok[u] = ls[u] < nloc && !(ls[u] >= cnt && ls[u] < nb);
            gs[u] = !ok[u] ? n0 : (ls[u] < nb ? n0 + ls[u] : mv.halo_ids[hbeg + ls[u] - nb]);
        }
        V v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
#pragma unroll
            for (int q = 0; q < V::kPad; ++q) v[u].v[q] = T(0);
#pragma unroll
            for (int q = 0; q < NC; ++q)
                if (live[q]) v[u].v[q] = a.in[static_cast<size_t>(q) * n + gs[u]];
        }
#pragma unroll
        for (int u = 0; u < kU; ++u)
            if (ok[u]) f[ls[u]] = v[u];
    }
    __syncthreads();
    double part[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) part[q] = 0.0;
    for (int i = threadIdx.x; i < cnt; i += kThreads) {
        const int g = n0 + i, sl = g >> 6, lane = g & 63;
        const V own = f[i];
        const T dg = D[g];
        T acc[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) acc[q] = dg * own.v[q];
        const int beg = rv.off[sl] + lane, w = (rv.off[sl + 1] - rv.off[sl]) >> 6;
        const uint16_t *cp = rv.col + beg;
        const T *ap = A + beg;
#pragma unroll 4
        for (int e = 0; e < w; ++e) {
            const int c = cp[64 * e];
            const T av = ap[64 * e];
            const V x = f[c];
#pragma unroll
            for (int q = 0; q < NC; ++q) acc[q] += av * x.v[q];
        }
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            if (!live[q]) continue;
            const size_t o = static_cast<size_t>(q) * n + g;
            if (a.mode == MV_RESID) {
                const T rvv = a.b[o] - acc[q];
                a.r[o] = rvv;
                part[q] += static_cast<double>(rvv) * rvv;
            } else {
                a.out[o] = acc[q];
            }
        }
    }
    if (a.mode == MV_RESID) block_atomic_add<NC>(part, a.cg.rr_at(0, 0), a.cg.comp_stride(), a.cg.det);
}

template <class T, int NC>
static void run_rows(const MeshView &mv, const GsRowsView &rv, const GsRowArgs<T, NC> &a, hipStream_t s) {
    const size_t lds = sizeof(RowVec<T, NC>) * static_cast<size_t>(mv.nloc_max);
    hipLaunchKernelGGL((k_gs_rows<T, NC>), dim3(mv.nblk), dim3(kThreads), lds, s, mv, rv, a);
    launch_det_finish(a.cg.det, s);
}

template <class T>
void launch_gs_rows(const MeshView &mv, const GsRowsView &rv, int nc, MatvecMode mode, const T *in, T *out,
                    const T *b, T *r, const CGScalars &cg, hipStream_t s) {
    const int md = static_cast<int>(mode);
    switch (nc) {
        case 1: run_rows<T, 1>(mv, rv, GsRowArgs<T, 1>{in, out, b, r, cg, md, mv.n}, s); break;
        case 2: run_rows<T, 2>(mv, rv, GsRowArgs<T, 2>{in, out, b, r, cg, md, mv.n}, s); break;
        default: run_rows<T, 3>(mv, rv, GsRowArgs<T, 3>{in, out, b, r, cg, md, mv.n}, s); break;
    }
}

template void launch_gs_rows<double>(const MeshView &, const GsRowsView &, int, MatvecMode, const double *, double *,
                                     const double *, double *, const CGScalars &, hipStream_t);
template void launch_gs_rows<float>(const MeshView &, const GsRowsView &, int, MatvecMode, const float *, float *,
                                    const float *, float *, const CGScalars &, hipStream_t);

// ------------------------------------------- single-reduction GS iteration

// One launch per CG iteration on the GS operator (NC independent components,
// Jacobi-preconditioned or plain; D = I for plain CG).  Launch k completes
// iteration k-1 from the sums its epilogue left, per component:
//   alpha = rz_{k-1} / (p.q),  rz = r . D^-1 r (true, r = r_{k-1}),
//   beta  = rz~_k / rz_{k-1},  rz~_k = rz_{k-1} - 2 alpha (r.D^-1 q) + alpha^2 (q.D^-1 q)
// (the expansion of r_k . D^-1 r_k with r_k = r_{k-1} - alpha q_{k-1}: it only
// sets the direction; the step length uses the true rz and the stopping test
// the true |r|, one launch later).  While staging it forms r_k, z_k = D^-1 r_k
// and p_k = z_k + beta p_{k-1} for owned and halo nodes, stores r_k and adds
// alpha p_{k-1} to x on owned nodes, then computes q_k = A p_k in row form
// and the sums of iteration k.  r, p and q alternate between two buffers.
// The launch that finds |r_{k-1}| converged records it (x_{k-1} is the
// answer); the launch after the last permitted iteration only adds the
// pending step.
template <class T, int NC>
struct GsCgArgs {
    const T *rin, *pin, *qin;     // r_{k-1}, p_{k-1}, q_{k-1} (rin = r_0 at k = 0)
    T *rout, *pout, *qout;        // r_k, p_k, q_k
    T *x;
    CGScalars cg;
    int k, n, last;
    double tol2;
    bool jacobi;
};

// the owned node's r_k, D and 1 / D, kept for the rows and the epilogue
template <class T, int NC>
struct RowOwn {
    T r[NC];
    T d, dinv;
};

// Launch structure (every load that does not depend on the iteration's
// scalars is in flight before they are summed):
//   1. the done flags (a converged solve makes later launches exit here);
//   2. loads of the previous iteration's sums (spread over the workgroup),
//      of the owned nodes' r, q, p, x and D, of the first batch of halo
//      indices and then halo r, q, p and D, and of the first kE entries of
//      each row;
//   3. the sums' totals (convergence test, alpha, beta);
//   4. r_k, z_k, p_k for owned and halo nodes into LDS (owned: r_k and x to
//      memory), then the rows and the epilogue.
template <class T, int NC>
__global__ void __launch_bounds__(kThreads) k_gs_rows_cg(const MeshView mv, const GsRowsView rv,
                                                         const GsCgArgs<T, NC> a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    using V = RowVec<T, NC>;
    using O = RowOwn<T, NC>;
    constexpr int kNS = 6 * NC;                 // sums read per launch: rr pq rz rzq qzq bb per component
    constexpr int kSh = (kNS * kShards + kThreads - 1) / kThreads;
    constexpr int kU = 2;                       // halo nodes per thread per batch
    constexpr int kE = (sizeof(T) == 4 && NC == 3) ? 16 : 8;   // row entries per batch (prefetch fits the VGPR budget of 4 waves/SIMD)
    __shared__ int32_t sflags[NC];
    __shared__ double sred[kNS * kShards];
    __shared__ double stot[kNS];
    V *f = reinterpret_cast<V *>(smem_raw);
    O *own = reinterpret_cast<O *>(f + mv.nloc_max);
    const int b = xcd_block(blockIdx.x, gridDim.x), tid = threadIdx.x;
    const int k = a.k, n = a.n;
    // 1. flags
    if (tid == 0)
        for (int q = 0; q < NC; ++q) sflags[q] = a.cg.done[q];
    __syncthreads();
    int live[NC];
    bool any = false;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        live[q] = sflags[q] == 0;
        any |= live[q] != 0;
    }
    if (!any || (a.last && k == 0)) return;   // (the start test ran in an earlier launch)
    const T *A = static_cast<const T *>(rv.a), *D = static_cast<const T *>(rv.d);
    const int nb = mv.nb, n0 = b * nb, cnt = min(nb, mv.n - n0);
    const int hbeg = mv.halo_ptr[b], nhalo = mv.halo_ptr[b + 1] - hbeg;
    // 2. loads
    double shv[kSh];
#pragma unroll
    for (int j = 0; j < kSh; ++j) {
        const int t = tid + j * kThreads, v = t / kShards, sh = t % kShards, q = v % NC;
        shv[j] = 0.0;
        if (k > 0 && t < kNS * kShards) {
            const int kind = v / NC;
            const double *src = kind == 0 ? a.cg.rr_at(q, k - 1) : kind == 1 ? a.cg.pq_at(q, k - 1)
                              : kind == 2 ? a.cg.rz_at(q, k - 1) : kind == 3 ? a.cg.rzq_at(q, k - 1)
                              : kind == 4 ? a.cg.qzq_at(q, k - 1) : a.cg.bb_at(q);
            shv[j] = src[sh];
        }
    }
    // owned node tid (the first of the thread's owned nodes); the loads are
    // unconditional so they stay in flight together (unused values: q, p, x
    // at k = 0).  A component that converged in an earlier launch reads
    // element 0 on every lane (one cached line) instead of its vectors.
    const bool has_own = tid < cnt;
    const int go = n0 + (has_own ? tid : 0);
    auto at = [&](int q, int node) -> size_t { return live[q] ? static_cast<size_t>(q) * n + node : 0; };
    T orr[NC], oq[NC], op[NC], ox[NC];
    const T od = D[go];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        const size_t o = at(q, go);
        orr[q] = a.rin[o];
        oq[q] = a.qin[o];
        op[q] = a.pin[o];
        ox[q] = a.x[o];
    }
    int gs[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int h = tid + u * kThreads;
        gs[u] = h < nhalo ? mv.halo_ids[hbeg + h] : n0;
    }
    // the first kE entries of row tid
    const int gr = n0 + (has_own ? tid : 0), sl = gr >> 6, lane = gr & 63;
    const int rbeg = rv.off[sl] + lane, w = (rv.off[sl + 1] - rv.off[sl]) >> 6;
    int pc[kE];
    T pa[kE];
#pragma unroll
    for (int u = 0; u < kE; ++u) {
        const bool in = u < w;
        pc[u] = in ? rv.col[rbeg + 64 * u] : 0;
        pa[u] = in ? A[rbeg + 64 * u] : T(0);
    }
    T hr[kU][NC], hq[kU][NC], hp[kU][NC], hd[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        hd[u] = D[gs[u]];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const size_t o = at(q, gs[u]);
            hr[u][q] = a.rin[o];
            hq[u][q] = a.qin[o];
            hp[u][q] = a.pin[o];
        }
    }
    // 3. totals of the previous iteration's sums
    double alpha[NC], beta[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) alpha[q] = beta[q] = 0.0;
    if (k > 0) {
#pragma unroll
        for (int j = 0; j < kSh; ++j) {
            const int t = tid + j * kThreads;
            if (t < kNS * kShards) sred[t] = shv[j];
        }
        __syncthreads();
        if (tid < kNS) {
            double sum = 0.0;
            for (int sh = 0; sh < kShards; ++sh) sum += sred[tid * kShards + sh];
            stot[tid] = sum;
        }
        __syncthreads();
        int stop[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            stop[q] = 0;
            if (!live[q]) continue;
            const double rrp = stot[q], pq = stot[NC + q], rz = stot[2 * NC + q];
            if (!isfinite(rrp)) stop[q] = 2;
            else if (rrp <= a.tol2 * stot[5 * NC + q]) stop[q] = 1;
            if (stop[q]) {
                live[q] = 0;
                continue;
            }
            alpha[q] = rz / pq;
            const double est = rz - 2.0 * alpha[q] * stot[3 * NC + q] + alpha[q] * alpha[q] * stot[4 * NC + q];
            beta[q] = (est > 0.0 ? est : 0.0) / rz;
        }
        if (b == 0 && tid == 0)
            for (int q = 0; q < NC; ++q)
                if (stop[q]) {
                    a.cg.done[q] = stop[q];
                    a.cg.iters[q] = k - 1;
                }
        any = false;
#pragma unroll
        for (int q = 0; q < NC; ++q) any |= live[q] != 0;
        if (!any) return;
        if (a.last) {
            for (int i = tid; i < cnt; i += kThreads)
#pragma unroll
                for (int q = 0; q < NC; ++q) {
                    if (!live[q]) continue;
                    const size_t o = static_cast<size_t>(q) * n + n0 + i;
                    a.x[o] += static_cast<T>(alpha[q]) * a.pin[o];
                }
            return;
        }
    }
    T al[NC], bt[NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        al[q] = static_cast<T>(alpha[q]);
        bt[q] = static_cast<T>(beta[q]);
    }
    // 4. r_k = r_{k-1} - alpha q_{k-1}, z_k = D^-1 r_k, p_k = z_k + beta p_{k-1}
    auto direction = [&](const T (&r)[NC], const T (&qv)[NC], const T (&pv)[NC], T d, T (&rk)[NC], T &dinv) {
        dinv = !a.jacobi ? T(1) : (d > T(0) ? T(1) / d : T(0));
        V v;
#pragma unroll
        for (int q = 0; q < V::kPad; ++q) v.v[q] = T(0);
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            rk[q] = (live[q] && k > 0) ? r[q] - al[q] * qv[q] : r[q];
            const T z = rk[q] * dinv;
            v.v[q] = !live[q] ? T(0) : (k > 0 ? z + bt[q] * pv[q] : z);
        }
        return v;
    };
    auto owned_node = [&](int i, const T (&r)[NC], const T (&qv)[NC], const T (&pv)[NC], const T (&xv)[NC], T d) {
        O ow;
        ow.d = d;
        f[i] = direction(r, qv, pv, d, ow.r, ow.dinv);
        own[i] = ow;
        if (k == 0) return;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            if (!live[q]) continue;
            const size_t o = static_cast<size_t>(q) * n + n0 + i;
            a.rout[o] = ow.r[q];
            a.x[o] = xv[q] + al[q] * pv[q];
        }
    };
    if (has_own) owned_node(tid, orr, oq, op, ox, od);
    for (int i = tid + kThreads; i < cnt; i += kThreads) {   // blocks of more than kThreads nodes
        T r[NC], qv[NC], pv[NC], xv[NC];
        const T d = D[n0 + i];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const size_t o = at(q, n0 + i);
            r[q] = a.rin[o];
            qv[q] = a.qin[o];
            pv[q] = a.pin[o];
            xv[q] = a.x[o];
        }
        owned_node(i, r, qv, pv, xv, d);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const int h = tid + u * kThreads;
        if (h >= nhalo) continue;
        T rk[NC], dinv;
        f[nb + h] = direction(hr[u], hq[u], hp[u], hd[u], rk, dinv);
    }
    for (int h = tid + kU * kThreads; h < nhalo; h += kThreads) {   // halo lists longer than one batch
        const int g = mv.halo_ids[hbeg + h];
        T r[NC], qv[NC], pv[NC];
        const T d = D[g];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const size_t o = at(q, g);
            r[q] = a.rin[o];
            qv[q] = a.qin[o];
            pv[q] = a.pin[o];
        }
        T rk[NC], dinv;
        f[nb + h] = direction(r, qv, pv, d, rk, dinv);
    }
    __syncthreads();
    // rows: q_k = A p_k; sums per component: p.q, r.r, r.D^-1 r, r.D^-1 q, q.D^-1 q
    double part[5 * NC];
#pragma unroll
    for (int j = 0; j < 5 * NC; ++j) part[j] = 0.0;
    for (int i = tid; i < cnt; i += kThreads) {
        const int g = n0 + i, sli = g >> 6, ln = g & 63;
        const int beg = rv.off[sli] + ln, wi = (rv.off[sli + 1] - rv.off[sli]) >> 6;
        const V pk = f[i];
        const O ow = own[i];
        T acc[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) acc[q] = ow.d * pk.v[q];
        int e0 = 0;
        if (i == tid) {   // the prefetched entries
#pragma unroll
            for (int u = 0; u < kE; ++u) {
                const V xv = f[u < wi ? pc[u] : i];
#pragma unroll
                for (int q = 0; q < NC; ++q) acc[q] += pa[u] * xv.v[q];
            }
            e0 = kE;
        }
        for (; e0 < wi; e0 += kE) {
            int c[kE];
            T av[kE];
#pragma unroll
            for (int u = 0; u < kE; ++u) {
                const bool in = e0 + u < wi;
                c[u] = in ? rv.col[beg + 64 * (e0 + u)] : i;
                av[u] = in ? A[beg + 64 * (e0 + u)] : T(0);
            }
#pragma unroll
            for (int u = 0; u < kE; ++u) {
                const V xv = f[c[u]];
#pragma unroll
                for (int q = 0; q < NC; ++q) acc[q] += av[u] * xv.v[q];
            }
        }
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            if (!live[q]) continue;
            const size_t o = static_cast<size_t>(q) * n + g;
            a.pout[o] = pk.v[q];
            a.qout[o] = acc[q];
            const double r = ow.r[q], qq = acc[q], di = ow.dinv;
            part[q] += static_cast<double>(pk.v[q]) * qq;
            part[NC + q] += r * r;
            part[2 * NC + q] += r * (di * r);
            part[3 * NC + q] += r * (di * qq);
            part[4 * NC + q] += qq * (di * qq);
        }
    }
    double *dst[5 * NC];
#pragma unroll
    for (int q = 0; q < NC; ++q) {
        const bool on = live[q] != 0;
        dst[q] = on ? a.cg.pq_at(q, k) : nullptr;
        dst[NC + q] = (on && k > 0) ? a.cg.rr_at(q, k) : nullptr;   // |r_0|^2 is in slot 0 already
        dst[2 * NC + q] = on ? a.cg.rz_at(q, k) : nullptr;
        dst[3 * NC + q] = on ? a.cg.rzq_at(q, k) : nullptr;
        dst[4 * NC + q] = on ? a.cg.qzq_at(q, k) : nullptr;
    }
    block_atomic_add_to<5 * NC>(part, dst, a.cg.det);
}

template <class T, int NC>
static void run_rows_cg(const MeshView &mv, const GsRowsView &rv, const GsCgArgs<T, NC> &a, hipStream_t s,
                        const hipEvent_t *ev) {
    const size_t lds = sizeof(RowVec<T, NC>) * static_cast<size_t>(mv.nloc_max) +
                       sizeof(RowOwn<T, NC>) * static_cast<size_t>(mv.nb);
    if (ev)
        hipExtLaunchKernelGGL((k_gs_rows_cg<T, NC>), dim3(mv.nblk), dim3(kThreads), lds, s, ev[0], ev[1], 0, mv, rv, a);
    else
        hipLaunchKernelGGL((k_gs_rows_cg<T, NC>), dim3(mv.nblk), dim3(kThreads), lds, s, mv, rv, a);
    launch_det_finish(a.cg.det, s);
}

size_t rows_lds_bytes(int32_t nb, int32_t nloc_max, bool fp64_cg) {
    const size_t nl = static_cast<size_t>(nloc_max), b = static_cast<size_t>(nb);
    size_t need = sizeof(RowVec<double, 3>) * nl;                                           // FP64 residuals
    need = std::max(need, sizeof(RowVec<float, 3>) * nl + sizeof(RowOwn<float, 3>) * b);  // FP32 CG
    if (fp64_cg) need = std::max(need, sizeof(RowVec<double, 3>) * nl + sizeof(RowOwn<double, 3>) * b);
    return need + 8192;   // the CG kernel's static arrays
}

template <class T>
void launch_gs_rows_cg(const MeshView &mv, const GsRowsView &rv, int nc, int k, bool last, const T *rin, const T *pin,
                       const T *qin, T *rout, T *pout, T *qout, T *x, const CGScalars &cg, double tol, bool jacobi,
                       hipStream_t s, const hipEvent_t *ev) {
    const double t2 = tol * tol;
    const int l = last ? 1 : 0;
    switch (nc) {
        case 1: run_rows_cg<T, 1>(mv, rv, GsCgArgs<T, 1>{rin, pin, qin, rout, pout, qout, x, cg, k, mv.n, l, t2, jacobi}, s, ev); break;
        case 2: run_rows_cg<T, 2>(mv, rv, GsCgArgs<T, 2>{rin, pin, qin, rout, pout, qout, x, cg, k, mv.n, l, t2, jacobi}, s, ev); break;
        default: run_rows_cg<T, 3>(mv, rv, GsCgArgs<T, 3>{rin, pin, qin, rout, pout, qout, x, cg, k, mv.n, l, t2, jacobi}, s, ev); break;
    }
}

template void launch_gs_rows_cg<double>(const MeshView &, const GsRowsView &, int, int, bool, const double *,
                                        const double *, const double *, double *, double *, double *, double *,
                                        const CGScalars &, double, bool, hipStream_t, const hipEvent_t *);
template void launch_gs_rows_cg<float>(const MeshView &, const GsRowsView &, int, int, bool, const float *,
                                       const float *, const float *, float *, float *, float *, float *,
                                       const CGScalars &, double, bool, hipStream_t, const hipEvent_t *);

template <class T>
__global__ void __launch_bounds__(kThreads) k_gs_combine(int64_t count, const double *kv, const double *mv, double eps,
                                                         double mass, double scale, T *out) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < count;
         i += static_cast<int64_t>(gridDim.x) * kThreads)
        out[i] = static_cast<T>(scale * (eps * kv[i] + mass * mv[i]));
}

template <class T>
void launch_gs_combine(int64_t count, const double *kv, const double *mv, double eps, double mass, double scale,
                       T *out, hipStream_t s) {
    if (count <= 0) return;
    const int64_t want = (count + kThreads - 1) / kThreads;
    const int grid = static_cast<int>(want < 4096 ? want : 4096);
    hipLaunchKernelGGL(k_gs_combine<T>, dim3(grid), dim3(kThreads), 0, s, count, kv, mv, eps, mass, scale, out);
}

template void launch_gs_combine<double>(int64_t, const double *, const double *, double, double, double, double *,
                                        hipStream_t);
template void launch_gs_combine<float>(int64_t, const double *, const double *, double, double, double, float *,
                                       hipStream_t);

}  // namespace gspm
