// Element passes of the GSPM step on gfx950.
//
// Every pass runs one 256-thread workgroup per owner block.  The block's
// threads stride over the block's element list (elements with at least one
// vertex in the block's node range), gather the vertex data from the SoA node
// arrays, recompute the P1 geometry from the coordinates, and add the
// contributions to owned vertices into LDS with ds_add_f64; halo vertices are
// dropped (their owner block computes the same element).  After one barrier
// each owned node is written once, coalesced, together with the fused
// epilogue of the pass (CG dot products, residuals, initial guesses).  No
// global atomics touch node data.
//
// Element arithmetic (Sec. 2.3, Eqs. LHS, RHS_F, RHS_b):
//   Laplacian  K^e_ij  = V g_i . g_j
//   mass       M^e_ij  = V (1 + delta_ij) / 20
//   elastic    (K^e u)_i = V sigma(u) g_i,  sigma = C sym(grad u), C cubic
//   elastic RHS b_i    = V (C <E0>_e) g_i,  <E0>_e the vertex mean of E0(m)
//   field RHS  b_i     = sum_j M^e_ij (y_j + c h^e_j)
// with h^e_j the local field of App. B at vertex j (anisotropy, Zeeman,
// far field, magnetoelastic with the element's total strain).
#include "device_common.h"

namespace gspm {

// ------------------------------------------------------------ the skeleton

template <class T, int NC>
__device__ __forceinline__ void scatter_owned(T *acc, int nb, int n0, const int4 c, const T (&y)[4][NC]) {
    const int v[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const unsigned loc = static_cast<unsigned>(v[j] - n0);
        if (loc < static_cast<unsigned>(nb)) {
#pragma unroll
            for (int k = 0; k < NC; ++k) atomicAdd(&acc[k * nb + loc], y[j][k]);
        }
    }
}

template <class T, int NC, class Op>
__global__ void __launch_bounds__(kThreads) k_elem(const MeshView<T> mv, const Op op_in) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *acc = reinterpret_cast<T *>(smem_raw);
    Op op = op_in;
    if (!op.prepare()) return;                 // uniform: e.g. every CG component converged
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int nb = mv.nb, n0 = b * nb;
    for (int i = threadIdx.x; i < NC * nb; i += kThreads) acc[i] = T(0);
    __syncthreads();
    const int e_beg = mv.blk_ptr[b];
    const int e_mag = e_beg + mv.blk_nmag[b];
    const int e_end = Op::kMagneticOnly ? e_mag : mv.blk_ptr[b + 1];
    for (int e = e_beg + static_cast<int>(threadIdx.x); e < e_end; e += kThreads) {
        const int4 c = mv.conn[e];
        Geo<T> G;
        tet_geometry(mv, c, G);
        T y[4][NC];
        op.element(c, G, e < e_mag, y);
        scatter_owned<T, NC>(acc, nb, n0, c, y);
    }
    __syncthreads();
    const int cnt = min(nb, mv.n - n0);
    op.finish(mv, n0, cnt, acc);
}

template <class T, int NC, class Op>
static void run_elem(const MeshView<T> &mv, const Op &op, hipStream_t s) {
    const size_t lds = sizeof(T) * NC * static_cast<size_t>(mv.nb);
    hipLaunchKernelGGL((k_elem<T, NC, Op>), dim3(mv.nblk), dim3(kThreads), lds, s, mv, op);
}

// --------------------------------------------------------- cubic material

template <class T>
struct Cubic {
    T c11, c12, c44;
    // sigma = C eps for symmetric eps given as (xx yy zz yz xz xy)
    __device__ __forceinline__ void stress(const T (&e)[6], T (&s)[6]) const {
        const T tr = e[0] + e[1] + e[2], d = c11 - c12;
        s[0] = d * e[0] + c12 * tr;
        s[1] = d * e[1] + c12 * tr;
        s[2] = d * e[2] + c12 * tr;
        s[3] = T(2) * c44 * e[3];
        s[4] = T(2) * c44 * e[4];
        s[5] = T(2) * c44 * e[5];
    }
};

// E0(m) of App. A: 3/2 [lambda100 (m_i^2 - 1/3); lambda111 m_i m_j]
template <class T>
__device__ __forceinline__ void spontaneous_strain(T l100, T l111, const T (&m)[3], T (&e)[6]) {
    const T a = T(1.5) * l100, b = T(1.5) * l111, third = T(1.0 / 3.0);
    e[0] = a * (m[0] * m[0] - third);
    e[1] = a * (m[1] * m[1] - third);
    e[2] = a * (m[2] * m[2] - third);
    e[3] = b * m[1] * m[2];
    e[4] = b * m[0] * m[2];
    e[5] = b * m[0] * m[1];
}

// y_j = S g_j for a symmetric S (xx yy zz yz xz xy), all four vertices
template <class T>
__device__ __forceinline__ void sym_times_grads(const T (&S)[6], const Geo<T> &G, T (&y)[4][3]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const T *g = G.g[j];
        y[j][0] = S[0] * g[0] + S[5] * g[1] + S[4] * g[2];
        y[j][1] = S[5] * g[0] + S[1] * g[1] + S[3] * g[2];
        y[j][2] = S[4] * g[0] + S[3] * g[1] + S[2] * g[2];
    }
}

// symmetric part of grad v = sum_{k=1..3} (v_k - v_0) (x) g_k
template <class T>
__device__ __forceinline__ void sym_grad(const T (&v)[4][3], const Geo<T> &G, T (&e)[6]) {
    T H[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T d1 = v[1][a] - v[0][a], d2 = v[2][a] - v[0][a], d3 = v[3][a] - v[0][a];
#pragma unroll
        for (int b = 0; b < 3; ++b) H[a][b] = d1 * G.g[1][b] + d2 * G.g[2][b] + d3 * G.g[3][b];
    }
    e[0] = H[0][0];
    e[1] = H[1][1];
    e[2] = H[2][2];
    e[3] = T(0.5) * (H[1][2] + H[2][1]);
    e[4] = T(0.5) * (H[0][2] + H[2][0]);
    e[5] = T(0.5) * (H[0][1] + H[1][0]);
}

template <class T>
__device__ __forceinline__ void gather3(const T *base, int n, const int4 c, T (&v)[4][3]) {
    const int id[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int a = 0; a < 3; ++a) v[j][a] = base[static_cast<size_t>(a) * n + id[j]];
}

// ------------------------------------------------------------- elasticity

// Matrix-free K^mech (Eq. LHS): y_i = V sigma(u) g_i over all elements.
// APPLY: out = K in.  ITER: out = q = K p, pq[k] += p.q.  RESID: r = p = b - K x,
// rr[0] += r.r.  Rows of the pinned node are zero.
template <class T>
struct ElasticMatvecOp {
    static constexpr bool kMagneticOnly = false;
    const T *in;
    T *out;
    const T *b;
    T *r, *p;
    CGScalars cg;
    int k, mode, n;
    Cubic<T> C;

    __device__ bool prepare() { return mode == MV_APPLY || cg.done[0] == 0; }

    __device__ __forceinline__ void element(const int4 c, const Geo<T> &G, bool, T (&y)[4][3]) const {
        T v[4][3], e[6], s[6];
        gather3(in, n, c, v);
        sym_grad(v, G, e);
        C.stress(e, s);
#pragma unroll
        for (int t = 0; t < 6; ++t) s[t] *= G.vol;
        sym_times_grads(s, G, y);
    }

    __device__ void finish(const MeshView<T> &mv, int n0, int cnt, const T *acc) const {
        double part = 0.0;
        for (int i = threadIdx.x; i < cnt; i += kThreads) {
            const int node = n0 + i;
            const bool pinned = node == mv.p0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const size_t o = static_cast<size_t>(a) * n + node;
                const T q = pinned ? T(0) : acc[a * mv.nb + i];
                if (mode == MV_RESID) {
                    const T rv = pinned ? T(0) : b[o] - q;
                    r[o] = rv;
                    p[o] = rv;
                    part += static_cast<double>(rv) * rv;
                } else {
                    out[o] = q;
                    if (mode == MV_ITER) part += static_cast<double>(in[o]) * q;
                }
            }
        }
        if (mode == MV_ITER) block_atomic_add1(part, cg.pq_at(0, k));
        else if (mode == MV_RESID) block_atomic_add1(part, cg.rr_at(0, 0));
    }
};

// Elastic right-hand side of Eq. (RHS_b): b_i = V (C <E0>_e) g_i on magnetic
// elements, <E0>_e the vertex mean of E0(m); zero on the pinned node, whose
// displacement is also set to zero; bb += b.b.
template <class T>
struct ElasticRhsOp {
    static constexpr bool kMagneticOnly = true;
    const T *m;
    T *b, *x;
    double *bb;
    int n;
    Cubic<T> C;
    T l100, l111;

    __device__ bool prepare() { return true; }

    __device__ __forceinline__ void element(const int4 c, const Geo<T> &G, bool, T (&y)[4][3]) const {
        T v[4][3], e0[6] = {0, 0, 0, 0, 0, 0};
        gather3(m, n, c, v);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            T ej[6];
            const T mj[3] = {v[j][0], v[j][1], v[j][2]};
            spontaneous_strain(l100, l111, mj, ej);
#pragma unroll
            for (int t = 0; t < 6; ++t) e0[t] += ej[t];
        }
#pragma unroll
        for (int t = 0; t < 6; ++t) e0[t] *= T(0.25);
        T s[6];
        C.stress(e0, s);
#pragma unroll
        for (int t = 0; t < 6; ++t) s[t] *= G.vol;
        sym_times_grads(s, G, y);
    }

    __device__ void finish(const MeshView<T> &mv, int n0, int cnt, const T *acc) const {
        double part = 0.0;
        for (int i = threadIdx.x; i < cnt; i += kThreads) {
            const int node = n0 + i;
            const bool pinned = node == mv.p0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const size_t o = static_cast<size_t>(a) * n + node;
                const T v = pinned ? T(0) : acc[a * mv.nb + i];
                b[o] = v;
                if (pinned) x[o] = T(0);
                part += static_cast<double>(v) * v;
            }
        }
        block_atomic_add1(part, bb);
    }
};

// ------------------------------------------------------------ GS operator

// (eps K + mass M) on NC scalar components stored [c][n], magnetic elements
// only (Eq. weak_GS).  Per-component CG: a converged component is skipped.
template <class T, int NC>
struct GsMatvecOp {
    static constexpr bool kMagneticOnly = true;
    const T *in;
    T *out;
    const T *b;
    T *r, *p;
    CGScalars cg;
    int k, mode, n;
    T eps, mass;
    int live[NC];

    __device__ bool prepare() {
        bool any = false;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            live[c] = (mode == MV_APPLY) ? 1 : (cg.done[c] == 0);
            any |= live[c] != 0;
        }
        return any;
    }

    __device__ __forceinline__ void element(const int4 c, const Geo<T> &G, bool, T (&y)[4][NC]) const {
        const int id[4] = {c.x, c.y, c.z, c.w};
        const T ev = eps * G.vol, mv20 = mass * G.vol * T(0.05);
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            if (!live[q]) {
#pragma unroll
                for (int j = 0; j < 4; ++j) y[j][q] = T(0);
                continue;
            }
            const T *src = in + static_cast<size_t>(q) * n;
            T v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = src[id[j]];
            const T d1 = v[1] - v[0], d2 = v[2] - v[0], d3 = v[3] - v[0];
            T gp[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) gp[a] = d1 * G.g[1][a] + d2 * G.g[2][a] + d3 * G.g[3][a];
            const T sum = v[0] + v[1] + v[2] + v[3];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                y[j][q] = ev * (G.g[j][0] * gp[0] + G.g[j][1] * gp[1] + G.g[j][2] * gp[2]) + mv20 * (v[j] + sum);
        }
    }

    __device__ void finish(const MeshView<T> &mv, int n0, int cnt, const T *acc) const {
        double part[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) part[q] = 0.0;
        for (int i = threadIdx.x; i < cnt; i += kThreads) {
            const int node = n0 + i;
#pragma unroll
            for (int q = 0; q < NC; ++q) {
                if (!live[q]) continue;
                const size_t o = static_cast<size_t>(q) * n + node;
                const T av = acc[q * mv.nb + i];
                if (mode == MV_RESID) {
                    const T rv = b[o] - av;
                    r[o] = rv;
                    p[o] = rv;
                    part[q] += static_cast<double>(rv) * rv;
                } else {
                    out[o] = av;
                    if (mode == MV_ITER) part[q] += static_cast<double>(in[o]) * av;
                }
            }
        }
        if (mode == MV_ITER) block_atomic_add<NC>(part, cg.pq_at(0, k), cg.comp_stride());
        else if (mode == MV_RESID) block_atomic_add<NC>(part, cg.rr_at(0, 0), cg.comp_stride());
    }
};

// ------------------------------------------------------------ field RHS

// Local field of App. B at one vertex (everything but exchange):
// h = -kan m_k (|m|^2 - m_k^2) + hc + kme sigma : dE0/dm_k, sigma = C (E - E0(m)).
template <class T>
__device__ __forceinline__ void local_field(const Cubic<T> &C, T l100, T l111, T kan, T kme, const T (&hc)[3],
                                            const T (&E)[6], const T (&m)[3], T (&h)[3]) {
    T e0[6], R[6], s[6];
    spontaneous_strain(l100, l111, m, e0);
#pragma unroll
    for (int t = 0; t < 6; ++t) R[t] = E[t] - e0[t];
    C.stress(R, s);
    const T m0s = m[0] * m[0], m1s = m[1] * m[1], m2s = m[2] * m[2];
    const T a = T(3) * kme * l100, b = T(3) * kme * l111;
    h[0] = -kan * m[0] * (m1s + m2s) + hc[0] + a * s[0] * m[0] + b * (s[5] * m[1] + s[4] * m[2]);
    h[1] = -kan * m[1] * (m0s + m2s) + hc[1] + a * s[1] * m[1] + b * (s[5] * m[0] + s[3] * m[2]);
    h[2] = -kan * m[2] * (m0s + m1s) + hc[2] + a * s[2] * m[2] + b * (s[4] * m[0] + s[3] * m[1]);
}

// b = M m + ch with ch = sum_e M^e (c h^e), per Eq. (RHS_b) with f = m + c h.
// Writes b, the initial guess x0 = m + ch / w (zero off the magnetic nodes),
// optionally ch's first two components, and bb[c] += b_c . b_c.
template <class T>
struct FieldRhsOp {
    static constexpr bool kMagneticOnly = true;
    const T *m, *u;
    const Derived *d;
    T *b, *x0, *ch2;
    double *bb;
    int n, bbstride;
    T c;
    Cubic<T> C;
    T l100, l111, kan, kme;
    T E0bar[6], hc[3];

    __device__ bool prepare() {
#pragma unroll
        for (int t = 0; t < 6; ++t) E0bar[t] = static_cast<T>(d->ebar[t]);
#pragma unroll
        for (int a = 0; a < 3; ++a) hc[a] = static_cast<T>(d->hc[a]);
        return true;
    }

    __device__ __forceinline__ void element(const int4 cn, const Geo<T> &G, bool, T (&y)[4][6]) const {
        T mv[4][3], uv[4][3], E[6];
        gather3(m, n, cn, mv);
        gather3(u, n, cn, uv);
        sym_grad(uv, G, E);
#pragma unroll
        for (int t = 0; t < 6; ++t) E[t] += E0bar[t];
        T f[4][3], sf[3] = {0, 0, 0}, sm[3] = {0, 0, 0};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const T mj[3] = {mv[j][0], mv[j][1], mv[j][2]};
            T h[3];
            local_field(C, l100, l111, kan, kme, hc, E, mj, h);
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                f[j][a] = c * h[a];
                sf[a] += f[j][a];
                sm[a] += mv[j][a];
            }
        }
        const T w20 = G.vol * T(0.05);
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                y[j][a] = w20 * (mv[j][a] + sm[a]);
                y[j][3 + a] = w20 * (f[j][a] + sf[a]);
            }
    }

    __device__ void finish(const MeshView<T> &mv, int n0, int cnt, const T *acc) const {
        double part[3] = {0.0, 0.0, 0.0};
        for (int i = threadIdx.x; i < cnt; i += kThreads) {
            const int node = n0 + i;
            const double w = mv.w[node];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const size_t o = static_cast<size_t>(a) * n + node;
                const T my = acc[a * mv.nb + i], chv = acc[(3 + a) * mv.nb + i];
                const T bv = my + chv;
                b[o] = bv;
                x0[o] = w > 0.0 ? m[o] + chv / static_cast<T>(w) : T(0);
                if (ch2 != nullptr && a < 2) ch2[o] = chv;
                part[a] += static_cast<double>(bv) * bv;
            }
        }
        block_atomic_add<3>(part, bb, bbstride);
    }
};

// b = M y + ch on the first two components (the g* solves of Algorithm B.1,
// Step 1, with h[m^n]); x0 = y + ch / w; bb[c] += b_c . b_c.
template <class T>
struct MassRhsOp {
    static constexpr bool kMagneticOnly = true;
    const T *y, *ch2;
    T *b, *x0;
    double *bb;
    int n, bbstride;

    __device__ bool prepare() { return true; }

    __device__ __forceinline__ void element(const int4 cn, const Geo<T> &G, bool, T (&out)[4][2]) const {
        const int id[4] = {cn.x, cn.y, cn.z, cn.w};
        const T w20 = G.vol * T(0.05);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            T v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = y[static_cast<size_t>(q) * n + id[j]];
            const T s = v[0] + v[1] + v[2] + v[3];
#pragma unroll
            for (int j = 0; j < 4; ++j) out[j][q] = w20 * (v[j] + s);
        }
    }

    __device__ void finish(const MeshView<T> &mv, int n0, int cnt, const T *acc) const {
        double part[2] = {0.0, 0.0};
        for (int i = threadIdx.x; i < cnt; i += kThreads) {
            const int node = n0 + i;
            const double w = mv.w[node];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const size_t o = static_cast<size_t>(q) * n + node;
                const T chv = ch2[o];
                const T bv = acc[q * mv.nb + i] + chv;
                b[o] = bv;
                x0[o] = w > 0.0 ? y[o] + chv / static_cast<T>(w) : T(0);
                part[q] += static_cast<double>(bv) * bv;
            }
        }
        block_atomic_add<2>(part, bb, bbstride);
    }
};

// ---------------------------------------------------------------- energies

// Element sums of the exchange energy A V |grad m|^2 (magnetic elements) and
// of the magnetoelastic energy V/4 sum_j 1/2 (E - chi E0(m_j)) : C (E - chi E0(m_j))
// (all elements).  Each element is counted by the block owning its smallest
// vertex id only.
template <class T>
__global__ void __launch_bounds__(kThreads) k_energy_elem(const MeshView<T> mv, Material mat, const T *m,
                                                          const T *u, const Derived *d, double *out) {
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int n0 = b * mv.nb, n1 = n0 + mv.nb;
    const Cubic<T> C{static_cast<T>(mat.c11), static_cast<T>(mat.c12), static_cast<T>(mat.c44)};
    T Eb[6];
#pragma unroll
    for (int t = 0; t < 6; ++t) Eb[t] = static_cast<T>(d->ebar[t]);
    double ex = 0.0, me = 0.0;
    const int e_beg = mv.blk_ptr[b], e_mag = e_beg + mv.blk_nmag[b], e_end = mv.blk_ptr[b + 1];
    for (int e = e_beg + static_cast<int>(threadIdx.x); e < e_end; e += kThreads) {
        const int4 c = mv.conn[e];
        const int vmin = min(min(c.x, c.y), min(c.z, c.w));
        if (vmin < n0 || vmin >= n1) continue;
        const bool mag = e < e_mag;
        Geo<T> G;
        tet_geometry(mv, c, G);
        T mv4[4][3], uv[4][3], E[6];
        gather3(m, mv.n, c, mv4);
        gather3(u, mv.n, c, uv);
        sym_grad(uv, G, E);
#pragma unroll
        for (int t = 0; t < 6; ++t) E[t] += Eb[t];
        if (mag) {
            double g2 = 0.0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const T d1 = mv4[1][a] - mv4[0][a], d2 = mv4[2][a] - mv4[0][a], d3 = mv4[3][a] - mv4[0][a];
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    const double gq = d1 * G.g[1][q] + d2 * G.g[2][q] + d3 * G.g[3][q];
                    g2 += gq * gq;
                }
            }
            ex += mat.A * static_cast<double>(G.vol) * g2;
        }
        double el = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            T R[6], s[6];
            if (mag) {
                const T mj[3] = {mv4[j][0], mv4[j][1], mv4[j][2]};
                T e0[6];
                spontaneous_strain(static_cast<T>(mat.l100), static_cast<T>(mat.l111), mj, e0);
#pragma unroll
                for (int t = 0; t < 6; ++t) R[t] = E[t] - e0[t];
            } else {
#pragma unroll
                for (int t = 0; t < 6; ++t) R[t] = E[t];
            }
            C.stress(R, s);
            el += 0.5 * (R[0] * s[0] + R[1] * s[1] + R[2] * s[2] + T(2) * (R[3] * s[3] + R[4] * s[4] + R[5] * s[5]));
        }
        me += 0.25 * static_cast<double>(G.vol) * el;
    }
    const double v2[2] = {ex, me};
    block_atomic_add<2>(v2, out, kShards);
}

// --------------------------------------------------------------- launchers

namespace {
template <class T>
Cubic<T> cubic_of(const Material &m) {
    return Cubic<T>{static_cast<T>(m.c11), static_cast<T>(m.c12), static_cast<T>(m.c44)};
}
}  // namespace

void launch_elastic_matvec(const MeshView<double> &mv, const Material &mat, MatvecMode mode, const double *in,
                           double *out, const double *b, double *r, double *p, const CGScalars &cg, int k,
                           hipStream_t s) {
    ElasticMatvecOp<double> op{in, out, b, r, p, cg, k, static_cast<int>(mode), mv.n, cubic_of<double>(mat)};
    run_elem<double, 3>(mv, op, s);
}

void launch_elastic_rhs(const MeshView<double> &mv, const Material &mat, const double *m, double *b, double *x,
                        double *bb, hipStream_t s) {
    ElasticRhsOp<double> op{m, b, x, bb, mv.n, cubic_of<double>(mat), mat.l100, mat.l111};
    run_elem<double, 3>(mv, op, s);
}

void launch_gs_matvec(const MeshView<double> &mv, int nc, double eps, double mass, MatvecMode mode,
                      const double *in, double *out, const double *b, double *r, double *p, const CGScalars &cg,
                      int k, hipStream_t s) {
    switch (nc) {
        case 1: run_elem<double, 1>(mv, GsMatvecOp<double, 1>{in, out, b, r, p, cg, k, static_cast<int>(mode), mv.n, eps, mass, {0}}, s); break;
        case 2: run_elem<double, 2>(mv, GsMatvecOp<double, 2>{in, out, b, r, p, cg, k, static_cast<int>(mode), mv.n, eps, mass, {0, 0}}, s); break;
        default: run_elem<double, 3>(mv, GsMatvecOp<double, 3>{in, out, b, r, p, cg, k, static_cast<int>(mode), mv.n, eps, mass, {0, 0, 0}}, s); break;
    }
}

void launch_field_rhs(const MeshView<double> &mv, const Material &mat, const double *m, const double *u,
                      const Derived *d, double c, double *b, double *x0, double *ch2, double *bb, int bbstride,
                      hipStream_t s) {
    FieldRhsOp<double> op{m, u, d, b, x0, ch2, bb, mv.n, bbstride, c, cubic_of<double>(mat), mat.l100, mat.l111,
                          mat.kan, mat.kme, {0, 0, 0, 0, 0, 0}, {0, 0, 0}};
    run_elem<double, 6>(mv, op, s);
}

void launch_mass_rhs(const MeshView<double> &mv, const double *y, const double *ch2, double *b, double *x0,
                     double *bb, int bbstride, hipStream_t s) {
    MassRhsOp<double> op{y, ch2, b, x0, bb, mv.n, bbstride};
    run_elem<double, 2>(mv, op, s);
}

void launch_energy_elem(const MeshView<double> &mv, const Material &mat, const double *m, const double *u,
                        const Derived *d, double *out2, hipStream_t s) {
    hipLaunchKernelGGL(k_energy_elem<double>, dim3(mv.nblk), dim3(kThreads), 0, s, mv, mat, m, u, d, out2);
}

}  // namespace gspm
