// Element passes of the GSPM step on gfx950.
//
// One 256-thread workgroup per owner block (a Morton range of nb nodes).
//   1. Staging: the block's node set -- its owned range followed by its halo
//      list (the other vertices of its elements) -- is copied into LDS once:
//      coordinates, shifted to the nearest periodic image of the block's first
//      node, and the field values the pass reads.  Owned nodes are a
//      contiguous, coalesced range; each halo node is fetched once per block
//      instead of once per element vertex.
//   2. Element loop: threads stride over the block's element copies (16-bit
//      local vertex indices), recompute the P1 geometry from the staged
//      coordinates, and add the contributions to owned vertices into LDS
//      accumulators with ds_add_f64 / ds_add_f32.  Contributions to halo
//      vertices are dropped: the halo node's owner block computes the same
//      element.
//   3. Epilogue: each owned node is written once, coalesced, with the pass's
//      fused work (CG dot products, residuals, initial guesses).
// No global atomics touch node data.
//
// Element arithmetic (Sec. 2.3, Eqs. LHS, RHS_F, RHS_b):
//   Laplacian   K^e_ij  = V g_i . g_j
//   mass        M^e_ij  = V (1 + delta_ij) / 20
//   elastic     (K^e u)_i = V sigma(u) g_i,  sigma = C sym(grad u), C cubic
//   elastic RHS b_i     = V (C <E0>_e) g_i,  <E0>_e the vertex mean of E0(m)
//   field RHS   b_i     = sum_j M^e_ij (y_j + c h^e_j)
// with h^e_j the local field of App. B at vertex j (anisotropy, Zeeman, far
// field, magnetoelastic with the element's total strain).
#include <algorithm>

#include <hip/hip_ext.h>

#include "device_common.h"

namespace gspm {

// ------------------------------------------------------------ the skeleton

// LDS layout of an element pass: acc[NC][nb] (FP64) | sx, sy, sz [nloc_max] | fields [NF][nloc_max]
// The owned-node accumulators are FP64 in both precisions: on gfx950 the
// FP64 LDS add (ds_add_f64) is far cheaper than the FP32 one, and FP32
// contributions lose nothing by being summed in FP64.
template <class T, int NC, int NF>
struct Staged {
    double *acc;
    T *sx, *sy, *sz, *f;
    int nloc_max;
    __device__ __forceinline__ T &fld(int k, int l) const { return f[k * nloc_max + l]; }
};

// Edge vectors from staged coordinates (scaled by sc), with the nearest
// periodic image when the block spans more than a quarter box.
template <class T>
__device__ __forceinline__ void stage_geometry(const T *sx, const T *sy, const T *sz, const ushort4 c, bool img,
                                               const MeshView &mv, double sc, Geo<T> &G) {
    const int v[4] = {c.x, c.y, c.z, c.w};
    T e[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        e[k][0] = sx[v[k + 1]] - sx[v[0]];
        e[k][1] = sy[v[k + 1]] - sy[v[0]];
        e[k][2] = sz[v[k + 1]] - sz[v[0]];
    }
    if (img) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            e[k][0] = near_image(e[k][0], static_cast<T>(mv.Lx * sc), static_cast<T>(mv.iLx / sc));
            e[k][1] = near_image(e[k][1], static_cast<T>(mv.Ly * sc), static_cast<T>(mv.iLy / sc));
            e[k][2] = near_image(e[k][2], static_cast<T>(mv.Lz * sc), static_cast<T>(mv.iLz / sc));
        }
    }
    tet_geometry_from_edges(e, G);
}

template <class T, int NC>
__device__ __forceinline__ void scatter_owned(double *acc, int nb, const ushort4 c, const T (&y)[4][NC]) {
    const int v[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (v[j] < nb) {
#pragma unroll
            for (int k = 0; k < NC; ++k) atomicAdd(&acc[k * nb + v[j]], static_cast<double>(y[j][k]));
        }
    }
}

template <class T, int NC, int NF, class Op>
__global__ void __launch_bounds__(kThreads) k_elem(const MeshView mv, const Op op_in) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Op op = op_in;
    if (!op.prepare()) return;                 // uniform: e.g. every CG component converged
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int nb = mv.nb, n0 = b * nb, cnt = min(nb, mv.n - n0);
    const int hbeg = mv.halo_ptr[b], nloc = nb + (mv.halo_ptr[b + 1] - hbeg);
    Staged<T, NC, NF> st;
    st.nloc_max = mv.nloc_max;
    st.acc = reinterpret_cast<double *>(smem_raw);
    st.sx = reinterpret_cast<T *>(st.acc + NC * nb);
    st.sy = st.sx + mv.nloc_max;
    st.sz = st.sy + mv.nloc_max;
    st.f = st.sz + mv.nloc_max;
    for (int i = threadIdx.x; i < NC * nb; i += kThreads) st.acc[i] = 0.0;
    const double xr = mv.x[n0], yr = mv.y[n0], zr = mv.z[n0], sc = op.coord_scale;
    for (int l = threadIdx.x; l < nloc; l += kThreads) {
        if (l >= cnt && l < nb) continue;      // owned slots past the last node
        const int g = l < nb ? n0 + l : mv.halo_ids[hbeg + l - nb];
        st.sx[l] = static_cast<T>(sc * near_image(mv.x[g] - xr, mv.Lx, mv.iLx));
        st.sy[l] = static_cast<T>(sc * near_image(mv.y[g] - yr, mv.Ly, mv.iLy));
        st.sz[l] = static_cast<T>(sc * near_image(mv.z[g] - zr, mv.Lz, mv.iLz));
        op.stage(st, l, g);
    }
    __syncthreads();
    const bool img = mv.img[b] != 0;
    const int e_beg = mv.blk_ptr[b];
    const int e_mag = e_beg + mv.blk_nmag[b];
    const int e_end = Op::kMagneticOnly ? e_mag : mv.blk_ptr[b + 1];
    if (mv.det.part != nullptr) {
        // deterministic mode: each owned node gathers its element copies in
        // copy order (each element evaluated once per owned vertex)
        for (int i = threadIdx.x; i < cnt; i += kThreads) {
            double acc[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) acc[k] = 0.0;
            const int t1 = mv.inc_ptr[b * nb + i + 1];
            for (int t = mv.inc_ptr[b * nb + i]; t < t1; ++t) {
                const int en = mv.inc_ent[t], e = e_beg + (en >> 2), j = en & 3;
                if (e >= e_end) break;              // magnetic copies come first
                const ushort4 c = mv.lconn[e];
                Geo<T> G;
                stage_geometry(st.sx, st.sy, st.sz, c, img, mv, sc, G);
                T y[4][NC];
                op.element(st, c, G, e < e_mag, y);
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (v == j) {
#pragma unroll
                        for (int k = 0; k < NC; ++k) acc[k] += static_cast<double>(y[v][k]);
                    }
            }
#pragma unroll
            for (int k = 0; k < NC; ++k) st.acc[k * nb + i] = acc[k];
        }
    } else {
        for (int e = e_beg + static_cast<int>(threadIdx.x); e < e_end; e += kThreads) {
            const ushort4 c = mv.lconn[e];
            Geo<T> G;
            stage_geometry(st.sx, st.sy, st.sz, c, img, mv, sc, G);
            T y[4][NC];
            op.element(st, c, G, e < e_mag, y);
            scatter_owned<T, NC>(st.acc, nb, c, y);
        }
    }
    __syncthreads();
    op.finish(mv, st, n0, cnt);
}

template <class T, int NC, int NF, class Op>
static void run_elem(const MeshView &mv, const Op &op, hipStream_t s) {
    const size_t lds = sizeof(double) * NC * static_cast<size_t>(mv.nb) + sizeof(T) * (3 + NF) * static_cast<size_t>(mv.nloc_max);
    hipLaunchKernelGGL((k_elem<T, NC, NF, Op>), dim3(mv.nblk), dim3(kThreads), lds, s, mv, op);
    launch_det_finish(mv.det, s);
}

__global__ void __launch_bounds__(kThreads) k_stage_coords(const MeshView mv, double *stc64, float *stc32) {
    const int b = blockIdx.x;
    const int nb = mv.nb, n0 = b * nb, cnt = min(nb, mv.n - n0);
    const int hbeg = mv.halo_ptr[b], nloc = nb + (mv.halo_ptr[b + 1] - hbeg);
    const size_t base = static_cast<size_t>(b) * nb + hbeg;
    const double xr = mv.x[n0], yr = mv.y[n0], zr = mv.z[n0], sc = 1.0 / mv.len_scale;
    for (int l = threadIdx.x; l < nloc; l += kThreads) {
        double cx = 0.0, cy = 0.0, cz = 0.0;
        if (!(l >= cnt && l < nb)) {
            const int g = l < nb ? n0 + l : mv.halo_ids[hbeg + l - nb];
            cx = near_image(mv.x[g] - xr, mv.Lx, mv.iLx);
            cy = near_image(mv.y[g] - yr, mv.Ly, mv.iLy);
            cz = near_image(mv.z[g] - zr, mv.Lz, mv.iLz);
        }
        stc64[base + l] = cx;
        stc64[mv.nstc + base + l] = cy;
        stc64[2 * mv.nstc + base + l] = cz;
        stc32[base + l] = static_cast<float>(sc * cx);
        stc32[mv.nstc + base + l] = static_cast<float>(sc * cy);
        stc32[2 * mv.nstc + base + l] = static_cast<float>(sc * cz);
    }
}

void launch_stage_coords(const MeshView &mv, double *stc64, float *stc32, hipStream_t s) {
    hipLaunchKernelGGL(k_stage_coords, dim3(mv.nblk), dim3(kThreads), 0, s, mv, stc64, stc32);
}

template <class T>
__device__ __forceinline__ const T *staged_coords(const MeshView &mv);
template <>
__device__ __forceinline__ const double *staged_coords<double>(const MeshView &mv) { return mv.stc64; }
template <>
__device__ __forceinline__ const float *staged_coords<float>(const MeshView &mv) { return mv.stc32; }

// The matrix-free operators walk tet strips instead of element lists.  Each
// thread takes one strip segment (at most one per thread; a block's segments
// have about the same number of window updates) and keeps a window of four
// vertices in registers (coordinates, fields, and the contributions
// accumulated for them).  Each update loads one staged vertex into one slot;
// after an update flagged as completing an element the window holds exactly
// that element's four vertices.  Lanes step through updates in lockstep, so
// a strip break in one lane (several loads before its next element) costs
// the other lanes nothing.  A
// vertex's accumulated contribution goes to LDS once, when it leaves the
// window, and only for owned vertices.  Along a strip each element loads one
// vertex instead of four, which cuts the LDS reads and atomics that bound the
// element-list form.  Staging and the per-node epilogue are the same.
// Staging of the matrix-free operators (strip and gather forms): LDS layout,
// accumulators cleared, the block's precomputed staged coordinates and the
// operand the op fetches (owned range, then halo list).
template <class T, int NC, int NF, class Op>
__device__ __forceinline__ Staged<T, NC, NF> stage_operator(const MeshView &mv, const Op &op, unsigned char *smem_raw,
                                                           int b, int n0, int cnt, int hbeg, int nloc) {
    const int nb = mv.nb;
    Staged<T, NC, NF> st;
    st.nloc_max = mv.nloc_max;
    st.acc = reinterpret_cast<double *>(smem_raw);
    st.sx = reinterpret_cast<T *>(st.acc + NC * nb);
    st.sy = st.sx + mv.nloc_max;
    st.sz = st.sy + mv.nloc_max;
    st.f = st.sz + mv.nloc_max;
    for (int i = threadIdx.x; i < NC * nb; i += kThreads) st.acc[i] = 0.0;
    // staging, four nodes per thread at a time: all their index loads, then
    // all their data loads, then the LDS stores (the halo gather is a chain of
    // two dependent loads; batching keeps many of them in flight).  The
    // coordinates come precomputed per block (contiguous, in the working
    // precision and units), only the operand is gathered.
    const T *stc = staged_coords<T>(mv);
    const size_t sbase = static_cast<size_t>(b) * nb + hbeg;
    constexpr int kU = 4;
    for (int l0 = threadIdx.x; l0 < nloc; l0 += kU * kThreads) {
        int ls[kU], gs[kU];
        bool ok[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            ls[u] = l0 + u * kThreads;
            ok[u] = ls[u] < nloc && !(ls[u] >= cnt && ls[u] < nb);   // owned slots past the last node are empty
            gs[u] = !ok[u] ? n0 : (ls[u] < nb ? n0 + ls[u] : mv.halo_ids[hbeg + ls[u] - nb]);
        }
        T cx[kU], cy[kU], cz[kU];
        T v[kU][NF];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const size_t o = sbase + static_cast<size_t>(ok[u] ? ls[u] : 0);
            cx[u] = stc[o];
            cy[u] = stc[mv.nstc + o];
            cz[u] = stc[2 * mv.nstc + o];
            op.fetch(gs[u], v[u], ok[u] && ls[u] < nb);
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            if (!ok[u]) continue;
            const int l = ls[u];
            st.sx[l] = cx[u];
            st.sy[l] = cy[u];
            st.sz[l] = cz[u];
#pragma unroll
            for (int q = 0; q < NF; ++q) st.fld(q, l) = v[u][q];
        }
    }
    return st;
}

template <class T, int NC, int NF, class Op>
__global__ void __launch_bounds__(kThreads) k_strip(const MeshView mv, const Op op_in) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Op op = op_in;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    if (!op.prepare(mv, b)) return;            // uniform: e.g. every CG component converged
    const int nb = mv.nb, n0 = b * nb, cnt = min(nb, mv.n - n0);
    const int hbeg = mv.halo_ptr[b], nloc = nb + (mv.halo_ptr[b + 1] - hbeg);
    Staged<T, NC, NF> st = stage_operator<T, NC, NF, Op>(mv, op, smem_raw, b, n0, cnt, hbeg, nloc);
    const double sc = op.coord_scale;
    __syncthreads();
    const bool img = mv.img[b] != 0;
    const T Lx = static_cast<T>(mv.Lx * sc), Ly = static_cast<T>(mv.Ly * sc), Lz = static_cast<T>(mv.Lz * sc);
    const T iLx = static_cast<T>(mv.iLx / sc), iLy = static_cast<T>(mv.iLy / sc), iLz = static_cast<T>(mv.iLz / sc);
    const int s_beg = mv.seg_ptr[b];
    const int s_end = Op::kMagneticOnly ? s_beg + mv.seg_nmag[b] : mv.seg_ptr[b + 1];
    for (int sg = s_beg + static_cast<int>(threadIdx.x); sg < s_end; sg += kThreads) {
        const int nel = mv.seg_nel[sg];
        // entries are consumed from the low half-word of q; the next eight are
        // already in flight in qn (the entry array carries 16 entries of tail
        // padding, so the lookahead stays in bounds)
        const uint4 *src = mv.seg_ent + mv.seg_off[sg];
        uint4 q = src[0], qn = src[1];
        src += 2;
        int avail = 8;
        int ids[4];
        T x[4][3], f[4][NF], acc[4][NC];
        // the element on the window: its contributions go to the four slots
        auto element = [&]() {
            T ed[3][3];
#pragma unroll
            for (int kk = 0; kk < 3; ++kk)
#pragma unroll
                for (int a = 0; a < 3; ++a) ed[kk][a] = x[kk + 1][a] - x[0][a];
            if (img) {
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    ed[kk][0] = near_image(ed[kk][0], Lx, iLx);
                    ed[kk][1] = near_image(ed[kk][1], Ly, iLy);
                    ed[kk][2] = near_image(ed[kk][2], Lz, iLz);
                }
            }
            RawGeo<T> R;
            tet_raw_geometry(ed, R);
            T y[4][NC];
            op.element_raw(f, R, y);
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[j][c] += y[j][c];
        };
        // A segment opens with its first element's four vertices loaded into
        // the empty slots 0..3 in order (the fourth entry flagged): all lanes
        // start together, so this part is peeled and loads without selects.
        {
            const uint32_t first[4] = {q.x & 0xFFFFu, q.x >> 16, q.y & 0xFFFFu, q.y >> 16};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int id = static_cast<int>(first[j] & kEntIdMask);
                ids[j] = id;
                x[j][0] = st.sx[id];
                x[j][1] = st.sy[id];
                x[j][2] = st.sz[id];
#pragma unroll
                for (int c = 0; c < NF; ++c) f[j][c] = st.fld(c, id);
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[j][c] = T(0);
            }
            q.x = q.z;
            q.y = q.w;
            q.z = 0u;
            q.w = 0u;
            avail = 4;
            element();
        }
        for (int k = 4; k < nel; ++k) {
            if (avail == 0) {
                q = qn;
                qn = *src++;
                avail = 8;
            }
            const uint32_t e = q.x & 0xFFFFu;
            q.x = (q.x >> 16) | (q.y << 16);
            q.y = (q.y >> 16) | (q.z << 16);
            q.z = (q.z >> 16) | (q.w << 16);
            q.w >>= 16;
            --avail;
            const int id = static_cast<int>(e & kEntIdMask), sl = static_cast<int>(e >> 14);
            // retire the vertex in slot sl
            int oid = ids[0];
            T oacc[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) oacc[c] = acc[0][c];
#pragma unroll
            for (int j = 1; j < 4; ++j) {
                const bool hit = sl == j;
                oid = hit ? ids[j] : oid;
#pragma unroll
                for (int c = 0; c < NC; ++c) oacc[c] = hit ? acc[j][c] : oacc[c];
            }
            if (oid < nb) {
#pragma unroll
                for (int c = 0; c < NC; ++c) atomicAdd(&st.acc[c * nb + oid], static_cast<double>(oacc[c]));
            }
            // the vertex of slot 3 moves into the freed slot, the new vertex
            // takes slot 3 (so only three slots need data-dependent selects)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const bool hit = sl == j;
                ids[j] = hit ? ids[3] : ids[j];
#pragma unroll
                for (int a = 0; a < 3; ++a) x[j][a] = hit ? x[3][a] : x[j][a];
#pragma unroll
                for (int c = 0; c < NF; ++c) f[j][c] = hit ? f[3][c] : f[j][c];
#pragma unroll
                for (int c = 0; c < NC; ++c) acc[j][c] = hit ? acc[3][c] : acc[j][c];
            }
            ids[3] = id;
            x[3][0] = st.sx[id];
            x[3][1] = st.sy[id];
            x[3][2] = st.sz[id];
#pragma unroll
            for (int c = 0; c < NF; ++c) f[3][c] = st.fld(c, id);
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[3][c] = T(0);
            if (e & kEntElem) element();
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (ids[j] < nb) {
#pragma unroll
                for (int c = 0; c < NC; ++c) atomicAdd(&st.acc[c * nb + ids[j]], static_cast<double>(acc[j][c]));
            }
    }
    __syncthreads();
    op.finish(mv, st, n0, cnt);
}

// Deterministic mode: the same operator with every owned node gathering the
// contributions of its element copies (the block's list, in copy order) in
// registers, so no LDS atomics decide the order of the sums.  Each element is
// evaluated once per owned vertex.
template <class T, int NC, int NF, class Op>
__global__ void __launch_bounds__(kThreads) k_strip_det(const MeshView mv, const Op op_in) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    Op op = op_in;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    if (!op.prepare(mv, b)) return;
    const int nb = mv.nb, n0 = b * nb, cnt = min(nb, mv.n - n0);
    const int hbeg = mv.halo_ptr[b], nloc = nb + (mv.halo_ptr[b + 1] - hbeg);
    Staged<T, NC, NF> st = stage_operator<T, NC, NF, Op>(mv, op, smem_raw, b, n0, cnt, hbeg, nloc);
    const double sc = op.coord_scale;
    __syncthreads();
    const bool img = mv.img[b] != 0;
    const T Lx = static_cast<T>(mv.Lx * sc), Ly = static_cast<T>(mv.Ly * sc), Lz = static_cast<T>(mv.Lz * sc);
    const T iLx = static_cast<T>(mv.iLx / sc), iLy = static_cast<T>(mv.iLy / sc), iLz = static_cast<T>(mv.iLz / sc);
    const int e_beg = mv.blk_ptr[b], e_mag = e_beg + mv.blk_nmag[b];
    for (int i = threadIdx.x; i < cnt; i += kThreads) {
        double acc[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = 0.0;
        const int t1 = mv.inc_ptr[b * nb + i + 1];
        for (int t = mv.inc_ptr[b * nb + i]; t < t1; ++t) {
            const int en = mv.inc_ent[t], e = e_beg + (en >> 2), j = en & 3;
            if (Op::kMagneticOnly && e >= e_mag) break;   // magnetic copies come first
            const ushort4 cv = mv.lconn[e];
            const int id[4] = {cv.x, cv.y, cv.z, cv.w};
            T x[4][3], f[4][NF];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                x[v][0] = st.sx[id[v]];
                x[v][1] = st.sy[id[v]];
                x[v][2] = st.sz[id[v]];
#pragma unroll
                for (int q = 0; q < NF; ++q) f[v][q] = st.fld(q, id[v]);
            }
            T ed[3][3];
#pragma unroll
            for (int kk = 0; kk < 3; ++kk)
#pragma unroll
                for (int a = 0; a < 3; ++a) ed[kk][a] = x[kk + 1][a] - x[0][a];
            if (img) {
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    ed[kk][0] = near_image(ed[kk][0], Lx, iLx);
                    ed[kk][1] = near_image(ed[kk][1], Ly, iLy);
                    ed[kk][2] = near_image(ed[kk][2], Lz, iLz);
                }
            }
            RawGeo<T> R;
            tet_raw_geometry(ed, R);
            T y[4][NC];
            op.element_raw(f, R, y);
#pragma unroll
            for (int v = 0; v < 4; ++v)
                if (v == j) {
#pragma unroll
                    for (int c = 0; c < NC; ++c) acc[c] += static_cast<double>(y[v][c]);
                }
        }
#pragma unroll
        for (int c = 0; c < NC; ++c) st.acc[c * nb + i] = acc[c];
    }
    __syncthreads();
    op.finish(mv, st, n0, cnt);
}

template <class T, int NC, int NF, class Op>
static void run_strip(const MeshView &mv, const Op &op, hipStream_t s, const hipEvent_t *ev = nullptr) {
    const size_t lds = sizeof(double) * NC * static_cast<size_t>(mv.nb) + sizeof(T) * (3 + NF) * static_cast<size_t>(mv.nloc_max);
    if (mv.det.part != nullptr) {
        if (ev)
            hipExtLaunchKernelGGL((k_strip_det<T, NC, NF, Op>), dim3(mv.nblk), dim3(kThreads), lds, s, ev[0], ev[1], 0,
                                  mv, op);
        else
            hipLaunchKernelGGL((k_strip_det<T, NC, NF, Op>), dim3(mv.nblk), dim3(kThreads), lds, s, mv, op);
        launch_det_finish(mv.det, s);
        return;
    }
    if (ev)
        hipExtLaunchKernelGGL((k_strip<T, NC, NF, Op>), dim3(mv.nblk), dim3(kThreads), lds, s, ev[0], ev[1], 0, mv, op);
    else
        hipLaunchKernelGGL((k_strip<T, NC, NF, Op>), dim3(mv.nblk), dim3(kThreads), lds, s, mv, op);
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
    // the same with the shear components given as engineering strains
    // (gamma = 2 eps_ij): s_ij = c44 gamma_ij
    __device__ __forceinline__ void stress_eng(const T (&e)[6], T (&s)[6]) const {
        const T tr = e[0] + e[1] + e[2], d = c11 - c12;
        s[0] = d * e[0] + c12 * tr;
        s[1] = d * e[1] + c12 * tr;
        s[2] = d * e[2] + c12 * tr;
        s[3] = c44 * e[3];
        s[4] = c44 * e[4];
        s[5] = c44 * e[5];
    }
};

// A general stiffness as a Voigt matrix (xx yy zz yz xz xy, engineering
// shear): the cubic crystal seen from a rotated sample frame (App. D).
template <class T>
struct Aniso {
    T c[36];
    __device__ __forceinline__ void stress_eng(const T (&e)[6], T (&s)[6]) const {
#pragma unroll
        for (int r = 0; r < 6; ++r)
            s[r] = c[6 * r] * e[0] + c[6 * r + 1] * e[1] + c[6 * r + 2] * e[2] + c[6 * r + 3] * e[3] +
                   c[6 * r + 4] * e[4] + c[6 * r + 5] * e[5];
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

// The staged 3-vectors (fields k0..k0+2) at the four vertices.
template <class T, int NC, int NF>
__device__ __forceinline__ void vertex3(const Staged<T, NC, NF> &st, int k0, const ushort4 c, T (&v)[4][3]) {
    const int id[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int a = 0; a < 3; ++a) v[j][a] = st.fld(k0 + a, id[j]);
}

// ------------------------------------------------------------- elasticity

// K^mech of one element (Eq. LHS) applied to its vertex values (strip form), on
// the unscaled geometry: H' = sum_k (v_k - v_0) (x) c_k = det grad v, so
// C sym(H') = det sigma, and V sigma grad(lambda_j) = w (C sym H') c_j; vertex
// 0 takes minus the sum of the others (the gradients sum to zero).
template <class T, class M>
__device__ __forceinline__ void elastic_element_raw(const M &C, const T (&v)[4][3], const RawGeo<T> &R,
                                                    T (&y)[4][3]) {
    T H[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T d1 = v[1][a] - v[0][a], d2 = v[2][a] - v[0][a], d3 = v[3][a] - v[0][a];
#pragma unroll
        for (int b = 0; b < 3; ++b) H[a][b] = d1 * R.c[1][b] + d2 * R.c[2][b] + d3 * R.c[3][b];
    }
    const T e[6] = {H[0][0], H[1][1], H[2][2], H[1][2] + H[2][1], H[0][2] + H[2][0], H[0][1] + H[1][0]};
    T s[6];
    C.stress_eng(e, s);
#pragma unroll
    for (int t = 0; t < 6; ++t) s[t] *= R.w;
#pragma unroll
    for (int j = 1; j < 4; ++j) {
        const T *c = R.c[j];
        y[j][0] = s[0] * c[0] + s[5] * c[1] + s[4] * c[2];
        y[j][1] = s[5] * c[0] + s[1] * c[1] + s[3] * c[2];
        y[j][2] = s[4] * c[0] + s[3] * c[1] + s[2] * c[2];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) y[0][a] = -(y[1][a] + y[2][a] + y[3][a]);
}

// Matrix-free K^mech (Eq. LHS): y_i = V sigma(u) g_i over all elements; rows of
// the pinned node are zero.  See launch_elastic_matvec for the modes.
template <class T, class M = Cubic<T>>
struct ElasticMatvecOp {
    static constexpr bool kMagneticOnly = false;
    const T *in;                  // APPLY/RESID: the vector; ITER: p_old
    T *out;                       // APPLY: A in; ITER: q
    const T *b;                   // RESID
    const T *r;                   // RESID: r (out); ITER: r (in)
    T *pout;                      // ITER: p_new
    CGScalars cg;
    int k, mode, n;
    double tol2;
    M C;
    int live[1];
    double beta[1];
    double coord_scale;           // staged coordinates in units of 1/coord_scale metres

    __device__ bool prepare(const MeshView &, int) {
        if (mode != MV_ITER) return mode == MV_APPLY || cg.done[0] == 0;
        return cg_direction_scalars<1>(cg, k, tol2, live, beta);
    }

    // the staged operand at node g: p_new = r + beta p_old (ITER), else in
    __device__ __forceinline__ void fetch(int g, T (&v)[3], bool) const {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const size_t o = static_cast<size_t>(a) * n + g;
            if (mode == MV_ITER) v[a] = (k == 0) ? r[o] : r[o] + static_cast<T>(beta[0]) * in[o];
            else v[a] = in[o];
        }
    }

    __device__ __forceinline__ void element_raw(const T (&v)[4][3], const RawGeo<T> &R, T (&y)[4][3]) const {
        elastic_element_raw(C, v, R, y);
    }

    template <int NF>
    __device__ void finish(const MeshView &mv, const Staged<T, 3, NF> &st, int n0, int cnt) const {
        double part = 0.0;
        for (int i = threadIdx.x; i < cnt; i += kThreads) {
            const int node = n0 + i;
            const bool pinned = node == mv.p0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const size_t o = static_cast<size_t>(a) * n + node;
                const T q = pinned ? T(0) : st.acc[a * mv.nb + i];
                if (mode == MV_RESID) {
                    const T rv = pinned ? T(0) : b[o] - q;
                    const_cast<T *>(r)[o] = rv;
                    part += static_cast<double>(rv) * rv;
                } else if (mode == MV_ITER) {
                    const T pv = st.fld(a, i);
                    pout[o] = pv;
                    out[o] = q;
                    part += static_cast<double>(pv) * q;
                } else {
                    out[o] = q;
                }
            }
        }
        if (mode == MV_ITER) block_atomic_add1(part, cg.pq_at(0, k), cg.det);
        else if (mode == MV_RESID) block_atomic_add1(part, cg.rr_at(0, 0), cg.det);
    }
};

// The prologue of single-reduction CG launch k (shared by the elastic and
// magnetostatic operators, NV values per node): completes iteration k-1 from
// the sums of launch k-1 (alpha, beta), records a stop (workgroup 0), and in
// the last launch only adds the pending alpha p_{k-1} to x on the owned nodes.
// Returns whether the launch has an iteration to run.
template <int NV, class T>
__device__ __forceinline__ bool sr_cg_prepare(const CGScalars &cg, int k, int last, double tol2, const MeshView &mv,
                                              int b, int n, T *x, const T *pin, double &alpha, double &beta) {
    alpha = beta = 0.0;
    // a test recorded by an earlier launch (or by workgroup 0 of this one,
    // which then leaves nothing to do either)
    if (cg.done[0] != 0) return false;
    if (k == 0) return !last;                // the start test ran in an earlier launch
    const double *const src[5] = {cg.rr_at(0, k - 1), cg.pq_at(0, k - 1), cg.rq_at(k - 1), cg.qq_at(k - 1),
                                  cg.bb_at(0)};
    double t[5];
    shard_totals<5>(src, t);
    const double rrp = t[0];
    const int stop = !isfinite(rrp) ? 2 : (rrp <= tol2 * t[4] ? 1 : 0);
    if (stop) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            cg.done[0] = stop;
            cg.iters[0] = k - 1;
        }
        return false;
    }
    alpha = rrp / t[1];
    const double est = rrp - 2.0 * alpha * t[2] + alpha * alpha * t[3];
    beta = (est > 0.0 ? est : 0.0) / rrp;
    if (last) {
        const int n0 = b * mv.nb, cnt = min(mv.nb, mv.n - n0);
        const T a = static_cast<T>(alpha);
        for (int i = threadIdx.x; i < cnt; i += kThreads)
#pragma unroll
            for (int c = 0; c < NV; ++c) {
                const size_t o = static_cast<size_t>(c) * n + n0 + i;
                x[o] += a * pin[o];
            }
        return false;
    }
    return true;
}

// One launch of single-reduction CG on the elastic system (one scalar set,
// Sec. 2.5; the iterates of the two-launch form up to rounding).  Launch k
// completes iteration k-1 from the sums of its epilogue, r.r, p.q, r.q and
// q.q with q = A p:
//   alpha = rr_{k-1} / (p.q) (rr_{k-1} the true |r_{k-1}|^2),
//   beta  = rr~_k / rr_{k-1},  rr~_k = rr_{k-1} - 2 alpha (r.q) + alpha^2 (q.q)
// (the expansion of |r_{k-1} - alpha q|^2, which cancels badly near tight
// tolerances, so it only sets the direction; the step length and the
// stopping test use the true norms, the test one launch later), forms
// r_k = r_{k-1} - alpha q_{k-1} and p_k = r_k + beta p_{k-1} while staging,
// adds alpha p_{k-1} to x on its owned nodes, and computes q_k = A p_k with
// the four sums of iteration k.  r, p and q alternate between two buffers
// (other workgroups still read iteration k-1's values as halo).  The launch
// that finds rr_{k-1} converged records it (x_{k-1} is the answer) and does
// nothing else; the final launch after the last permitted iteration only adds
// the pending alpha p_{k-1} to x when rr_{k-1} has not converged.
template <class T, class M = Cubic<T>>
struct ElasticCgOp {
    static constexpr bool kMagneticOnly = false;
    const T *rin, *pin, *qin;     // r_{k-1}, p_{k-1}, q_{k-1} (rin = r_0 at k = 0)
    T *rout, *pout, *qout;        // r_k, p_k, q_k
    T *x;
    CGScalars cg;
    int k, n, last;               // last: the launch after the last permitted iteration
    double tol2;
    M C;
    double alpha, beta;
    double coord_scale;

    __device__ bool prepare(const MeshView &mv, int b) {
        return sr_cg_prepare<3>(cg, k, last, tol2, mv, b, n, x, pin, alpha, beta);
    }

    // the staged operand p_k at node g; owned nodes also store r_k and take
    // the pending step of x
    __device__ __forceinline__ void fetch(int g, T (&v)[3], bool owned) const {
        const T a = static_cast<T>(alpha), bt = static_cast<T>(beta);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t o = static_cast<size_t>(c) * n + g;
            if (k == 0) {
                v[c] = rin[o];
                continue;
            }
            const T pold = pin[o];
            const T rk = rin[o] - a * qin[o];
            v[c] = rk + bt * pold;
            if (owned) {
                rout[o] = rk;
                x[o] += a * pold;
            }
        }
    }

    __device__ __forceinline__ void element_raw(const T (&v)[4][3], const RawGeo<T> &R, T (&y)[4][3]) const {
        elastic_element_raw(C, v, R, y);
    }

    template <int NF>
    __device__ void finish(const MeshView &mv, const Staged<T, 3, NF> &st, int n0, int cnt) const {
        double part[4] = {0.0, 0.0, 0.0, 0.0};   // p.q, r.q, q.q, r.r
        const T *rk = k == 0 ? rin : rout;
        for (int i = threadIdx.x; i < cnt; i += kThreads) {
            const int node = n0 + i;
            const bool pinned = node == mv.p0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const size_t o = static_cast<size_t>(a) * n + node;
                const T q = pinned ? T(0) : st.acc[a * mv.nb + i];
                const T pv = st.fld(a, i);
                pout[o] = pv;
                qout[o] = q;
                const double rv = static_cast<double>(rk[o]);
                part[0] += static_cast<double>(pv) * q;
                part[1] += rv * q;
                part[2] += static_cast<double>(q) * q;
                part[3] += rv * rv;
            }
        }
        // r_0.r_0 is already in slot 0 (the residual launch wrote it)
        double *const dst[4] = {cg.pq_at(0, k), cg.rq_at(k), cg.qq_at(k), k == 0 ? nullptr : cg.rr_at(0, k)};
        block_atomic_add_to<4>(part, dst, cg.det);
    }
};

// The matvec of preconditioned CG iteration k on the periodic elastic system
// (no pinned node): the direction p_k = z_k + beta p_{k-1}, beta = rz_k /
// rz_{k-1} (p_0 = z_0), formed in the staging; q = K^mech p_k and p_k . q in
// the epilogue.  A converged set (decided by the preconditioner's restriction
// pass, which tests |r|) makes the launch return at once.
template <class T, class M = Cubic<T>>
struct ElasticPcgOp {
    static constexpr bool kMagneticOnly = false;
    const T *z, *pin;             // z_k, p_{k-1}
    T *pout, *q;                  // p_k, q_k
    CGScalars cg;
    int k, n;
    M C;
    double beta;
    double coord_scale;

    __device__ bool prepare(const MeshView &, int) {
        if (cg.done[0] != 0) return false;
        beta = 0.0;
        if (k > 0) {
            const double *const src[2] = {pcg_rz_at(cg, k), pcg_rz_at(cg, k - 1)};
            double t[2];
            shard_totals<2>(src, t);
            beta = t[0] / t[1];
        }
        return true;
    }

    __device__ __forceinline__ void fetch(int g, T (&v)[3], bool) const {
        const T bt = static_cast<T>(beta);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const size_t o = static_cast<size_t>(c) * n + g;
            v[c] = k == 0 ? z[o] : z[o] + bt * pin[o];
        }
    }

    __device__ __forceinline__ void element_raw(const T (&v)[4][3], const RawGeo<T> &R, T (&y)[4][3]) const {
        elastic_element_raw(C, v, R, y);
    }

    template <int NF>
    __device__ void finish(const MeshView &mv, const Staged<T, 3, NF> &st, int n0, int cnt) const {
        double part = 0.0;
        for (int i = threadIdx.x; i < cnt; i += kThreads) {
            const int node = n0 + i;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const size_t o = static_cast<size_t>(a) * n + node;
                const T qv = static_cast<T>(st.acc[a * mv.nb + i]);
                const T pv = st.fld(a, i);
                pout[o] = pv;
                q[o] = qv;
                part += static_cast<double>(pv) * qv;
            }
        }
        block_atomic_add1(part, cg.pq_at(0, k), cg.det);
    }
};

// One launch of single-reduction CG on K^ms (Eq. weak_demag: the Laplacian
// over all elements, one scalar component, the pinned node's rows zero), with
// the control of ElasticCgOp: the direction and the residual formed in the
// staging, q = K^ms p and the four sums p.q, r.q, q.q, r.r in the epilogue.
template <class T>
struct MsCgOp {
    static constexpr bool kMagneticOnly = false;
    const T *rin, *pin, *qin;     // r_{k-1}, p_{k-1}, q_{k-1} (rin = r_0 at k = 0)
    T *rout, *pout, *qout;        // r_k, p_k, q_k
    T *x;
    CGScalars cg;
    int k, n, last;
    double tol2;
    T eps;                        // 1 (FP64) or 1 / len_scale^2 (FP32 on scaled coordinates)
    double alpha, beta;
    double coord_scale;

    __device__ bool prepare(const MeshView &mv, int b) {
        return sr_cg_prepare<1>(cg, k, last, tol2, mv, b, n, x, pin, alpha, beta);
    }

    __device__ __forceinline__ void fetch(int g, T (&v)[1], bool owned) const {
        if (k == 0) {
            v[0] = rin[g];
            return;
        }
        const T a = static_cast<T>(alpha), bt = static_cast<T>(beta);
        const T pold = pin[g];
        const T rk = rin[g] - a * qin[g];
        v[0] = rk + bt * pold;
        if (owned) {
            rout[g] = rk;
            x[g] += a * pold;
        }
    }

    // V grad(lambda_i) . grad(u_h) = w c_i . (sum_k (u_k - u_0) c_k)
    __device__ __forceinline__ void element_raw(const T (&f)[4][1], const RawGeo<T> &R, T (&y)[4][1]) const {
        const T ev = eps * R.w;
        const T d1 = f[1][0] - f[0][0], d2 = f[2][0] - f[0][0], d3 = f[3][0] - f[0][0];
        T gp[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) gp[a] = d1 * R.c[1][a] + d2 * R.c[2][a] + d3 * R.c[3][a];
        T t[4];
#pragma unroll
        for (int j = 1; j < 4; ++j) t[j] = R.c[j][0] * gp[0] + R.c[j][1] * gp[1] + R.c[j][2] * gp[2];
        t[0] = -(t[1] + t[2] + t[3]);
#pragma unroll
        for (int j = 0; j < 4; ++j) y[j][0] = ev * t[j];
    }

    template <int NF>
    __device__ void finish(const MeshView &mv, const Staged<T, 1, NF> &st, int n0, int cnt) const {
        double part[4] = {0.0, 0.0, 0.0, 0.0};   // p.q, r.q, q.q, r.r
        const T *rk = k == 0 ? rin : rout;
        for (int i = threadIdx.x; i < cnt; i += kThreads) {
            const int node = n0 + i;
            const T q = node == mv.p0 ? T(0) : static_cast<T>(st.acc[i]);
            const T pv = st.fld(0, i);
            pout[node] = pv;
            qout[node] = q;
            const double rv = static_cast<double>(rk[node]);
            part[0] += static_cast<double>(pv) * q;
            part[1] += rv * q;
            part[2] += static_cast<double>(q) * q;
            part[3] += rv * rv;
        }
        double *const dst[4] = {cg.pq_at(0, k), cg.rq_at(k), cg.qq_at(k), k == 0 ? nullptr : cg.rr_at(0, k)};
        block_atomic_add_to<4>(part, dst, cg.det);
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
    int rot;                      // crystal orientation R (App. D)
    double R[9];
    double coord_scale = 1.0;

    __device__ bool prepare() { return true; }

    template <int NF>
    __device__ __forceinline__ void stage(const Staged<T, 3, NF> &st, int l, int g) const {
#pragma unroll
        for (int a = 0; a < 3; ++a) st.fld(a, l) = m[static_cast<size_t>(a) * n + g];
    }

    template <int NF>
    __device__ __forceinline__ void element(const Staged<T, 3, NF> &st, const ushort4 c, const Geo<T> &G, bool,
                                            T (&y)[4][3]) const {
        T v[4][3], e0[6] = {0, 0, 0, 0, 0, 0};
        vertex3(st, 0, c, v);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            T ej[6], mj[3] = {v[j][0], v[j][1], v[j][2]};
            if (rot) {
                const T ms[3] = {mj[0], mj[1], mj[2]};
                to_crystal3(R, ms, mj);
            }
            spontaneous_strain(l100, l111, mj, ej);
#pragma unroll
            for (int t = 0; t < 6; ++t) e0[t] += ej[t];
        }
#pragma unroll
        for (int t = 0; t < 6; ++t) e0[t] *= T(0.25);
        T s[6];
        C.stress(e0, s);              // crystal frame when rotated
        if (rot) {
            const T sc[6] = {s[0], s[1], s[2], s[3], s[4], s[5]};
            sym_rotate(R, true, sc, s);
        }
#pragma unroll
        for (int t = 0; t < 6; ++t) s[t] *= G.vol;
        sym_times_grads(s, G, y);
    }

    template <int NF>
    __device__ void finish(const MeshView &mv, const Staged<T, 3, NF> &st, int n0, int cnt) const {
        double part = 0.0;
        for (int i = threadIdx.x; i < cnt; i += kThreads) {
            const int node = n0 + i;
            const bool pinned = node == mv.p0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const size_t o = static_cast<size_t>(a) * n + node;
                const T v = pinned ? T(0) : st.acc[a * mv.nb + i];
                b[o] = v;
                if (pinned) x[o] = T(0);
                part += static_cast<double>(v) * v;
            }
        }
        block_atomic_add1(part, bb, mv.det);
    }
};

// ----------------------------------------------------- magnetostatic operator

// K^ms of Eq. (weak_demag): the Laplacian over all elements with the pinned
// node's rows zero, on NC scalar components stored [c][n], one CG scalar set
// per component; a converged component is skipped.  (The GS operator eps K +
// M runs in row form, row_kernels.hip.)
template <class T, int NC>
struct MsMatvecOp {
    static constexpr bool kMagneticOnly = false;
    const T *in;
    T *out;
    const T *b;
    const T *r;
    T *pout;
    CGScalars cg;
    int k, mode, n;
    double tol2;
    T eps;                        // 1 (FP64) or 1 / len_scale^2 (FP32 on scaled coordinates)
    int live[NC];
    double beta[NC];
    double coord_scale;

    __device__ bool prepare(const MeshView &, int) {
        if (mode == MV_ITER) return cg_direction_scalars<NC>(cg, k, tol2, live, beta);
        bool any = false;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            live[c] = (mode == MV_APPLY) ? 1 : (cg.done[c] == 0);
            beta[c] = 0.0;
            any |= live[c] != 0;
        }
        return any;
    }

    // the staged operand at node g (zero for components that are not live)
    __device__ __forceinline__ void fetch(int g, T (&v)[NC], bool) const {
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const size_t o = static_cast<size_t>(q) * n + g;
            if (!live[q]) v[q] = T(0);
            else if (mode == MV_ITER) v[q] = (k == 0) ? r[o] : r[o] + static_cast<T>(beta[q]) * in[o];
            else v[q] = in[o];
        }
    }

    // the element with its vertex values given (strip form), on the unscaled
    // geometry: eps V g_i . g_j = (eps w) c_i . c_j
    __device__ __forceinline__ void element_raw(const T (&f)[4][NC], const RawGeo<T> &R, T (&y)[4][NC]) const {
        const T ev = eps * R.w;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            if (!live[q]) {
#pragma unroll
                for (int j = 0; j < 4; ++j) y[j][q] = T(0);
                continue;
            }
            T v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = f[j][q];
            const T d1 = v[1] - v[0], d2 = v[2] - v[0], d3 = v[3] - v[0];
            T gp[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) gp[a] = d1 * R.c[1][a] + d2 * R.c[2][a] + d3 * R.c[3][a];
            T t[4];
#pragma unroll
            for (int j = 1; j < 4; ++j) t[j] = R.c[j][0] * gp[0] + R.c[j][1] * gp[1] + R.c[j][2] * gp[2];
            t[0] = -(t[1] + t[2] + t[3]);
#pragma unroll
            for (int j = 0; j < 4; ++j) y[j][q] = ev * t[j];
        }
    }

    template <int NF>
    __device__ void finish(const MeshView &mv, const Staged<T, NC, NF> &st, int n0, int cnt) const {
        double part[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) part[q] = 0.0;
        for (int i = threadIdx.x; i < cnt; i += kThreads) {
            const int node = n0 + i;
#pragma unroll
            for (int q = 0; q < NC; ++q) {
                if (!live[q]) continue;
                const size_t o = static_cast<size_t>(q) * n + node;
                const T av = node == mv.p0 ? T(0) : static_cast<T>(st.acc[q * mv.nb + i]);
                if (mode == MV_RESID) {
                    const T rv = b[o] - av;
                    const_cast<T *>(r)[o] = rv;
                    part[q] += static_cast<double>(rv) * rv;
                } else if (mode == MV_ITER) {
                    const T pv = st.fld(q, i);
                    pout[o] = pv;
                    out[o] = av;
                    part[q] += static_cast<double>(pv) * av;
                } else {
                    out[o] = av;
                }
            }
        }
        if (mode == MV_ITER) block_atomic_add<NC>(part, cg.pq_at(0, k), cg.comp_stride(), cg.det);
        else if (mode == MV_RESID) block_atomic_add<NC>(part, cg.rr_at(0, 0), cg.comp_stride(), cg.det);
    }
};

// ------------------------------------------------- magnetostatic RHS

// Right-hand side of Eq. (weak_demag), b = Ms F^ms m (Eqs. RHS_F, RHS_b), in
// the element form b_i = Ms V_e grad(lambda_i) . <m>_e summed over all
// elements (<m>_e the vertex mean).  This equals -Ms int phi_i div(m_h) on a
// periodic mesh: int d_a(phi_i phi_j) over the cell vanishes.  Zero at the
// pinned node, whose potential x is also zeroed; bb += b.b.
template <class T>
struct MsRhsOp {
    static constexpr bool kMagneticOnly = false;
    const T *m;
    T *b, *x;
    double *bb;
    int n;
    T Ms;
    double coord_scale = 1.0;

    __device__ bool prepare() { return true; }

    template <int NF>
    __device__ __forceinline__ void stage(const Staged<T, 1, NF> &st, int l, int g) const {
#pragma unroll
        for (int a = 0; a < 3; ++a) st.fld(a, l) = m[static_cast<size_t>(a) * n + g];
    }

    template <int NF>
    __device__ __forceinline__ void element(const Staged<T, 1, NF> &st, const ushort4 cn, const Geo<T> &G, bool,
                                            T (&y)[4][1]) const {
        T mv[4][3];
        vertex3(st, 0, cn, mv);
        const T q = Ms * G.vol * T(0.25);
        T mm[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) mm[a] = q * (mv[0][a] + mv[1][a] + mv[2][a] + mv[3][a]);
#pragma unroll
        for (int j = 0; j < 4; ++j) y[j][0] = G.g[j][0] * mm[0] + G.g[j][1] * mm[1] + G.g[j][2] * mm[2];
    }

    template <int NF>
    __device__ void finish(const MeshView &mv, const Staged<T, 1, NF> &st, int n0, int cnt) const {
        double part = 0.0;
        for (int i = threadIdx.x; i < cnt; i += kThreads) {
            const int node = n0 + i;
            const bool pinned = node == mv.p0;
            const T v = pinned ? T(0) : static_cast<T>(st.acc[i]);
            b[node] = v;
            if (pinned) x[node] = T(0);
            part += static_cast<double>(v) * v;
        }
        block_atomic_add1(part, bb, mv.det);
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
template <class T, bool kUd = false>
struct FieldRhsOp {
    static constexpr bool kMagneticOnly = true;
    const T *m, *u;
    const Derived *d;
    const T *ud;                  // kUd: the local magnetostatic potential
    T inv_ms;
    T *b, *x0, *ch2;
    double *bb;
    int n, bbstride;
    T c;
    Cubic<T> C;
    T l100, l111, kan, kme;
    T E0bar[6], hc[3];
    int rot;                      // crystal orientation R (App. D)
    double R[9];
    double coord_scale = 1.0;

    __device__ bool prepare() {
#pragma unroll
        for (int t = 0; t < 6; ++t) E0bar[t] = static_cast<T>(d->ebar[t]);
#pragma unroll
        for (int a = 0; a < 3; ++a) hc[a] = static_cast<T>(d->hc[a]);
        return true;
    }

    template <int NF>
    __device__ __forceinline__ void stage(const Staged<T, 6, NF> &st, int l, int g) const {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            st.fld(a, l) = m[static_cast<size_t>(a) * n + g];
            st.fld(3 + a, l) = u[static_cast<size_t>(a) * n + g];
        }
        if constexpr (kUd) st.fld(6, l) = ud[g];
    }

    template <int NF>
    __device__ __forceinline__ void element(const Staged<T, 6, NF> &st, const ushort4 cn, const Geo<T> &G, bool,
                                            T (&y)[4][6]) const {
        T mv[4][3], uv[4][3], E[6];
        vertex3(st, 0, cn, mv);
        vertex3(st, 3, cn, uv);
        sym_grad(uv, G, E);
#pragma unroll
        for (int t = 0; t < 6; ++t) E[t] += E0bar[t];
        T hce[3] = {hc[0], hc[1], hc[2]};
        if constexpr (kUd) {
            // the element's local demagnetising field -grad(U~) / Ms (Sec. 2.1)
            const int id[4] = {cn.x, cn.y, cn.z, cn.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const T uj = st.fld(6, id[j]) * inv_ms;
#pragma unroll
                for (int a = 0; a < 3; ++a) hce[a] -= uj * G.g[j][a];
            }
        }
        T f[4][3], sf[3] = {0, 0, 0}, sm[3] = {0, 0, 0};
        T Ec[6];
        if (rot) sym_rotate(R, false, E, Ec);   // the element strain in the crystal frame
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const T mj[3] = {mv[j][0], mv[j][1], mv[j][2]};
            T h[3];
            if (rot) {
                // anisotropy and magnetoelastic field in the crystal frame, rotated back (App. D, Step 4)
                T mc[3], hcr[3];
                const T zero[3] = {T(0), T(0), T(0)};
                to_crystal3(R, mj, mc);
                local_field(C, l100, l111, kan, kme, zero, Ec, mc, hcr);
                to_sample3(R, hcr, h);
#pragma unroll
                for (int a = 0; a < 3; ++a) h[a] += hce[a];
            } else {
                local_field(C, l100, l111, kan, kme, hce, E, mj, h);
            }
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

    template <int NF>
    __device__ void finish(const MeshView &mv, const Staged<T, 6, NF> &st, int n0, int cnt) const {
        double part[3] = {0.0, 0.0, 0.0};
        for (int i = threadIdx.x; i < cnt; i += kThreads) {
            const int node = n0 + i;
            const double w = mv.w[node];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const size_t o = static_cast<size_t>(a) * n + node;
                const T my = st.acc[a * mv.nb + i], chv = st.acc[(3 + a) * mv.nb + i];
                const T bv = my + chv;
                b[o] = bv;
                x0[o] = w > 0.0 ? st.fld(a, i) + chv / static_cast<T>(w) : T(0);
                if (ch2 != nullptr && a < 2) ch2[o] = chv;
                part[a] += static_cast<double>(bv) * bv;
            }
        }
        block_atomic_add<3>(part, bb, bbstride, mv.det);
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
    double coord_scale = 1.0;

    __device__ bool prepare() { return true; }

    template <int NF>
    __device__ __forceinline__ void stage(const Staged<T, 2, NF> &st, int l, int g) const {
        st.fld(0, l) = y[g];
        st.fld(1, l) = y[static_cast<size_t>(n) + g];
    }

    template <int NF>
    __device__ __forceinline__ void element(const Staged<T, 2, NF> &st, const ushort4 cn, const Geo<T> &G, bool,
                                            T (&out)[4][2]) const {
        const int id[4] = {cn.x, cn.y, cn.z, cn.w};
        const T w20 = G.vol * T(0.05);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            T v[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = st.fld(q, id[j]);
            const T s = v[0] + v[1] + v[2] + v[3];
#pragma unroll
            for (int j = 0; j < 4; ++j) out[j][q] = w20 * (v[j] + s);
        }
    }

    template <int NF>
    __device__ void finish(const MeshView &mv, const Staged<T, 2, NF> &st, int n0, int cnt) const {
        double part[2] = {0.0, 0.0};
        for (int i = threadIdx.x; i < cnt; i += kThreads) {
            const int node = n0 + i;
            const double w = mv.w[node];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const size_t o = static_cast<size_t>(q) * n + node;
                const T chv = ch2[o];
                const T bv = st.acc[q * mv.nb + i] + chv;
                b[o] = bv;
                x0[o] = w > 0.0 ? st.fld(q, i) + chv / static_cast<T>(w) : T(0);
                part[q] += static_cast<double>(bv) * bv;
            }
        }
        block_atomic_add<2>(part, bb, bbstride, mv.det);
    }
};

// ---------------------------------------------------------------- energies

// Element sums of the exchange energy A V |grad m|^2 (magnetic elements) and
// of the magnetoelastic energy V/4 sum_j 1/2 (E - chi E0(m_j)) : C (E - chi E0(m_j))
// (all elements), E = Ebar + sym grad u.  Each element is counted only by the
// block owning its smallest vertex id: a copy is skipped when one of its
// vertices is a halo node below the block's range (halo slots [nb, nb + halo_lo)).
template <class T>
__global__ void __launch_bounds__(kThreads) k_energy_elem(const MeshView mv, Material mat, const T *m, const T *u,
                                                          const T *ud, const Derived *d, double *out) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const int nb = mv.nb, n0 = b * nb, cnt = min(nb, mv.n - n0);
    const int hbeg = mv.halo_ptr[b], nloc = nb + (mv.halo_ptr[b + 1] - hbeg), below = mv.halo_lo[b];
    Staged<T, 1, 7> st;
    st.nloc_max = mv.nloc_max;
    st.acc = reinterpret_cast<double *>(smem_raw);
    st.sx = reinterpret_cast<T *>(st.acc + nb);
    st.sy = st.sx + mv.nloc_max;
    st.sz = st.sy + mv.nloc_max;
    st.f = st.sz + mv.nloc_max;
    const double xr = mv.x[n0], yr = mv.y[n0], zr = mv.z[n0];
    for (int l = threadIdx.x; l < nloc; l += kThreads) {
        if (l >= cnt && l < nb) continue;
        const int g = l < nb ? n0 + l : mv.halo_ids[hbeg + l - nb];
        st.sx[l] = static_cast<T>(near_image(mv.x[g] - xr, mv.Lx, mv.iLx));
        st.sy[l] = static_cast<T>(near_image(mv.y[g] - yr, mv.Ly, mv.iLy));
        st.sz[l] = static_cast<T>(near_image(mv.z[g] - zr, mv.Lz, mv.iLz));
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            st.fld(a, l) = m[static_cast<size_t>(a) * mv.n + g];
            st.fld(3 + a, l) = u[static_cast<size_t>(a) * mv.n + g];
        }
        st.fld(6, l) = ud ? ud[g] : T(0);
    }
    __syncthreads();
    const Cubic<T> C{static_cast<T>(mat.c11), static_cast<T>(mat.c12), static_cast<T>(mat.c44)};
    T Eb[6];
#pragma unroll
    for (int t = 0; t < 6; ++t) Eb[t] = static_cast<T>(d->ebar[t]);
    const bool img = mv.img[b] != 0;
    const bool rot = mat.rot != 0;
    double ex = 0.0, me = 0.0, dl = 0.0;
    const int e_beg = mv.blk_ptr[b], e_mag = e_beg + mv.blk_nmag[b], e_end = mv.blk_ptr[b + 1];
    for (int e = e_beg + static_cast<int>(threadIdx.x); e < e_end; e += kThreads) {
        const ushort4 c = mv.lconn[e];
        const int v[4] = {c.x, c.y, c.z, c.w};
        bool skip = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) skip |= v[j] >= nb && v[j] < nb + below;
        if (skip) continue;
        const bool mag = e < e_mag;
        Geo<T> G;
        stage_geometry(st.sx, st.sy, st.sz, c, img, mv, 1.0, G);
        T mv4[4][3], uv[4][3], E[6];
        vertex3(st, 0, c, mv4);
        vertex3(st, 3, c, uv);
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
        if (rot) {
            // the energy density is frame independent: evaluate it in the crystal frame
            const T Es[6] = {E[0], E[1], E[2], E[3], E[4], E[5]};
            sym_rotate(mat.R, false, Es, E);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const T ms[3] = {mv4[j][0], mv4[j][1], mv4[j][2]};
                T mc[3];
                to_crystal3(mat.R, ms, mc);
#pragma unroll
                for (int a = 0; a < 3; ++a) mv4[j][a] = mc[a];
            }
        }
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
        if (ud) {
            // |grad U~|^2 over the element (all elements: the field fills the inclusions too)
            double gu[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double uj = st.fld(6, v[j]);
#pragma unroll
                for (int a = 0; a < 3; ++a) gu[a] += uj * G.g[j][a];
            }
            dl += static_cast<double>(G.vol) * (gu[0] * gu[0] + gu[1] * gu[1] + gu[2] * gu[2]);
        }
    }
    const double v2[2] = {ex, me};
    block_atomic_add<2>(v2, out, kShards, mv.det);
    if (ud) block_atomic_add1(dl, out + 4 * kShards, mv.det, 2);
}

// --------------------------------------------------------------- launchers

// The launches of this file request sizeof(double) NC nb + sizeof(T) (3 + NF)
// nloc_max bytes (energy pass: 8 (nb + 10 nloc_max)); the field right-hand
// side with the local potential (FP64, NC = 6, NF = 7) is the largest.
size_t elem_lds_bytes(int32_t nb, int32_t nloc_max) {
    const size_t b = static_cast<size_t>(nb), l = static_cast<size_t>(nloc_max);
    return std::max(sizeof(double) * 6 * b + sizeof(double) * 10 * l, sizeof(double) * (b + 10 * l));
}

namespace {
template <class T>
Cubic<T> cubic_of(const Material &m) {
    return Cubic<T>{static_cast<T>(m.c11), static_cast<T>(m.c12), static_cast<T>(m.c44)};
}

// The sample-frame stiffness; nd: divided by c11 (the FP32 operators' scaling).
template <class T>
Aniso<T> aniso_of(const Material &m, bool nd) {
    Aniso<T> a;
    for (int k = 0; k < 36; ++k) a.c[k] = static_cast<T>(nd ? m.C6[k] / m.c11 : m.C6[k]);
    return a;
}
}  // namespace

// FP64 works in SI units.  FP32 works on the non-dimensional operator
// A' = A / (len_scale * c11): coordinates divided by the mesh length scale and
// stiffness divided by c11, which keeps every product inside FP32's normal range.
template <class T>
void launch_elastic_matvec(const MeshView &mv, const Material &mat, MatvecMode mode, const T *in, T *out, const T *b,
                           const T *r, T *pout, const CGScalars &cg, int k, double tol, hipStream_t s,
                           const hipEvent_t *ev) {
    const bool nd = sizeof(T) == sizeof(float);
    Material m2 = mat;
    if (nd) {
        m2.c12 = mat.c12 / mat.c11;
        m2.c44 = mat.c44 / mat.c11;
        m2.c11 = 1.0;
    }
    if (mat.rot) {
        ElasticMatvecOp<T, Aniso<T>> op{in, out, b, r, pout, cg, k, static_cast<int>(mode), mv.n, tol * tol,
                                        aniso_of<T>(mat, nd), {0}, {0.0}, nd ? 1.0 / mv.len_scale : 1.0};
        run_strip<T, 3, 3>(mv, op, s, ev);
        return;
    }
    ElasticMatvecOp<T> op{in, out, b, r, pout, cg, k, static_cast<int>(mode), mv.n, tol * tol, cubic_of<T>(m2), {0},
                          {0.0}, nd ? 1.0 / mv.len_scale : 1.0};
    run_strip<T, 3, 3>(mv, op, s, ev);
}

template void launch_elastic_matvec<double>(const MeshView &, const Material &, MatvecMode, const double *, double *,
                                            const double *, const double *, double *, const CGScalars &, int, double,
                                            hipStream_t, const hipEvent_t *);
template void launch_elastic_matvec<float>(const MeshView &, const Material &, MatvecMode, const float *, float *,
                                           const float *, const float *, float *, const CGScalars &, int, double,
                                           hipStream_t, const hipEvent_t *);

template <class T>
void launch_elastic_cg(const MeshView &mv, const Material &mat, int k, bool last, const T *rin, const T *pin,
                       const T *qin, T *rout, T *pout, T *qout, T *x, const CGScalars &cg, double tol, hipStream_t s,
                       const hipEvent_t *ev) {
    const bool nd = sizeof(T) == sizeof(float);
    Material m2 = mat;
    if (nd) {
        m2.c12 = mat.c12 / mat.c11;
        m2.c44 = mat.c44 / mat.c11;
        m2.c11 = 1.0;
    }
    if (mat.rot) {
        ElasticCgOp<T, Aniso<T>> op{rin, pin, qin, rout, pout, qout, x, cg, k, mv.n, last ? 1 : 0, tol * tol,
                                    aniso_of<T>(mat, nd), 0.0, 0.0, nd ? 1.0 / mv.len_scale : 1.0};
        run_strip<T, 3, 3>(mv, op, s, ev);
        return;
    }
    ElasticCgOp<T> op{rin, pin, qin, rout, pout, qout, x, cg, k, mv.n, last ? 1 : 0, tol * tol, cubic_of<T>(m2),
                      0.0, 0.0, nd ? 1.0 / mv.len_scale : 1.0};
    run_strip<T, 3, 3>(mv, op, s, ev);
}

template void launch_elastic_cg<double>(const MeshView &, const Material &, int, bool, const double *, const double *,
                                        const double *, double *, double *, double *, double *, const CGScalars &,
                                        double, hipStream_t, const hipEvent_t *);
template void launch_elastic_cg<float>(const MeshView &, const Material &, int, bool, const float *, const float *,
                                       const float *, float *, float *, float *, float *, const CGScalars &, double,
                                       hipStream_t, const hipEvent_t *);

template <class T>
void launch_elastic_pcg(const MeshView &mv, const Material &mat, int k, const T *z, const T *pin, T *pout, T *q,
                        const CGScalars &cg, hipStream_t s, const hipEvent_t *ev) {
    const bool nd = sizeof(T) == sizeof(float);
    Material m2 = mat;
    if (nd) {
        m2.c12 = mat.c12 / mat.c11;
        m2.c44 = mat.c44 / mat.c11;
        m2.c11 = 1.0;
    }
    if (mat.rot) {
        ElasticPcgOp<T, Aniso<T>> op{z, pin, pout, q, cg, k, mv.n, aniso_of<T>(mat, nd), 0.0,
                                     nd ? 1.0 / mv.len_scale : 1.0};
        run_strip<T, 3, 3>(mv, op, s, ev);
        return;
    }
    ElasticPcgOp<T> op{z, pin, pout, q, cg, k, mv.n, cubic_of<T>(m2), 0.0, nd ? 1.0 / mv.len_scale : 1.0};
    run_strip<T, 3, 3>(mv, op, s, ev);
}

template void launch_elastic_pcg<double>(const MeshView &, const Material &, int, const double *, const double *,
                                         double *, double *, const CGScalars &, hipStream_t, const hipEvent_t *);
template void launch_elastic_pcg<float>(const MeshView &, const Material &, int, const float *, const float *,
                                        float *, float *, const CGScalars &, hipStream_t, const hipEvent_t *);

void launch_elastic_rhs(const MeshView &mv, const Material &mat, const double *m, double *b, double *x, double *bb,
                        hipStream_t s) {
    ElasticRhsOp<double> op{m, b, x, bb, mv.n, cubic_of<double>(mat), mat.l100, mat.l111, mat.rot, {}};
    for (int k = 0; k < 9; ++k) op.R[k] = mat.R[k];
    run_elem<double, 3, 3>(mv, op, s);
}

// K^ms on the same strips (all segments), eps = 1 and no mass; FP32 uses the
// GS operator's scaling, A' = K^ms / len_scale^3.
template <class T>
void launch_ms_matvec(const MeshView &mv, int nc, MatvecMode mode, const T *in, T *out, const T *b, const T *r,
                      T *pout, const CGScalars &cg, int k, double tol, hipStream_t s) {
    const bool nd = sizeof(T) == sizeof(float);
    const double sc = nd ? 1.0 / mv.len_scale : 1.0;
    const int md = static_cast<int>(mode);
    const double t2 = tol * tol;
    const T e = static_cast<T>(sc * sc);
    if (nc == 1)
        run_strip<T, 1, 1>(mv, MsMatvecOp<T, 1>{in, out, b, r, pout, cg, k, md, mv.n, t2, e, {0}, {0.0}, sc}, s);
    else
        run_strip<T, 3, 3>(mv, MsMatvecOp<T, 3>{in, out, b, r, pout, cg, k, md, mv.n, t2, e, {0, 0, 0}, {0.0, 0.0, 0.0},
                                                sc}, s);
}

template <class T>
void launch_ms_cg(const MeshView &mv, int k, bool last, const T *rin, const T *pin, const T *qin, T *rout, T *pout,
                  T *qout, T *x, const CGScalars &cg, double tol, hipStream_t s) {
    const bool nd = sizeof(T) == sizeof(float);
    const double sc = nd ? 1.0 / mv.len_scale : 1.0;
    MsCgOp<T> op{rin, pin, qin, rout, pout, qout, x, cg, k, mv.n, last ? 1 : 0, tol * tol, static_cast<T>(sc * sc),
                 0.0, 0.0, sc};
    run_strip<T, 1, 1>(mv, op, s);
}

template void launch_ms_cg<double>(const MeshView &, int, bool, const double *, const double *, const double *,
                                   double *, double *, double *, double *, const CGScalars &, double, hipStream_t);
template void launch_ms_cg<float>(const MeshView &, int, bool, const float *, const float *, const float *, float *,
                                  float *, float *, float *, const CGScalars &, double, hipStream_t);

template void launch_ms_matvec<double>(const MeshView &, int, MatvecMode, const double *, double *, const double *,
                                       const double *, double *, const CGScalars &, int, double, hipStream_t);
template void launch_ms_matvec<float>(const MeshView &, int, MatvecMode, const float *, float *, const float *,
                                      const float *, float *, const CGScalars &, int, double, hipStream_t);

void launch_field_rhs(const MeshView &mv, const Material &mat, const double *m, const double *u, const Derived *d,
                      double c, double *b, double *x0, double *ch2, double *bb, int bbstride, const double *ud,
                      double inv_ms, hipStream_t s) {
    if (ud) {
        FieldRhsOp<double, true> op{m, u, d, ud, inv_ms, b, x0, ch2, bb, mv.n, bbstride, c, cubic_of<double>(mat),
                                    mat.l100, mat.l111, mat.kan, mat.kme, {0, 0, 0, 0, 0, 0}, {0, 0, 0}, mat.rot, {}};
        for (int k = 0; k < 9; ++k) op.R[k] = mat.R[k];
        run_elem<double, 6, 7>(mv, op, s);
    } else {
        FieldRhsOp<double> op{m, u, d, nullptr, 0.0, b, x0, ch2, bb, mv.n, bbstride, c, cubic_of<double>(mat),
                              mat.l100, mat.l111, mat.kan, mat.kme, {0, 0, 0, 0, 0, 0}, {0, 0, 0}, mat.rot, {}};
        for (int k = 0; k < 9; ++k) op.R[k] = mat.R[k];
        run_elem<double, 6, 6>(mv, op, s);
    }
}

void launch_ms_rhs(const MeshView &mv, double Ms, const double *m, double *b, double *x, double *bb,
                   hipStream_t s) {
    MsRhsOp<double> op{m, b, x, bb, mv.n, Ms};
    run_elem<double, 1, 3>(mv, op, s);
}

void launch_mass_rhs(const MeshView &mv, const double *y, const double *ch2, double *b, double *x0, double *bb,
                     int bbstride, hipStream_t s) {
    MassRhsOp<double> op{y, ch2, b, x0, bb, mv.n, bbstride};
    run_elem<double, 2, 2>(mv, op, s);
}

void launch_energy_elem(const MeshView &mv, const Material &mat, const double *m, const double *u, const double *ud,
                        const Derived *d, double *out2, hipStream_t s) {
    const size_t lds = sizeof(double) * (static_cast<size_t>(mv.nb) + 10 * static_cast<size_t>(mv.nloc_max));
    hipLaunchKernelGGL(k_energy_elem<double>, dim3(mv.nblk), dim3(kThreads), lds, s, mv, mat, m, u, ud, d, out2);
    launch_det_finish(mv.det, s);
}

}  // namespace gspm
