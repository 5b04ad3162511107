// Node and grid passes of the elastic preconditioner B = Q A_g^+ Q^T + omega
// D^-1 (elastic_precond; host setup in green.cpp): the restriction Q^T to the
// auxiliary grid, the mode-by-mode inverse of the grid operator between the
// two FFTs, the prolongation Q back to the nodes with the diagonal term, and
// the CG vector update of the preconditioned iteration.  Node vectors are
// component-major [3][n], grid arrays [3][G] real and [3][Gh] complex, so the
// FFTs run as one batch of three.
#include "device_common.h"

namespace gspm {

namespace {

// one thread per item: these passes are bound by the latency of their
// gathers, so every item's loads should be in flight at once
inline int grid_of(int64_t n) {
    const int64_t g = (n + kThreads - 1) / kThreads;
    return static_cast<int>(g < (1 << 30) ? (g > 0 ? g : 1) : (1 << 30));
}

// streaming passes with a per-workgroup reduction: a bounded grid keeps the
// number of atomic adds on the sharded sums small
inline int reduce_grid_of(int64_t n) {
    const int64_t g = (n + kThreads - 1) / kThreads;
    return static_cast<int>(g < 2048 ? (g > 0 ? g : 1) : 2048);
}

// The test of |r_j|^2 <= tol2 |b|^2 (recorded by workgroup 0 as iteration
// j) and the converged state of the set; true when the launch has work.
__device__ __forceinline__ bool pc_live(const CGScalars &cg, int test_k, double tol2) {
    if (cg.done[0] != 0) return false;
    if (test_k < 0) return true;
    const double *const src[2] = {cg.rr_at(0, test_k), cg.bb_at(0)};
    double t[2];
    shard_totals<2>(src, t);
    const int stop = !isfinite(t[0]) ? 2 : (t[0] <= tol2 * t[1] ? 1 : 0);
    if (stop) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            cg.done[0] = stop;
            cg.iters[0] = test_k;
        }
        return false;
    }
    return true;
}

// Trilinear corners of the node at p: the lower grid indices and the weights
// along each axis (FP64), the position wrapped into the periodic cell.
__device__ __forceinline__ void corners(const GreenView &gv, const double p[3], int (&i0)[3], int (&i1)[3],
                                        double (&t)[3]) {
    const int g[3] = {gv.gx, gv.gy, gv.gz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double f = (p[a] - gv.lo[a]) / gv.h[a];
        f -= g[a] * floor(f / g[a]);
        int k = static_cast<int>(floor(f));
        if (k >= g[a]) k = g[a] - 1;
        if (k < 0) k = 0;
        i0[a] = k;
        i1[a] = k + 1 == g[a] ? 0 : k + 1;
        t[a] = f - k;
    }
}

}  // namespace

// Q^T r: each row (a grid point, rows in Morton order so that neighbouring
// threads gather nearby nodes) sums w r over its list, after the test of |r_j|.
template <class T>
__global__ void __launch_bounds__(kThreads) k_pc_restrict(GreenView gv, int n, const T *r, CGScalars cg, int test_k,
                                                          double tol2) {
    if (!pc_live(cg, test_k, tol2)) return;
    const T *w = static_cast<const T *>(gv.rw);
    T *grid = static_cast<T *>(gv.grid);
    constexpr int kB = 8;   // entries gathered per batch: their index loads, then their data loads
    for (int64_t t = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; t < gv.G;
         t += static_cast<int64_t>(gridDim.x) * kThreads) {
        T s0 = T(0), s1 = T(0), s2 = T(0);
        const int e0 = gv.rptr[t], e1 = gv.rptr[t + 1];
        const int64_t g = gv.rgrid[t];
        for (int eb = e0; eb < e1; eb += kB) {
            int j[kB];
            T wj[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                const bool in = eb + u < e1;
                j[u] = in ? gv.rnode[eb + u] : 0;
                wj[u] = in ? w[eb + u] : T(0);
            }
            T v0[kB], v1[kB], v2[kB];
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                v0[u] = r[j[u]];
                v1[u] = r[static_cast<size_t>(n) + j[u]];
                v2[u] = r[2 * static_cast<size_t>(n) + j[u]];
            }
#pragma unroll
            for (int u = 0; u < kB; ++u) {
                s0 += wj[u] * v0[u];
                s1 += wj[u] * v1[u];
                s2 += wj[u] * v2[u];
            }
        }
        // packed for the complex transforms: w0 = x0 + i x1, w1 = x2
        grid[2 * g] = s0;
        grid[2 * g + 1] = s1;
        grid[2 * (gv.G + g)] = s2;
        grid[2 * (gv.G + g) + 1] = T(0);
    }
}

// Y(k) = A(k)^-1 X(k) / G on the packed spectra.  The two complex grids hold
// the transforms of w0 = x0 + i x1 and w1 = x2 (x real), so
//   X0(k) = (W0(k) + conj W0(-k)) / 2,  X1(k) = (W0(k) - conj W0(-k)) / 2i,
//   X2(k) = (W1(k) + conj W1(-k)) / 2,
// and the results go back packed the same way with Y(-k) = conj Y(k) (A(-k)
// = conj A(k) for the real stencil), so the inverse transform returns
// y0 + i y1 and y2.  One thread takes a mode k of the half spectrum (kx <=
// gx / 2, the table's index) together with its mirror -k; a pair whose mirror
// is in the half spectrum too is taken once.
template <class T>
__global__ void __launch_bounds__(kThreads) k_pc_modes(GreenView gv, CGScalars cg) {
    if (cg.done[0] != 0) return;
    const T *M = static_cast<const T *>(gv.ainv);
    T *w0 = static_cast<T *>(gv.spec);      // (re, im) pairs, [2][G]
    T *w1 = w0 + 2 * gv.G;
    for (int64_t m = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; m < gv.Gh;
         m += static_cast<int64_t>(gridDim.x) * kThreads) {
        const int kx = static_cast<int>(m % gv.gxh);
        const int ky = static_cast<int>((m / gv.gxh) % gv.gy);
        const int kz = static_cast<int>(m / (static_cast<int64_t>(gv.gxh) * gv.gy));
        const int mx = (gv.gx - kx) % gv.gx, my = (gv.gy - ky) % gv.gy, mz = (gv.gz - kz) % gv.gz;
        const int64_t f = (static_cast<int64_t>(kz) * gv.gy + ky) * gv.gx + kx;
        const int64_t fm = (static_cast<int64_t>(mz) * gv.gy + my) * gv.gx + mx;
        if (mx < gv.gxh && fm < f) continue;
        const T ar = w0[2 * f], ai = w0[2 * f + 1], br = w0[2 * fm], bi = w0[2 * fm + 1];
        const T cr = w1[2 * f], ci = w1[2 * f + 1], dr = w1[2 * fm], di = w1[2 * fm + 1];
        const T h = T(0.5);
        const T xr[3] = {h * (ar + br), h * (ai + bi), h * (cr + dr)};
        const T xi[3] = {h * (ai - bi), h * (br - ar), h * (ci - di)};
        const T *a = M + 9 * m;
        // off-diagonal (a01, a02, a12) and their conjugates below the diagonal
        const T r01 = a[3], i01 = a[4], r02 = a[5], i02 = a[6], r12 = a[7], i12 = a[8];
        const T yr0 = a[0] * xr[0] + (r01 * xr[1] - i01 * xi[1]) + (r02 * xr[2] - i02 * xi[2]);
        const T yi0 = a[0] * xi[0] + (r01 * xi[1] + i01 * xr[1]) + (r02 * xi[2] + i02 * xr[2]);
        const T yr1 = (r01 * xr[0] + i01 * xi[0]) + a[1] * xr[1] + (r12 * xr[2] - i12 * xi[2]);
        const T yi1 = (r01 * xi[0] - i01 * xr[0]) + a[1] * xi[1] + (r12 * xi[2] + i12 * xr[2]);
        const T yr2 = (r02 * xr[0] + i02 * xi[0]) + (r12 * xr[1] + i12 * xi[1]) + a[2] * xr[2];
        const T yi2 = (r02 * xi[0] - i02 * xr[0]) + (r12 * xi[1] - i12 * xr[1]) + a[2] * xi[2];
        if (fm == f) {
            // a self-conjugate mode: X and A^-1 are real there (up to rounding)
            w0[2 * f] = yr0;
            w0[2 * f + 1] = yr1;
            w1[2 * f] = yr2;
            w1[2 * f + 1] = T(0);
            continue;
        }
        // W0(k) = Y0 + i Y1, W0(-k) = conj Y0 + i conj Y1, W1(+-k) = Y2, conj Y2
        w0[2 * f] = yr0 - yi1;
        w0[2 * f + 1] = yi0 + yr1;
        w0[2 * fm] = yr0 + yi1;
        w0[2 * fm + 1] = yr1 - yi0;
        w1[2 * f] = yr2;
        w1[2 * f + 1] = yi2;
        w1[2 * fm] = yr2;
        w1[2 * fm + 1] = -yi2;
    }
}

// z = Q y + omega D^-1 r at every node; rz += r.z.
template <class T>
__global__ void __launch_bounds__(kThreads) k_pc_prolong(GreenView gv, MeshView mv, const T *r, T *z, double *rz,
                                                         CGScalars cg) {
    if (cg.done[0] != 0) return;
    const int n = mv.n;
    const T *y = static_cast<const T *>(gv.grid);
    const T *dv = static_cast<const T *>(gv.dinv);
    double part = 0.0;
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
        const double p[3] = {mv.x[i], mv.y[i], mv.z[i]};
        int i0[3], i1[3];
        double t[3];
        corners(gv, p, i0, i1, t);
        T acc[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int ix = (c & 1) ? i1[0] : i0[0], iy = (c & 2) ? i1[1] : i0[1], iz = (c & 4) ? i1[2] : i0[2];
            const double wd = ((c & 1) ? t[0] : 1.0 - t[0]) * ((c & 2) ? t[1] : 1.0 - t[1]) *
                              ((c & 4) ? t[2] : 1.0 - t[2]);
            const T wc = static_cast<T>(wd);
            const int64_t g = (static_cast<int64_t>(iz) * gv.gy + iy) * gv.gx + ix;
            // packed: y0 + i y1 in the first complex grid, y2 in the second
            acc[0] += wc * y[2 * g];
            acc[1] += wc * y[2 * g + 1];
            acc[2] += wc * y[2 * (gv.G + g)];
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const size_t o = static_cast<size_t>(a) * n + i;
            const T rv = r[o];
            const T zv = acc[a] + dv[o] * rv;
            z[o] = zv;
            part += static_cast<double>(rv) * zv;
        }
    }
    block_atomic_add1(part, rz, cg.det);
}

template <class T>
__global__ void __launch_bounds__(kThreads) k_pcg_update(int n, T *x, T *r, const T *p, const T *q, CGScalars cg,
                                                         int k) {
    if (cg.done[0] != 0) return;
    const double *const src[2] = {pcg_rz_at(cg, k), cg.pq_at(0, k)};
    double t[2];
    shard_totals<2>(src, t);
    const T alpha = static_cast<T>(t[0] / t[1]);
    double part = 0.0;
    const size_t n3 = 3 * static_cast<size_t>(n);
    for (size_t i = blockIdx.x * static_cast<size_t>(kThreads) + threadIdx.x; i < n3;
         i += static_cast<size_t>(gridDim.x) * kThreads) {
        x[i] += alpha * p[i];
        const T rv = r[i] - alpha * q[i];
        r[i] = rv;
        part += static_cast<double>(rv) * rv;
    }
    block_atomic_add1(part, cg.rr_at(0, k + 1), cg.det);
}

__global__ void __launch_bounds__(kThreads) k_sum3(int n, const double *b, double *aux, DetSums det) {
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads)
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[a] += b[static_cast<size_t>(a) * n + i];
    block_atomic_add<3>(acc, aux, kShards, det);
}

__global__ void __launch_bounds__(kThreads) k_sub_mean3(int n, double *b, const double *aux, double *bb,
                                                        DetSums det) {
    const double *const src[3] = {aux, aux + kShards, aux + 2 * kShards};
    double t[3];
    shard_totals<3>(src, t);
    double part = 0.0;
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const size_t o = static_cast<size_t>(a) * n + i;
            const double v = b[o] - t[a] / n;
            b[o] = v;
            part += v * v;
        }
    block_atomic_add1(part, bb, det);
}

__global__ void k_pin_copy(int n, const double *x, int p0, double *aux) {
    if (threadIdx.x < 3) aux[threadIdx.x] = x[static_cast<size_t>(threadIdx.x) * n + p0];
}

__global__ void __launch_bounds__(kThreads) k_pin_sub(int n, double *x, const double *aux) {
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads)
#pragma unroll
        for (int a = 0; a < 3; ++a) x[static_cast<size_t>(a) * n + i] -= aux[a];
}

// A(k) = sum_o S(o) exp(2 pi i k.o / g) on the half spectrum, inverted by
// cofactors in complex FP64, times factor, stored in its Hermitian form.
struct Stencil27 {
    double s[27 * 9];
};

template <class T>
__global__ void __launch_bounds__(kThreads) k_pc_symbol(GreenView gv, Stencil27 st, double factor) {
    T *out = static_cast<T *>(const_cast<void *>(gv.ainv));
    for (int64_t m = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; m < gv.Gh;
         m += static_cast<int64_t>(gridDim.x) * kThreads) {
        const int kx = static_cast<int>(m % gv.gxh);
        const int ky = static_cast<int>((m / gv.gxh) % gv.gy);
        const int kz = static_cast<int>(m / (static_cast<int64_t>(gv.gxh) * gv.gy));
        T *o = out + 9 * m;
        if (m == 0) {
#pragma unroll
            for (int q = 0; q < 9; ++q) o[q] = T(0);
            continue;
        }
        double ar[3][3] = {}, ai[3][3] = {};
        const double two_pi = 6.283185307179586476925286766559;
        for (int oz = -1; oz <= 1; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    const double ph = two_pi * (static_cast<double>(kx) * ox / gv.gx +
                                                static_cast<double>(ky) * oy / gv.gy +
                                                static_cast<double>(kz) * oz / gv.gz);
                    double sn, cs;
                    sincos(ph, &sn, &cs);
                    const double *S = st.s + 9 * ((oz + 1) * 9 + (oy + 1) * 3 + (ox + 1));
#pragma unroll
                    for (int a = 0; a < 3; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b) {
                            ar[a][b] += S[3 * a + b] * cs;
                            ai[a][b] += S[3 * a + b] * sn;
                        }
                }
        // cofactors: C(i, j) = A(i+1, j+1) A(i+2, j+2) - A(i+1, j+2) A(i+2, j+1)
        double cr[3][3], ci[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const int r0 = (i + 1) % 3, r1 = (i + 2) % 3, c0 = (j + 1) % 3, c1 = (j + 2) % 3;
                const double pr = ar[r0][c0] * ar[r1][c1] - ai[r0][c0] * ai[r1][c1];
                const double pi = ar[r0][c0] * ai[r1][c1] + ai[r0][c0] * ar[r1][c1];
                const double qr = ar[r0][c1] * ar[r1][c0] - ai[r0][c1] * ai[r1][c0];
                const double qi = ar[r0][c1] * ai[r1][c0] + ai[r0][c1] * ar[r1][c0];
                cr[i][j] = pr - qr;
                ci[i][j] = pi - qi;
            }
        double dr = 0.0, di = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            dr += ar[0][j] * cr[0][j] - ai[0][j] * ci[0][j];
            di += ar[0][j] * ci[0][j] + ai[0][j] * cr[0][j];
        }
        const double den = dr * dr + di * di;
        // inverse(i, j) = C(j, i) / det
        auto inv_re = [&](int i, int j) { return (cr[j][i] * dr + ci[j][i] * di) / den * factor; };
        auto inv_im = [&](int i, int j) { return (ci[j][i] * dr - cr[j][i] * di) / den * factor; };
        o[0] = static_cast<T>(inv_re(0, 0));
        o[1] = static_cast<T>(inv_re(1, 1));
        o[2] = static_cast<T>(inv_re(2, 2));
        o[3] = static_cast<T>(inv_re(0, 1));
        o[4] = static_cast<T>(inv_im(0, 1));
        o[5] = static_cast<T>(inv_re(0, 2));
        o[6] = static_cast<T>(inv_im(0, 2));
        o[7] = static_cast<T>(inv_re(1, 2));
        o[8] = static_cast<T>(inv_im(1, 2));
    }
}

template <class T>
void launch_pc_restrict(const GreenView &gv, int n, const T *r, const CGScalars &cg, int test_k, double tol,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_pc_restrict<T>, dim3(grid_of(gv.G)), dim3(kThreads), 0, s, gv, n, r, cg, test_k, tol * tol);
}

template <class T>
void launch_pc_modes(const GreenView &gv, const CGScalars &cg, hipStream_t s) {
    hipLaunchKernelGGL(k_pc_modes<T>, dim3(grid_of(gv.Gh)), dim3(kThreads), 0, s, gv, cg);
}

template <class T>
void launch_pc_prolong(const GreenView &gv, const MeshView &mv, const T *r, T *z, double *rz, const CGScalars &cg,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_pc_prolong<T>, dim3(grid_of(mv.n)), dim3(kThreads), 0, s, gv, mv, r, z, rz, cg);
    launch_det_finish(cg.det, s);
}

template <class T>
void launch_pcg_update(int n, T *x, T *r, const T *p, const T *q, const CGScalars &cg, int k, hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_update<T>, dim3(reduce_grid_of(3 * static_cast<int64_t>(n))), dim3(kThreads), 0, s, n, x, r, p, q,
                       cg, k);
    launch_det_finish(cg.det, s);
}

void launch_remove_mean3(int n, double *b, double *aux, double *bb, hipStream_t s, const DetSums &det) {
    launch_fill(aux, 3 * kShards, 0.0, s);
    launch_fill(bb, kShards, 0.0, s);
    hipLaunchKernelGGL(k_sum3, dim3(reduce_grid_of(n)), dim3(kThreads), 0, s, n, b, aux, det);
    launch_det_finish(det, s);
    hipLaunchKernelGGL(k_sub_mean3, dim3(reduce_grid_of(n)), dim3(kThreads), 0, s, n, b, aux, bb, det);
    launch_det_finish(det, s);
}

void launch_pin_shift(int n, double *x, int p0, double *aux, hipStream_t s) {
    hipLaunchKernelGGL(k_pin_copy, dim3(1), dim3(64), 0, s, n, x, p0, aux);
    hipLaunchKernelGGL(k_pin_sub, dim3(grid_of(n)), dim3(kThreads), 0, s, n, x, aux);
}

template <class T>
void launch_pc_symbol(const GreenView &gv, const double *stencil27, double factor, hipStream_t s) {
    Stencil27 st;
    for (int q = 0; q < 27 * 9; ++q) st.s[q] = stencil27[q];
    hipLaunchKernelGGL(k_pc_symbol<T>, dim3(grid_of(gv.Gh)), dim3(kThreads), 0, s, gv, st, factor);
}

#define GSPM_PC_INST(T)                                                                                              \
    template void launch_pc_restrict<T>(const GreenView &, int, const T *, const CGScalars &, int, double,         \
                                        hipStream_t);                                                               \
    template void launch_pc_modes<T>(const GreenView &, const CGScalars &, hipStream_t);                            \
    template void launch_pc_prolong<T>(const GreenView &, const MeshView &, const T *, T *, double *,               \
                                       const CGScalars &, hipStream_t);                                             \
    template void launch_pcg_update<T>(int, T *, T *, const T *, const T *, const CGScalars &, int, hipStream_t);  \
    template void launch_pc_symbol<T>(const GreenView &, const double *, double, hipStream_t);
GSPM_PC_INST(double)
GSPM_PC_INST(float)
#undef GSPM_PC_INST

}  // namespace gspm
