// Device-side helpers shared by the library's kernels.
#pragma once

#include "common.h"

namespace gspm {

// Workgroups are dispatched round-robin over the eight XCDs (workgroup w goes
// to XCD w % 8).  Give each XCD a contiguous range of owner blocks, so that the
// halo nodes a block gathers were mostly touched by the same XCD's L2.
__device__ __forceinline__ int xcd_block(int wg, int nwg) {
    const int q = nwg >> 3, r = nwg & 7, x = wg & 7, slot = wg >> 3;
    return x * q + (x < r ? x : r) + slot;
}

__device__ __forceinline__ double round_even(double v) { return rint(v); }
__device__ __forceinline__ float round_even(float v) { return rintf(v); }

template <class T>
__device__ __forceinline__ T near_image(T d, T L, T iL) {
    return d - L * round_even(d * iL);
}

// P1 geometry of a tetrahedron from its edge vectors e_k = x_k - x_0: the
// gradients of the barycentric coordinates, g_k = (e_{k+1} x e_{k+2}) / det,
// g_0 = -sum g_k, and the volume |det| / 6.
template <class T>
struct Geo {
    T g[4][3];
    T vol;
};
// Unscaled P1 geometry, for operators that only need products of gradients:
// with e_k = x_k - x_0, c_k = e_{k+1} x e_{k+2} (k = 1..3, cyclic) equals
// det * grad(lambda_k), det = e_1 . c_1 = 6 V with the orientation's sign, and
// w = 1 / (6 |det|) = V / det^2, so that V grad(lambda_i) . grad(lambda_j) =
// w c_i . c_j and V = |det| / 6.  (c_0 = -(c_1 + c_2 + c_3) is left implicit.)
// One reciprocal and no gradient scaling per element.
template <class T>
struct RawGeo {
    T c[4][3];                               // c[1..3] set; c[0] unused
    T adet, w;                               // |det|, 1 / (6 |det|)
};

__device__ __forceinline__ float rcp_approx(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_approx(double x) { return 1.0 / x; }

// Crystal orientation (App. D), R row-major with v_sample = R v_crystal.
// c = R^T v (sample -> crystal) and v = R c (crystal -> sample).
template <class T>
__device__ __forceinline__ void to_crystal3(const double *R, const T (&v)[3], T (&c)[3]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) c[a] = R[a] * v[0] + R[3 + a] * v[1] + R[6 + a] * v[2];
}

template <class T>
__device__ __forceinline__ void to_sample3(const double *R, const T (&c)[3], T (&v)[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) v[i] = R[3 * i] * c[0] + R[3 * i + 1] * c[1] + R[3 * i + 2] * c[2];
}

// A symmetric tensor (xx yy zz yz xz xy): R A R^T (to the sample frame) or
// R^T A R (to the crystal frame).
template <class T>
__device__ __forceinline__ void sym_rotate(const double *R, bool to_sample, const T (&a)[6], T (&b)[6]) {
    const T A[3][3] = {{a[0], a[5], a[4]}, {a[5], a[1], a[3]}, {a[4], a[3], a[2]}};
    T Q[3][3], X[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Q[i][j] = static_cast<T>(to_sample ? R[3 * i + j] : R[3 * j + i]);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) X[i][j] = Q[i][0] * A[0][j] + Q[i][1] * A[1][j] + Q[i][2] * A[2][j];
    T B[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) B[i][j] = X[i][0] * Q[j][0] + X[i][1] * Q[j][1] + X[i][2] * Q[j][2];
    b[0] = B[0][0]; b[1] = B[1][1]; b[2] = B[2][2];
    b[3] = B[1][2]; b[4] = B[0][2]; b[5] = B[0][1];
}

template <class T>
__device__ __forceinline__ void tet_raw_geometry(const T (&e)[3][3], RawGeo<T> &R) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T *a = e[(k + 1) % 3], *b = e[(k + 2) % 3];
        R.c[k + 1][0] = a[1] * b[2] - a[2] * b[1];
        R.c[k + 1][1] = a[2] * b[0] - a[0] * b[2];
        R.c[k + 1][2] = a[0] * b[1] - a[1] * b[0];
    }
    R.adet = fabs(e[0][0] * R.c[1][0] + e[0][1] * R.c[1][1] + e[0][2] * R.c[1][2]);
    R.w = rcp_approx(T(6) * R.adet);
}

template <class T>
__device__ __forceinline__ void tet_geometry_from_edges(const T (&e)[3][3], Geo<T> &G) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T *a = e[(k + 1) % 3], *b = e[(k + 2) % 3];
        G.g[k + 1][0] = a[1] * b[2] - a[2] * b[1];
        G.g[k + 1][1] = a[2] * b[0] - a[0] * b[2];
        G.g[k + 1][2] = a[0] * b[1] - a[1] * b[0];
    }
    const T det = e[0][0] * G.g[1][0] + e[0][1] * G.g[1][1] + e[0][2] * G.g[1][2];
    const T inv = T(1) / det;
#pragma unroll
    for (int k = 1; k < 4; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) G.g[k][a] *= inv;
#pragma unroll
    for (int a = 0; a < 3; ++a) G.g[0][a] = -(G.g[1][a] + G.g[2][a] + G.g[3][a]);
    G.vol = fabs(det) * T(1.0 / 6.0);
}

// Workgroup sums of NR per-thread values: wave shuffles, then per-wave totals
// in LDS (fixed order).
template <int NR>
__device__ __forceinline__ void block_partials(const double (&v)[NR], double (&red)[kThreads / 64][NR]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        double s = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) red[wv][k] = s;
    }
    __syncthreads();
}

// The workgroup total s of sum k (thread k) to its destination: an atomic add
// to shard (blockIdx.x % kShards), or in the deterministic mode a store to
// the workgroup's slot of sum base + k (workgroup 0 records the destination
// and how many sums the launch produced).
__device__ __forceinline__ void sum_out(int k, int nr, double s, double *dst, const DetSums &det, int base) {
    if (det.part == nullptr) {
        if (dst != nullptr) unsafeAtomicAdd(dst + (blockIdx.x % kShards), s);
        return;
    }
    // (every launch that adds sums is sized within max_blocks at upload; the test only keeps a
    // mis-sized launch inside the slot array)
    if (static_cast<int>(blockIdx.x) < det.max_blocks)
        det.part[static_cast<size_t>(base + k) * det.max_blocks + blockIdx.x] = s;
    if (blockIdx.x == 0) {
        det.dst[base + k] = dst;
        if (k == 0) *det.count = base + nr;
    }
}

// Sum NR per-thread values over the workgroup and add the totals with one FP64
// atomic each to shard (blockIdx.x % kShards) of the sharded scalars
// dst + k * stride (deterministic mode: to the workgroup's slots, see sum_out).
// Spreading the atomics of thousands of workgroups over kShards addresses keeps
// them from serialising on one.  All threads of the workgroup call it.
template <int NR>
__device__ __forceinline__ void block_atomic_add(const double (&v)[NR], double *dst, int stride,
                                                 const DetSums &det = DetSums{}, int base = 0) {
    __shared__ double red[kThreads / 64][NR];
    block_partials<NR>(v, red);
    if (threadIdx.x < NR && dst != nullptr) {
        double s = 0.0;
#pragma unroll
        for (int w2 = 0; w2 < kThreads / 64; ++w2) s += red[w2][threadIdx.x];
        sum_out(threadIdx.x, NR, s, dst + threadIdx.x * stride, det, base);
    }
}

// The same with the NR totals going to NR separate sharded scalars (a null
// destination drops its total).
template <int NR>
__device__ __forceinline__ void block_atomic_add_to(const double (&v)[NR], double *const (&dst)[NR],
                                                    const DetSums &det = DetSums{}, int base = 0) {
    __shared__ double red[kThreads / 64][NR];
    block_partials<NR>(v, red);
    if (threadIdx.x < NR) {
        double s = 0.0;
#pragma unroll
        for (int w2 = 0; w2 < kThreads / 64; ++w2) s += red[w2][threadIdx.x];
        sum_out(threadIdx.x, NR, s, dst[threadIdx.x], det, base);
    }
}

__device__ __forceinline__ void block_atomic_add1(double v, double *dst, const DetSums &det = DetSums{},
                                                  int base = 0) {
    const double a[1] = {v};
    block_atomic_add<1>(a, dst, 0, det, base);
}

// Totals of NR sharded scalars (each kShards consecutive doubles at src[k]),
// summed in a fixed order by the first wave and broadcast through LDS.  All
// threads of the workgroup call it.
template <int NR>
__device__ __forceinline__ void shard_totals(const double *const (&src)[NR], double (&out)[NR]) {
    static_assert(kShards <= 32, "one shard per lane of the low half-wave");
    __shared__ double tot[NR];
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        // every load in flight before the first reduction: the sums sit on the
        // critical path of each launch that needs them
        double v[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) v[k] = 0.0;
        if (lane < kShards) {
#pragma unroll
            for (int k = 0; k < NR; ++k)
                if (src[k] != nullptr) v[k] = src[k][lane];
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            double s = v[k];
#pragma unroll
            for (int off = 16; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
            if (lane == 0) tot[k] = s;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NR; ++k) out[k] = tot[k];
    __syncthreads();
}

__device__ __forceinline__ double shard_total(const double *src) {
    const double *const a[1] = {src};
    double o[1];
    shard_totals<1>(a, o);
    return o[0];
}

// Totals of the CG scalars an iteration's matvec needs: rr[k], rr[k-1], bb
// per scalar set; decides convergence of rr[k] (recorded by workgroup 0) and
// the direction coefficient beta_k = rr[k] / rr[k-1].
template <int NS>
__device__ __forceinline__ bool cg_direction_scalars(const CGScalars &cg, int k, double tol2, int (&live)[NS],
                                                     double (&beta)[NS]) {
    __shared__ int32_t flags[NS];
    if (threadIdx.x == 0)
        for (int s = 0; s < NS; ++s) flags[s] = cg.done[s];
    __syncthreads();
    for (int s = 0; s < NS; ++s) {
        live[s] = flags[s] == 0;
        beta[s] = 0.0;
    }
    __syncthreads();
    if (k == 0) {
        bool any = false;
        for (int s = 0; s < NS; ++s) any |= live[s] != 0;
        return any;
    }
    const double *src[3 * NS];
    for (int s = 0; s < NS; ++s) {
        src[s] = cg.rr_at(s, k);
        src[NS + s] = cg.rr_at(s, k - 1);
        src[2 * NS + s] = cg.bb_at(s);
    }
    double t[3 * NS];
    shard_totals<3 * NS>(src, t);
    bool any = false;
    int stop[NS];
    for (int s = 0; s < NS; ++s) {
        stop[s] = 0;
        if (!live[s]) continue;
        const double rrk = t[s];
        if (!isfinite(rrk)) stop[s] = 2;
        else if (rrk <= tol2 * t[2 * NS + s]) stop[s] = 1;
        else beta[s] = rrk / t[NS + s];
        if (stop[s]) live[s] = 0;
        any |= live[s] != 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int s = 0; s < NS; ++s)
            if (stop[s]) {
                cg.done[s] = stop[s];
                cg.iters[s] = k;
            }
    return any;
}

}  // namespace gspm
