// Node-parallel kernels of the GSPM step: fills, volume averages, the
// quantities derived from them, the CG vector updates and the GSPM node
// updates.  Vectors are component-major [c][n]; one thread per node per
// grid-stride step, so every access is coalesced.
#include <mutex>

#include "device_common.h"

namespace gspm {

namespace {

template <class T>
struct Vec16;
template <>
struct Vec16<float> {
    using type = float4;
};
template <>
struct Vec16<double> {
    using type = double2;
};

inline int node_grid(int64_t n) {
    const int64_t g = (n + kThreads - 1) / kThreads;
    return static_cast<int>(g < 2048 ? (g > 0 ? g : 1) : 2048);
}

}  // namespace

// ------------------------------------------------------------------- fills

__global__ void __launch_bounds__(kThreads) k_fill(double *p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kThreads)
        p[i] = v;
}

__global__ void __launch_bounds__(kThreads) k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kThreads)
        p[i] = v;
}

void launch_fill(double *p, int64_t n, double v, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(node_grid(n)), dim3(kThreads), 0, s, p, n, v);
}

void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3(node_grid(n)), dim3(kThreads), 0, s, p, n, v);
}

// ------------------------------------------------- corrected GS start vector

// x0 <- x0 + corr (the last step's correction, when `use`), start <- x0
__global__ void __launch_bounds__(kThreads) k_gs_start(int64_t n, double *x, const double *corr, double *start,
                                                       int use) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kThreads) {
        const double v = use ? x[i] + corr[i] : x[i];
        x[i] = v;
        start[i] = v;
    }
}

// corr <- corr + x - start: the solution minus the lumped start
__global__ void __launch_bounds__(kThreads) k_gs_correction(int64_t n, const double *x, const double *start,
                                                            double *corr, int use) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kThreads)
        corr[i] = (use ? corr[i] : 0.0) + (x[i] - start[i]);
}

void launch_gs_start(int64_t n, double *x, const double *corr, double *start, bool use, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_gs_start, dim3(node_grid(n)), dim3(kThreads), 0, s, n, x, corr, start, use ? 1 : 0);
}

void launch_gs_correction(int64_t n, const double *x, const double *start, double *corr, bool use, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_gs_correction, dim3(node_grid(n)), dim3(kThreads), 0, s, n, x, start, corr, use ? 1 : 0);
}

// ------------------------------------------------ host-visible small values

// Small results the host polls are written straight into its pinned memory
// (device-accessible), and small inputs arrive as kernel arguments: a copy
// engine transfer of a few bytes costs more device time than these launches.
__global__ void __launch_bounds__(64) k_i32_to_host(const int32_t *src, int count, int32_t *dst) {
    if (static_cast<int>(threadIdx.x) < count) dst[threadIdx.x] = src[threadIdx.x];
    __threadfence_system();
}

void launch_i32_to_host(const int32_t *src, int count, int32_t *host_dst, hipStream_t s) {
    hipLaunchKernelGGL(k_i32_to_host, dim3(1), dim3(64), 0, s, src, count, host_dst);
}

__global__ void __launch_bounds__(64) k_totals_to_host(ShardSources src, int count, double *dst) {
    const int lane = threadIdx.x;
    double v[ShardSources::kMax];
#pragma unroll
    for (int k = 0; k < ShardSources::kMax; ++k) v[k] = (k < count && lane < kShards) ? src.p[k][lane] : 0.0;
#pragma unroll
    for (int k = 0; k < ShardSources::kMax; ++k) {
        double t = v[k];
#pragma unroll
        for (int off = 16; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
        if (lane == 0 && k < count) dst[k] = t;
    }
    __threadfence_system();
}

void launch_totals_to_host(const ShardSources &src, int count, double *host_dst, hipStream_t s) {
    hipLaunchKernelGGL(k_totals_to_host, dim3(1), dim3(64), 0, s, src, count, host_dst);
}

// ---------------------------------------------------------------- averages

// Volume averages of Sec. 2.4 for P1 fields: int_Omega g = sum_j w_j g_j with
// the magnetic lumped weights w_j (m and E0(m) vanish in the inclusions).
// With a rotated crystal (App. D) the E0 sums are taken at the crystal-frame
// m_c = R^T m and k_derive carries their mean back to the sample frame.
__global__ void __launch_bounds__(kThreads) k_avg_sums(int n, const double *w, const double *m, Material mat,
                                                       double *sums, DetSums det) {
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const double a = 1.5 * mat.l100, b = 1.5 * mat.l111, third = 1.0 / 3.0;
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
        const double wi = w[i];
        double m0 = m[i], m1 = m[n + i], m2 = m[2 * static_cast<size_t>(n) + i];
        acc[0] += wi * m0;
        acc[1] += wi * m1;
        acc[2] += wi * m2;
        if (mat.rot) {
            const double ms[3] = {m0, m1, m2};
            double mc[3];
            to_crystal3(mat.R, ms, mc);
            m0 = mc[0]; m1 = mc[1]; m2 = mc[2];
        }
        acc[3] += wi * a * (m0 * m0 - third);
        acc[4] += wi * a * (m1 * m1 - third);
        acc[5] += wi * a * (m2 * m2 - third);
        acc[6] += wi * b * m1 * m2;
        acc[7] += wi * b * m0 * m2;
        acc[8] += wi * b * m0 * m1;
    }
    block_atomic_add<9>(acc, sums, kShards, det);
}

void launch_avg_sums(int n, const double *w, const double *m, const Material &mat, double *sums, hipStream_t s,
                     const DetSums &det) {
    launch_fill(sums, 9 * kShards, 0.0, s);
    hipLaunchKernelGGL(k_avg_sums, dim3(node_grid(n)), dim3(kThreads), 0, s, n, w, m, mat, sums, det);
    launch_det_finish(det, s);
}

// mbar = sum w m / V_c; Ebar = <E0(m)> + C^-1 sigma_ext (the homogeneous strain
// that minimises the energy when the heterogeneous strain has zero mean);
// hc = H_ext / Ms - N_d mbar (Zeeman plus far-field demagnetisation, Sec. 2.1).
__global__ void __launch_bounds__(kThreads) k_derive(const double *sums, DeriveArgs a, Derived *out) {
    const double *const src[9] = {sums, sums + kShards, sums + 2 * kShards, sums + 3 * kShards, sums + 4 * kShards,
                                  sums + 5 * kShards, sums + 6 * kShards, sums + 7 * kShards, sums + 8 * kShards};
    double t[9];
    shard_totals<9>(src, t);
    if (threadIdx.x == 0) {
        double mb[3];
        for (int k = 0; k < 3; ++k) mb[k] = t[k] / a.vc;
        for (int k = 0; k < 3; ++k) out->mbar[k] = mb[k];
        double e0[6];
        for (int k = 0; k < 6; ++k) e0[k] = t[3 + k] / a.vc;
        if (a.rot) {
            const double ec[6] = {e0[0], e0[1], e0[2], e0[3], e0[4], e0[5]};
            sym_rotate(a.R, true, ec, e0);
        }
        for (int k = 0; k < 6; ++k) out->ebar[k] = e0[k] + a.csig[k];
        for (int k = 0; k < 3; ++k)
            out->hc[k] = a.hz[k] - (a.Nd[3 * k] * mb[0] + a.Nd[3 * k + 1] * mb[1] + a.Nd[3 * k + 2] * mb[2]);
    }
}

void launch_derive(const double *sums, const DeriveArgs &a, Derived *out, hipStream_t s) {
    hipLaunchKernelGGL(k_derive, dim3(1), dim3(kThreads), 0, s, sums, a, out);
}

// ------------------------------------------- averages without allocation

// Device memory of gspm_averages_noalloc: per-workgroup partial sums
// [group][9], the nine totals in the sharded layout k_derive reads, and the
// Derived record.  One copy per GPU, held until the process ends; every call
// on a GPU overwrites it, so calls that overlap on one GPU race.  Host code
// never passes `scratch` itself (in host code the name is a stand-in, not a
// device address): it uses the address hipGetSymbolAddress returns for the
// current device (noalloc_scratch_address).
constexpr int kNaPartials = kNaMaxGroups * 9;
constexpr int kNaSums = 9 * kShards;
constexpr int kNaDerived = 16;
static_assert(sizeof(Derived) <= kNaDerived * sizeof(double), "Derived record larger than its scratch slot");
static __device__ __align__(256) double scratch[kNaPartials + kNaSums + kNaDerived];

namespace {
std::mutex g_na_mutex;
double *g_na_ptr[kNaMaxDevices] = {};
}  // namespace

int noalloc_scratch_address(int device, double **out) {
    *out = nullptr;
    if (device < 0 || device >= kNaMaxDevices) return static_cast<int>(hipErrorInvalidDevice);
    std::lock_guard<std::mutex> lock(g_na_mutex);
    if (!g_na_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return static_cast<int>(e);
        g_na_ptr[device] = static_cast<double *>(p);
    }
    *out = g_na_ptr[device];
    return 0;
}

// Sum NR per-thread values over the workgroup in a fixed order (wave
// shuffles, then the waves in order); every thread gets the totals.
template <int NR>
__device__ __forceinline__ void block_sum_fixed(double (&v)[NR]) {
    __shared__ double red[kThreads / 64][NR];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        double s = v[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
        if (lane == 0) red[wv][k] = s;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NR; ++k) {
        double s = 0.0;
#pragma unroll
        for (int w2 = 0; w2 < kThreads / 64; ++w2) s += red[w2][k];
        v[k] = s;
    }
    __syncthreads();
}

// The sums of k_avg_sums with m in the caller's node order (n_user x 3,
// row-major, read at one caller node `rep[i]` of each unique node i); group g
// covers the unique nodes [g kNaNodesPerGroup, (g + 1) kNaNodesPerGroup) and
// writes its nine sums to partials[9 g ..] (no atomics).
__global__ void __launch_bounds__(kThreads) k_avg_partials_user(int n, const double *w, const int32_t *rep,
                                                                const double *m_user, Material mat,
                                                                double *partials) {
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const double a = 1.5 * mat.l100, b = 1.5 * mat.l111, third = 1.0 / 3.0;
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kNaNodesPerGroup;
    for (int t = threadIdx.x; t < kNaNodesPerGroup; t += kThreads) {
        const int64_t i = base + t;
        if (i >= n) break;
        const double wi = w[i];
        const double *mu = m_user + 3 * static_cast<int64_t>(rep[i]);
        double m0 = mu[0], m1 = mu[1], m2 = mu[2];
        acc[0] += wi * m0;
        acc[1] += wi * m1;
        acc[2] += wi * m2;
        if (mat.rot) {
            const double ms[3] = {m0, m1, m2};
            double mc[3];
            to_crystal3(mat.R, ms, mc);
            m0 = mc[0]; m1 = mc[1]; m2 = mc[2];
        }
        acc[3] += wi * a * (m0 * m0 - third);
        acc[4] += wi * a * (m1 * m1 - third);
        acc[5] += wi * a * (m2 * m2 - third);
        acc[6] += wi * b * m1 * m2;
        acc[7] += wi * b * m0 * m2;
        acc[8] += wi * b * m0 * m1;
    }
    block_sum_fixed<9>(acc);
    if (threadIdx.x < 9) partials[9 * static_cast<int64_t>(blockIdx.x) + threadIdx.x] = acc[threadIdx.x];
}

// One workgroup: the totals of `groups` partial sums in a fixed order, stored
// as shard 0 of the sharded layout (the other shards zero).
__global__ void __launch_bounds__(kThreads) k_avg_fold(int groups, const double *partials, double *sums) {
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int g = threadIdx.x; g < groups; g += kThreads)
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[k] += partials[9 * static_cast<int64_t>(g) + k];
    block_sum_fixed<9>(acc);
    for (int q = threadIdx.x; q < kNaSums; q += kThreads) sums[q] = (q % kShards == 0) ? acc[q / kShards] : 0.0;
}

__global__ void k_avg_out(const Derived *der, double *out) {
    const int t = threadIdx.x;
    if (t < 3) out[t] = der->mbar[t];
    else if (t < 9) out[t] = der->ebar[t - 3];
}

int launch_averages_noalloc(double *scr, int n, const double *w, const int32_t *rep, const double *m_user,
                            const Material &mat, const DeriveArgs &da, double *out, hipStream_t s) {
    const int groups = static_cast<int>((static_cast<int64_t>(n) + kNaNodesPerGroup - 1) / kNaNodesPerGroup);
    if (groups < 1 || groups > kNaMaxGroups) return static_cast<int>(hipErrorInvalidValue);
    double *partials = scr, *sums = scr + kNaPartials;
    Derived *der = reinterpret_cast<Derived *>(scr + kNaPartials + kNaSums);
    hipLaunchKernelGGL(k_avg_partials_user, dim3(groups), dim3(kThreads), 0, s, n, w, rep, m_user, mat, partials);
    hipLaunchKernelGGL(k_avg_fold, dim3(1), dim3(kThreads), 0, s, groups, partials, sums);
    hipLaunchKernelGGL(k_derive, dim3(1), dim3(kThreads), 0, s, sums, da, der);
    hipLaunchKernelGGL(k_avg_out, dim3(1), dim3(64), 0, s, der, out);
    return static_cast<int>(hipGetLastError());
}

// Anisotropy and Zeeman energies by the vertex rule: sum_j w_j psi(m_j).
__global__ void __launch_bounds__(kThreads) k_energy_nodes(int n, const double *w, const double *m, Material mat,
                                                           double h0, double h1, double h2, double *out,
                                                           DetSums det) {
    double acc[2] = {0.0, 0.0};
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
        const double m0 = m[i], m1 = m[n + i], m2 = m[2 * static_cast<size_t>(n) + i];
        double c[3] = {m0, m1, m2};
        if (mat.rot) {
            const double ms[3] = {m0, m1, m2};
            to_crystal3(mat.R, ms, c);    // anisotropy of the crystal-frame components (App. D)
        }
        acc[0] += w[i] * mat.K1 * (c[0] * c[0] * c[1] * c[1] + c[1] * c[1] * c[2] * c[2] + c[2] * c[2] * c[0] * c[0]);
        acc[1] -= w[i] * mat.mu0Ms * (h0 * m0 + h1 * m1 + h2 * m2);
    }
    block_atomic_add<2>(acc, out, kShards, det);
}

void launch_energy_nodes(int n, const double *w, const double *m, const Material &mat, const double hext[3],
                         double *out2, hipStream_t s, const DetSums &det) {
    hipLaunchKernelGGL(k_energy_nodes, dim3(node_grid(n)), dim3(kThreads), 0, s, n, w, m, mat, hext[0], hext[1],
                       hext[2], out2, det);
    launch_det_finish(det, s);
}

// ---------------------------------------------------------------------- CG

namespace {

// Scalar set of component c (all components share set 0 when joint).
__device__ __forceinline__ int set_of(int c, int joint) { return joint ? 0 : c; }

// Which of the ns solves are still running.  One thread reads the flags and
// broadcasts them, so every wave of the workgroup takes the same decision
// even while workgroup 0 of the direction kernel is writing them.
__device__ __forceinline__ bool read_live(const int32_t *done, int ns, bool (&live)[3]) {
    __shared__ int32_t f[3];
    if (threadIdx.x == 0)
        for (int s = 0; s < 3; ++s) f[s] = s < ns ? done[s] : 1;
    __syncthreads();
    bool any = false;
    for (int s = 0; s < 3; ++s) {
        live[s] = f[s] == 0;
        any |= live[s];
    }
    __syncthreads();
    return any;
}

}  // namespace

// After the residual matvec: b = 0 gives x = 0 with no iterations; a
// residual already below tol ||b|| converges with no iterations.
template <class T>
__global__ void __launch_bounds__(kThreads) k_cg_start(int n, int nc, int joint, T *x, CGScalars cg, double tol2) {
    const int ns = joint ? 1 : nc;
    const double *const src[6] = {cg.bb_at(0), ns > 1 ? cg.bb_at(1) : nullptr, ns > 2 ? cg.bb_at(2) : nullptr,
                                  cg.rr_at(0, 0), ns > 1 ? cg.rr_at(1, 0) : nullptr, ns > 2 ? cg.rr_at(2, 0) : nullptr};
    double t[6];
    shard_totals<6>(src, t);
    bool zero[3], conv[3];
    for (int s = 0; s < 3; ++s) {
        zero[s] = s < ns && t[s] == 0.0;
        conv[s] = s < ns && (zero[s] || t[3 + s] <= tol2 * t[s]);
    }
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads)
        for (int c = 0; c < nc; ++c)
            if (zero[set_of(c, joint)]) x[static_cast<size_t>(c) * n + i] = T(0);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        for (int s = 0; s < ns; ++s)
            if (conv[s]) {
                cg.done[s] = 1;
                cg.iters[s] = 0;
            }
}

// Iteration k, after the matvec wrote p_k, q = A p_k and pq[k]:
// alpha = rr[k] / pq[k]; x += alpha p; r -= alpha q; rr[k+1] += r.r.  The
// convergence test of rr[k+1] and the next direction happen in the next
// iteration's matvec.
template <class T>
__global__ void __launch_bounds__(kThreads) k_cg_update(int n, int nc, int joint, int flat, T *x, T *r, const T *p,
                                                        const T *q, CGScalars cg, int k) {
    const int ns = joint ? 1 : nc;
    bool live[3];
    if (!read_live(cg.done, ns, live)) return;
    const double *const src[6] = {cg.rr_at(0, k), ns > 1 ? cg.rr_at(1, k) : nullptr, ns > 2 ? cg.rr_at(2, k) : nullptr,
                                  cg.pq_at(0, k), ns > 1 ? cg.pq_at(1, k) : nullptr, ns > 2 ? cg.pq_at(2, k) : nullptr};
    double t[6];
    shard_totals<6>(src, t);
    double alpha[3];
    for (int s = 0; s < 3; ++s) alpha[s] = live[s] ? t[s] / t[3 + s] : 0.0;
    double part[3] = {0.0, 0.0, 0.0};
    constexpr int W = 16 / sizeof(T);
    using V = typename Vec16<T>::type;
    const int tid = blockIdx.x * kThreads + threadIdx.x, nthr = gridDim.x * kThreads;
    auto vec = [&](size_t o, T a, double &acc) {
        V xv = *reinterpret_cast<const V *>(x + o);
        V rv = *reinterpret_cast<const V *>(r + o);
        const V pv = *reinterpret_cast<const V *>(p + o);
        const V qv = *reinterpret_cast<const V *>(q + o);
        T *xe = reinterpret_cast<T *>(&xv), *re = reinterpret_cast<T *>(&rv);
        const T *pe = reinterpret_cast<const T *>(&pv), *qe = reinterpret_cast<const T *>(&qv);
#pragma unroll
        for (int j = 0; j < W; ++j) {
            xe[j] += a * pe[j];
            re[j] -= a * qe[j];
            acc += static_cast<double>(re[j]) * re[j];
        }
        *reinterpret_cast<V *>(x + o) = xv;
        *reinterpret_cast<V *>(r + o) = rv;
    };
    if (flat) {
        // joint solve, one step length for every component: the nc components
        // are one contiguous array of nc * n values (each 16-byte aligned at
        // its start, the host checks), streamed as 16-byte vectors, two per
        // lane per pass, then a scalar tail
        if (!live[0]) return;
        const T a = static_cast<T>(alpha[0]);
        const size_t m = static_cast<size_t>(nc) * n, nv = m / W;
        size_t v = tid;
        for (; v + nthr < nv; v += 2 * static_cast<size_t>(nthr)) {
            vec(v * W, a, part[0]);
            vec((v + nthr) * W, a, part[0]);
        }
        if (v < nv) vec(v * W, a, part[0]);
        for (size_t i = nv * W + tid; i < m; i += nthr) {
            x[i] += a * p[i];
            const T rv = r[i] - a * q[i];
            r[i] = rv;
            part[0] += static_cast<double>(rv) * rv;
        }
        block_atomic_add<3>(part, cg.rr_at(0, k + 1), cg.comp_stride(), cg.det);
        return;
    }
    // per component: a scalar head up to the first 16-byte boundary, a body of
    // 16-byte vectors (4 floats or 2 doubles per lane per load), a scalar tail
    for (int c = 0; c < nc; ++c) {
        const int s = set_of(c, joint);
        if (!live[s]) continue;
        const size_t c0 = static_cast<size_t>(c) * n;
        const T a = static_cast<T>(alpha[s]);
        const int head = min(n, static_cast<int>((W - c0 % W) % W));
        const int nv = (n - head) / W;
        auto scalar = [&](int i) {
            const size_t o = c0 + i;
            x[o] += a * p[o];
            const T rv = r[o] - a * q[o];
            r[o] = rv;
            part[s] += static_cast<double>(rv) * rv;
        };
        if (tid < head) scalar(tid);
        for (int v = tid; v < nv; v += nthr) vec(c0 + head + static_cast<size_t>(v) * W, a, part[s]);
        for (int i = head + nv * W + tid; i < n; i += nthr) scalar(i);
    }
    block_atomic_add<3>(part, cg.rr_at(0, k + 1), cg.comp_stride(), cg.det);
}

// Convergence test of rr[k] alone (after the last permitted iteration, when no
// further matvec will test it): ||r|| <= tol ||b|| converges with k
// iterations, a non-finite residual breaks down.  One workgroup.
__global__ void __launch_bounds__(kThreads) k_cg_check(int nc, int joint, CGScalars cg, int k, double tol2) {
    const int ns = joint ? 1 : nc;
    bool live[3];
    if (!read_live(cg.done, ns, live)) return;
    const double *const src[6] = {cg.rr_at(0, k), ns > 1 ? cg.rr_at(1, k) : nullptr, ns > 2 ? cg.rr_at(2, k) : nullptr,
                                  cg.bb_at(0), ns > 1 ? cg.bb_at(1) : nullptr, ns > 2 ? cg.bb_at(2) : nullptr};
    double t[6];
    shard_totals<6>(src, t);
    if (threadIdx.x == 0)
        for (int s = 0; s < ns; ++s) {
            if (!live[s]) continue;
            if (!isfinite(t[s])) {
                cg.done[s] = 2;
                cg.iters[s] = k;
            } else if (t[s] <= tol2 * t[3 + s]) {
                cg.done[s] = 1;
                cg.iters[s] = k;
            }
        }
}

template <class T>
void launch_cg_start(int n, int nc, bool joint, T *x, const CGScalars &cg, double tol, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_start<T>, dim3(node_grid(n)), dim3(kThreads), 0, s, n, nc, joint ? 1 : 0, x, cg, tol * tol);
}

template <class T>
void launch_cg_update(int n, int nc, bool joint, T *x, T *r, const T *p, const T *q, const CGScalars &cg, int k,
                      hipStream_t s) {
    auto a16 = [](const void *v) { return (reinterpret_cast<uintptr_t>(v) & 15u) == 0; };
    const int flat = joint && a16(x) && a16(r) && a16(p) && a16(q) ? 1 : 0;
    hipLaunchKernelGGL(k_cg_update<T>, dim3(node_grid(n)), dim3(kThreads), 0, s, n, nc, joint ? 1 : 0, flat, x, r, p, q,
                       cg, k);
    launch_det_finish(cg.det, s);
}

template void launch_cg_start<double>(int, int, bool, double *, const CGScalars &, double, hipStream_t);
template void launch_cg_start<float>(int, int, bool, float *, const CGScalars &, double, hipStream_t);
template void launch_cg_update<double>(int, int, bool, double *, double *, const double *, const double *,
                                       const CGScalars &, int, hipStream_t);
template void launch_cg_update<float>(int, int, bool, float *, float *, const float *, const float *,
                                      const CGScalars &, int, hipStream_t);

// ------------------------------------------------------ precision conversions

__global__ void __launch_bounds__(kThreads) k_to_f32(int64_t n, const double *src, float *dst) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kThreads)
        dst[i] = static_cast<float>(src[i]);
}

__global__ void __launch_bounds__(kThreads) k_add_f32(int64_t n, double *x, const float *d) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kThreads)
        x[i] += static_cast<double>(d[i]);
}

__global__ void __launch_bounds__(kThreads) k_fill_f32(float *p, int64_t n) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * kThreads)
        p[i] = 0.0f;
}

// The start of an inner FP32 solve of the mixed form in one launch: the
// inner scalars (threshold and per-component done flags, written by
// workgroup 0), r32 = (float) (scale * r64) on nc components with ||r32||^2
// per scalar set into slot 0 of the r.r ring (zeroed by an earlier launch),
// and x32 = 0 on nx values.
__global__ void __launch_bounds__(kThreads) k_inner_start(int n, int nc, int joint, const double *src, double scale,
                                                          float *dst, float *x32, int64_t nx, CGScalars cg,
                                                          InnerStart st) {
    if (blockIdx.x == 0) {
        const int t = threadIdx.x;
        if (t < kMaxComp * kShards) cg.bb[t] = (t % kShards == 0) ? st.bb[t / kShards] : 0.0;
        if (t < kMaxComp) {
            cg.done[t] = st.done[t];
            cg.iters[t] = 0;
        }
    }
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < nx;
         i += static_cast<int64_t>(gridDim.x) * kThreads)
        x32[i] = 0.0f;
    double part[3] = {0.0, 0.0, 0.0};
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads)
        for (int c = 0; c < nc; ++c) {
            const size_t o = static_cast<size_t>(c) * n + i;
            const float v = static_cast<float>(scale * src[o]);
            dst[o] = v;
            part[joint ? 0 : c] += static_cast<double>(v) * v;
        }
    block_atomic_add<3>(part, cg.rr_at(0, 0), cg.comp_stride(), cg.det);
}

void launch_inner_start(int n, int nc, bool joint, const double *src, double scale, float *dst, float *x32,
                        int64_t nx, const CGScalars &cg, const InnerStart &st, hipStream_t s) {
    static_assert(kMaxComp * kShards <= kThreads, "one workgroup sets every shard");
    hipLaunchKernelGGL(k_inner_start, dim3(node_grid(n)), dim3(kThreads), 0, s, n, nc, joint ? 1 : 0, src, scale, dst,
                       x32, nx, cg, st);
    launch_det_finish(cg.det, s);
}

void launch_to_f32(int64_t n, const double *src, float *dst, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_to_f32, dim3(node_grid(n)), dim3(kThreads), 0, s, n, src, dst);
}

void launch_add_f32(int64_t n, double *x, const float *d, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_add_f32, dim3(node_grid(n)), dim3(kThreads), 0, s, n, x, d);
}

void launch_fill_f32(float *p, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill_f32, dim3(node_grid(n)), dim3(kThreads), 0, s, p, n);
}

void launch_cg_check(int nc, bool joint, const CGScalars &cg, int k, double tol, hipStream_t s) {
    hipLaunchKernelGGL(k_cg_check, dim3(1), dim3(kThreads), 0, s, nc, joint ? 1 : 0, cg, k, tol * tol);
}

// ------------------------------------------------------ GSPM node updates

// Algorithm B.1, Step 2, rows 1 and 2 (time-n values as printed):
// m1* = m1 + g2 m3 - g3 m2, m2* = m2 + g3 m1 - g1 m3; m3* starts as m3.
__global__ void __launch_bounds__(kThreads) k_update_m12(int n, const double *m, const double *g, double *ms) {
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
        const size_t n1 = n, n2 = 2 * static_cast<size_t>(n);
        const double m0 = m[i], m1 = m[n1 + i], m2 = m[n2 + i];
        const double g0 = g[i], g1 = g[n1 + i], g2 = g[n2 + i];
        ms[i] = m0 + (g1 * m2 - g2 * m1);
        ms[n1 + i] = m1 + (g2 * m0 - g0 * m2);
        ms[n2 + i] = m2;
    }
}

// Step 2, row 3: m3* = m3 + g*1 m2* - g*2 m1*.
__global__ void __launch_bounds__(kThreads) k_update_m3(int n, const double *m, const double *gs, double *ms) {
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
        const size_t n1 = n, n2 = 2 * static_cast<size_t>(n);
        ms[n2 + i] = m[n2 + i] + (gs[i] * ms[n1 + i] - gs[n1 + i] * ms[i]);
    }
}

// Step 4: m^{n+1} = m** / |m**| on magnetic nodes (zero elsewhere), written to
// mnew; sums |m^{n+1} - m^n| for the convergence measure of Sec. 3.2; flags a
// zero or non-finite m**.
__global__ void __launch_bounds__(kThreads) k_normalize(int n, const double *w, const double *mss, const double *mold,
                                                        double *mnew, double *dm_sum, int32_t *bad, DetSums det) {
    double dsum = 0.0;
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
        const size_t n1 = n, n2 = 2 * static_cast<size_t>(n);
        if (!(w[i] > 0.0)) {
            mnew[i] = 0.0;
            mnew[n1 + i] = 0.0;
            mnew[n2 + i] = 0.0;
            continue;
        }
        const double a = mss[i], b = mss[n1 + i], c = mss[n2 + i];
        const double rr = sqrt(a * a + b * b + c * c);
        if (!(rr > 0.0) || !isfinite(rr)) {
            *bad = 1;
            continue;
        }
        const double inv = 1.0 / rr;
        const double na = a * inv, nb = b * inv, nc = c * inv;
        const double da = na - mold[i], db = nb - mold[n1 + i], dc = nc - mold[n2 + i];
        dsum += sqrt(da * da + db * db + dc * dc);
        mnew[i] = na;
        mnew[n1 + i] = nb;
        mnew[n2 + i] = nc;
    }
    block_atomic_add1(dsum, dm_sum, det);
}

// Zero the ring slots that iterations [rr_from, rr_to) of r.r and
// [pq_from, pq_to) of p.Ap will accumulate into; with `reset` also the b.b
// shards and the done and iteration flags of every component (a new solve).
__global__ void __launch_bounds__(kThreads) k_zero_ring(CGScalars cg, int ns, int rr_from, int rr_to, int pq_from,
                                                        int pq_to, int reset) {
    if (reset && blockIdx.x == 0) {
        const int t = threadIdx.x;
        if (t < kMaxComp * kShards) cg.bb[t] = 0.0;
        if (t < kMaxComp) {
            cg.done[t] = 0;
            cg.iters[t] = 0;
        }
    }
    const int nrr = rr_to - rr_from, npq = pq_to - pq_from;
    const int total = ns * (nrr + npq) * kShards;
    for (int t = blockIdx.x * kThreads + threadIdx.x; t < total; t += gridDim.x * kThreads) {
        const int sh = t % kShards, rest = t / kShards;
        const int c = rest % ns, slot = rest / ns;
        double *base = slot < nrr ? cg.rr_at(c, rr_from + slot) : cg.pq_at(c, pq_from + slot - nrr);
        base[sh] = 0.0;
        // r . D^-1 r of the Jacobi-preconditioned solves shares the r.r slots
        if (slot < nrr && cg.rz) cg.rz_at(c, rr_from + slot)[sh] = 0.0;
        // the single-reduction GS sums share the p.q slots of their component
        if (slot >= nrr && cg.rzq) {
            cg.rzq_at(c, pq_from + slot - nrr)[sh] = 0.0;
            cg.qzq_at(c, pq_from + slot - nrr)[sh] = 0.0;
        }
        // the single-reduction sums of one scalar set share the p.q slots
        if (slot >= nrr && c == 0 && cg.rq) {
            cg.rq_at(pq_from + slot - nrr)[sh] = 0.0;
            cg.qq_at(pq_from + slot - nrr)[sh] = 0.0;
        }
    }
}

void launch_zero_ring(const CGScalars &cg, int ns, int rr_from, int rr_to, int pq_from, int pq_to, hipStream_t s) {
    const int total = ns * ((rr_to - rr_from) + (pq_to - pq_from)) * kShards;
    if (total <= 0) return;
    hipLaunchKernelGGL(k_zero_ring, dim3(node_grid(total)), dim3(kThreads), 0, s, cg, ns, rr_from, rr_to, pq_from,
                       pq_to, 0);
}

void launch_cg_reset(const CGScalars &cg, int ns, hipStream_t s) {
    static_assert(kMaxComp * kShards <= kThreads, "one workgroup clears every shard");
    hipLaunchKernelGGL(k_zero_ring, dim3(node_grid(ns * kShards)), dim3(kThreads), 0, s, cg, ns, 0, 1, 0, 0, 1);
}

void launch_update_m12(int n, const double *m, const double *g, double *ms, hipStream_t s) {
    hipLaunchKernelGGL(k_update_m12, dim3(node_grid(n)), dim3(kThreads), 0, s, n, m, g, ms);
}

void launch_update_m3(int n, const double *m, const double *gs, double *ms, hipStream_t s) {
    hipLaunchKernelGGL(k_update_m3, dim3(node_grid(n)), dim3(kThreads), 0, s, n, m, gs, ms);
}

void launch_normalize(int n, const double *w, const double *mss, const double *mold, double *mnew, double *dm_sum,
                      int32_t *bad, hipStream_t s, const DetSums &det) {
    hipLaunchKernelGGL(k_normalize, dim3(node_grid(n)), dim3(kThreads), 0, s, n, w, mss, mold, mnew, dm_sum, bad, det);
    launch_det_finish(det, s);
}

// ------------------------------------------------------- deterministic sums

// The recorded sums of the last producer launch: each sum's workgroup slots
// added in workgroup order (every thread a strided run, then a fixed
// reduction tree) to shard 0 of its destination, and the slots cleared.
__global__ void __launch_bounds__(kThreads) k_det_finish(DetSums det) {
    const int k = blockIdx.x;
    if (k >= *det.count) return;
    double *slots = det.part + static_cast<size_t>(k) * det.max_blocks;
    double acc = 0.0;
    for (int b = threadIdx.x; b < det.max_blocks; b += kThreads) {
        acc += slots[b];
        slots[b] = 0.0;
    }
    __shared__ double red[kThreads / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) red[wv] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w2 = 0; w2 < kThreads / 64; ++w2) t += red[w2];
        double *d = det.dst[k];
        if (d != nullptr) d[0] += t;
    }
}

void launch_det_finish(const DetSums &det, hipStream_t s) {
    if (det.part != nullptr) hipLaunchKernelGGL(k_det_finish, dim3(kDetSlots), dim3(kThreads), 0, s, det);
}

}  // namespace gspm
