// Kernels of the learned elastic warm start (layout and network in mpnn.h).
//
// Node GEMMs run on MFMA (v_mfma_f32_16x16x32_bf16): the output is computed
// transposed, out^T = W x in^T, so the weights are the A operand (held in VGPRs
// for the whole launch) and each lane stores four consecutive channels of one
// node row.  Edge passes give one wave to a node with lane = channel, so every
// neighbour row is one coalesced 128-byte read; the neighbour's edge vector is
// computed once per lane-slot and broadcast with readlane.
#include <cmath>

#include "device_common.h"
#include "mpnn.h"

namespace gspm {
namespace mpnn {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = kThreads / 64;
constexpr int kBatch = 8;       // neighbour rows loaded before they are used (edge passes)

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

// FP32 -> BF16 bits, round to nearest, ties to even; NaN stays NaN.
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float round_bf(float f) { return bf2f(f2bf(f)); }

__device__ __forceinline__ float silu(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = __builtin_amdgcn_rcpf(1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

__device__ __forceinline__ float rdlane(float v, int t) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), t));
}
__device__ __forceinline__ int rdlane(int v, int t) { return __builtin_amdgcn_readlane(v, t); }

__device__ __forceinline__ bf16x8 as_bf8(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

// Eight consecutive BF16 values of an input row as an MFMA operand; FP32
// sources are rounded to BF16 on the way.
__device__ __forceinline__ bf16x8 load8(const uint16_t *p) { return as_bf8(*reinterpret_cast<const uint4 *>(p)); }
__device__ __forceinline__ bf16x8 load8(const float *p) {
    const float4 a = reinterpret_cast<const float4 *>(p)[0], b = reinterpret_cast<const float4 *>(p)[1];
    uint4 r;
    r.x = f2bf(a.x) | (static_cast<uint32_t>(f2bf(a.y)) << 16);
    r.y = f2bf(a.z) | (static_cast<uint32_t>(f2bf(a.w)) << 16);
    r.z = f2bf(b.x) | (static_cast<uint32_t>(f2bf(b.y)) << 16);
    r.w = f2bf(b.z) | (static_cast<uint32_t>(f2bf(b.w)) << 16);
    return as_bf8(r);
}

int grid_for(int64_t items, int per_block) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return static_cast<int>(g);
}

// Mean spacing, nearest-image edge vector (x_j - x_i) / hbar in FP32.
__device__ __forceinline__ void edge_vec(const MeshView &mv, float ihbar, double xi, double yi, double zi, int j,
                                         float &ex, float &ey, float &ez) {
    ex = static_cast<float>(near_image(mv.x[j] - xi, mv.Lx, mv.iLx)) * ihbar;
    ey = static_cast<float>(near_image(mv.y[j] - yi, mv.Ly, mv.iLy)) * ihbar;
    ez = static_cast<float>(near_image(mv.z[j] - zi, mv.Lz, mv.iLz)) * ihbar;
}

// ------------------------------------------------------------ node GEMMs

enum Epi { EPI_BF16 = 0, EPI_RESID_BF16 = 1, EPI_F32 = 2, EPI_ADD2_F32 = 3 };

struct GemmArgs {
    void *out;
    int ldo;
    const uint16_t *res;        // EPI_RESID_BF16: out = res + acc + bias
    int ldr;
    const float *bias;
    const float *add0, *add1;   // EPI_ADD2_F32: out = acc + add0 + add1
    int lda0, lda1;
};

// out[r][o] = sum_k in[r][k] W[o][k] for r < n, with in = [src0 | src1]
// (64 columns each when K = 128, src0 alone when K = 64).  W is O x K BF16.
template <int O, int K, class TIn, int EPI>
__global__ void __launch_bounds__(kThreads) k_rowgemm(int n, const TIn *src0, int ld0, const TIn *src1, int ld1,
                                                      const uint16_t *W, GemmArgs ga) {
    constexpr int OT = O / 16, KS = K / 32;
    const int lane = threadIdx.x & 63, grp = lane >> 4, col = lane & 15;
    bf16x8 wa[OT][KS];
#pragma unroll
    for (int ot = 0; ot < OT; ++ot)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) wa[ot][ks] = load8(W + (ot * 16 + col) * K + ks * 32 + grp * 8);
    const int ntile = (n + 15) >> 4;
    for (int tile = blockIdx.x * kWaves + (threadIdx.x >> 6); tile < ntile; tile += gridDim.x * kWaves) {
        const int row = tile * 16 + col;
        const bool live = row < n;
        bf16x8 xb[KS];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int k = ks * 32 + grp * 8;
            if (!live) {
                xb[ks] = as_bf8(make_uint4(0, 0, 0, 0));
            } else if (K == 64 || k < 64) {
                xb[ks] = load8(src0 + static_cast<size_t>(row) * ld0 + k);
            } else {
                xb[ks] = load8(src1 + static_cast<size_t>(row) * ld1 + (k - 64));
            }
        }
        floatx4 acc[OT];
#pragma unroll
        for (int ot = 0; ot < OT; ++ot) {
            acc[ot] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
                acc[ot] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[ot][ks], xb[ks], acc[ot], 0, 0, 0);
        }
        if (!live) continue;
#pragma unroll
        for (int ot = 0; ot < OT; ++ot) {
            const int o = ot * 16 + grp * 4;     // this lane holds out[row][o .. o+3]
            float v[4] = {acc[ot][0], acc[ot][1], acc[ot][2], acc[ot][3]};
            if (EPI == EPI_BF16 || EPI == EPI_RESID_BF16) {
                if (EPI == EPI_RESID_BF16) {
                    const uint2 rr = *reinterpret_cast<const uint2 *>(ga.res + static_cast<size_t>(row) * ga.ldr + o);
                    v[0] += bf2f(rr.x & 0xffffu) + ga.bias[o];
                    v[1] += bf2f(rr.x >> 16) + ga.bias[o + 1];
                    v[2] += bf2f(rr.y & 0xffffu) + ga.bias[o + 2];
                    v[3] += bf2f(rr.y >> 16) + ga.bias[o + 3];
                }
                uint2 st;
                st.x = f2bf(v[0]) | (static_cast<uint32_t>(f2bf(v[1])) << 16);
                st.y = f2bf(v[2]) | (static_cast<uint32_t>(f2bf(v[3])) << 16);
                *reinterpret_cast<uint2 *>(static_cast<uint16_t *>(ga.out) + static_cast<size_t>(row) * ga.ldo + o) =
                    st;
            } else {
                if (EPI == EPI_ADD2_F32) {
                    const float4 a0 = *reinterpret_cast<const float4 *>(ga.add0 + static_cast<size_t>(row) * ga.lda0 + o);
                    const float4 a1 = *reinterpret_cast<const float4 *>(ga.add1 + static_cast<size_t>(row) * ga.lda1 + o);
                    v[0] += a0.x + a1.x;
                    v[1] += a0.y + a1.y;
                    v[2] += a0.z + a1.z;
                    v[3] += a0.w + a1.w;
                }
                *reinterpret_cast<float4 *>(static_cast<float *>(ga.out) + static_cast<size_t>(row) * ga.ldo + o) =
                    make_float4(v[0], v[1], v[2], v[3]);
            }
        }
    }
}

template <int O, int K, class TIn, int EPI>
void rowgemm(int n, const TIn *src0, int ld0, const TIn *src1, int ld1, const uint16_t *W, const GemmArgs &ga,
             hipStream_t s) {
    hipLaunchKernelGGL((k_rowgemm<O, K, TIn, EPI>), dim3(grid_for((n + 15) / 16, kWaves)), dim3(kThreads), 0, s, n,
                       src0, ld0, src1, ld1, W, ga);
}

// Weight gradients: part[wg][o][k] = sum over the workgroup's rows of
// G[r][o] X[r][k], G FP32 (n x O, row stride ldg), X = [x0 | x1] BF16 (K
// columns).  Rows are staged 32 at a time into LDS, transposed, so that each
// MFMA operand is one 16-byte LDS read.
template <int O, int K>
__global__ void __launch_bounds__(kThreads) k_wgrad(int n, int rows_per_wg, const float *G, int ldg, const uint16_t *x0,
                                                    int ldx0, const uint16_t *x1, int ldx1, float *part) {
    constexpr int OT = O / 16, KT = K / 16, TILES = OT * KT, PER_WAVE = TILES / kWaves;
    __shared__ __align__(16) uint16_t gs[O * 32];
    __shared__ __align__(16) uint16_t xs[K * 32];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, grp = lane >> 4, col = lane & 15;
    const int r0 = blockIdx.x * rows_per_wg, r1 = min(n, r0 + rows_per_wg);
    floatx4 acc[PER_WAVE];
#pragma unroll
    for (int t = 0; t < PER_WAVE; ++t) acc[t] = floatx4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int base = r0; base < r1; base += 32) {
        __syncthreads();
        for (int idx = threadIdx.x; idx < 32 * O; idx += kThreads) {
            const int rr = idx / O, o = idx % O, row = base + rr;
            gs[o * 32 + rr] = row < r1 ? f2bf(G[static_cast<size_t>(row) * ldg + o]) : uint16_t(0);
        }
        for (int idx = threadIdx.x; idx < 32 * K; idx += kThreads) {
            const int rr = idx / K, k = idx % K, row = base + rr;
            uint16_t v = 0;
            if (row < r1) v = (K == 64 || k < 64) ? x0[static_cast<size_t>(row) * ldx0 + k]
                                                   : x1[static_cast<size_t>(row) * ldx1 + (k - 64)];
            xs[k * 32 + rr] = v;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < PER_WAVE; ++t) {
            const int tile = wv * PER_WAVE + t, ot = tile / KT, kt = tile % KT;
            const bf16x8 a = as_bf8(*reinterpret_cast<const uint4 *>(gs + (ot * 16 + col) * 32 + grp * 8));
            const bf16x8 b = as_bf8(*reinterpret_cast<const uint4 *>(xs + (kt * 16 + col) * 32 + grp * 8));
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
        }
    }
    float *dst = part + static_cast<size_t>(blockIdx.x) * kPartStride;
#pragma unroll
    for (int t = 0; t < PER_WAVE; ++t) {
        const int tile = wv * PER_WAVE + t, ot = tile / KT, kt = tile % KT;
#pragma unroll
        for (int i = 0; i < 4; ++i) dst[(ot * 16 + grp * 4 + i) * K + kt * 16 + col] = acc[t][i];
    }
}

// grad[off + j] = sum_w part[w][j] (FP64 accumulation in a fixed order).
__global__ void __launch_bounds__(kThreads) k_reduce_part(const float *part, int nwg, int count, float *out) {
    for (int j = blockIdx.x * kThreads + threadIdx.x; j < count; j += gridDim.x * kThreads) {
        double s = 0.0;
        for (int w = 0; w < nwg; ++w) s += part[static_cast<size_t>(w) * kPartStride + j];
        out[j] = static_cast<float>(s);
    }
}

void reduce_part(const float *part, int nwg, int count, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_part, dim3(grid_for(count, kThreads)), dim3(kThreads), 0, s, part, nwg, count, out);
}

// ------------------------------------------------------------ node passes

// Sharded sums of w |m - mprev|^2 and w.
__global__ void __launch_bounds__(kThreads) k_dm_sums(int n, const double *w, const double *m, const double *mp,
                                                      double *red) {
    double a[2] = {0.0, 0.0};
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
        double d2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double d = m[static_cast<size_t>(c) * n + i] - mp[static_cast<size_t>(c) * n + i];
            d2 += d * d;
        }
        a[0] += w[i] * d2;
        a[1] += w[i];
    }
    block_atomic_add<2>(a, red + R_DM2 * kShards, kShards);
}

__device__ __forceinline__ double dm_scale(const double *red) {
    const double *const src[2] = {red + R_DM2 * kShards, red + R_W * kShards};
    double t[2];
    shard_totals<2>(src, t);
    return t[1] > 0.0 ? sqrt(t[0] / t[1]) : 0.0;
}

// The 7 node inputs tag [dm / s_m, m, 1] (zero off the magnetic nodes),
// rounded to BF16 as the network stores them.
__device__ __forceinline__ void node_features(int n, int i, const double *w, const double *m, const double *mp,
                                              double ism, float (&x)[kIn]) {
    const bool mag = w[i] > 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double mc = m[static_cast<size_t>(c) * n + i];
        x[c] = mag ? round_bf(static_cast<float>((mc - mp[static_cast<size_t>(c) * n + i]) * ism)) : 0.0f;
        x[3 + c] = mag ? round_bf(static_cast<float>(mc)) : 0.0f;
    }
    x[6] = mag ? 1.0f : 0.0f;
}

// h0 = SiLU(W0 x + b0); one wave per node, lane = channel.
__global__ void __launch_bounds__(kThreads) k_encode(int n, const double *w, const double *m, const double *mp,
                                                     const double *red, const float *wr, uint16_t *H0) {
    const double sm = dm_scale(red), ism = sm > 0.0 ? 1.0 / sm : 0.0;
    const int lane = threadIdx.x & 63;
    float w0[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) w0[k] = wr[kOffW0 + lane * kIn + k];
    const float b0 = wr[kOffB0 + lane];
    for (int i = blockIdx.x * kWaves + (threadIdx.x >> 6); i < n; i += gridDim.x * kWaves) {
        float x[kIn];
        node_features(n, i, w, m, mp, ism, x);
        float pre = b0;
#pragma unroll
        for (int k = 0; k < kIn; ++k) pre += w0[k] * x[k];
        H0[static_cast<size_t>(i) * kHid + lane] = f2bf(silu(pre));
    }
}

// a_i = mean_j SiLU(A_i + B_j + We e_ij + c).
__global__ void __launch_bounds__(kThreads) k_edge_fwd(Graph g, MeshView mv, const float *wl, const uint16_t *AB,
                                                       uint16_t *AGG) {
    const int lane = threadIdx.x & 63;
    const float we0 = wl[kLWe + lane * 3], we1 = wl[kLWe + lane * 3 + 1], we2 = wl[kLWe + lane * 3 + 2];
    const float cb = wl[kLC + lane];
    for (int i = blockIdx.x * kWaves + (threadIdx.x >> 6); i < g.n; i += gridDim.x * kWaves) {
        const int beg = g.ptr[i], end = g.ptr[i + 1];
        const float ai = bf2f(AB[static_cast<size_t>(i) * 128 + lane]) + cb;
        const double xi = mv.x[i], yi = mv.y[i], zi = mv.z[i];
        float acc = 0.0f;
        for (int base = beg; base < end; base += 64) {
            const int cnt = min(64, end - base);
            int jl = 0;
            float ex = 0.0f, ey = 0.0f, ez = 0.0f;
            if (lane < cnt) {
                jl = g.nbr[base + lane];
                edge_vec(mv, g.ihbar, xi, yi, zi, jl, ex, ey, ez);
            }
            // eight neighbour rows in flight at a time: the loads are issued
            // back to back (indices clamped to the last neighbour), then used
            for (int t0 = 0; t0 < cnt; t0 += kBatch) {
                float bv[kBatch];
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const int j = rdlane(jl, min(t0 + u, cnt - 1));
                    bv[u] = bf2f(AB[static_cast<size_t>(j) * 128 + 64 + lane]);
                }
#pragma unroll
                for (int u = 0; u < kBatch; ++u) {
                    const int t = t0 + u;
                    if (t < cnt) {
                        const float z = ai + bv[u] + we0 * rdlane(ex, t) + we1 * rdlane(ey, t) + we2 * rdlane(ez, t);
                        acc += silu(z);
                    }
                }
            }
        }
        const int deg = end - beg;
        AGG[static_cast<size_t>(i) * kHid + lane] = f2bf(deg > 0 ? acc / static_cast<float>(deg) : 0.0f);
    }
}

// y = Wd h + bd (FP32, n x 3); optionally d = scale (y - y_p0) as 3 x n FP64.
__global__ void __launch_bounds__(kThreads) k_decode(int n, int p0, const uint16_t *H, const float *wr,
                                                     const double *red, double lambda100, double hbar, float *y,
                                                     double *dvec) {
    const double sm = dm_scale(red), scale = lambda100 * hbar * sm;
    auto dec = [&](int i, float (&o)[3]) {
        o[0] = wr[kOffBd];
        o[1] = wr[kOffBd + 1];
        o[2] = wr[kOffBd + 2];
        const uint4 *row = reinterpret_cast<const uint4 *>(H + static_cast<size_t>(i) * kHid);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const uint4 v = row[q];
            const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int c = q * 8 + h * 2;
                const float h0 = bf2f(u[h] & 0xffffu), h1 = bf2f(u[h] >> 16);
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    o[a] += wr[kOffWd + a * kHid + c] * h0 + wr[kOffWd + a * kHid + c + 1] * h1;
            }
        }
    };
    float op[3] = {0.0f, 0.0f, 0.0f};
    if (dvec) dec(p0, op);
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
        float o[3];
        dec(i, o);
#pragma unroll
        for (int a = 0; a < 3; ++a) y[static_cast<size_t>(i) * 3 + a] = o[a];
        if (dvec) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
                dvec[static_cast<size_t>(a) * n + i] = i == p0 ? 0.0 : scale * (static_cast<double>(o[a]) - op[a]);
        }
    }
}

// ------------------------------------------------------------ loss

// Sharded sums of y (3) and of the normalised target t = du / (lambda100 hbar s_m) (3).
__global__ void __launch_bounds__(kThreads) k_loss_sums(int n, const float *y, const double *du, double lambda100,
                                                        double hbar, double *red) {
    const double sm = dm_scale(red);
    const double it = sm > 0.0 ? 1.0 / (lambda100 * hbar * sm) : 0.0;
    double a[6] = {0, 0, 0, 0, 0, 0};
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a[c] += y[static_cast<size_t>(i) * 3 + c];
            a[3 + c] += du[static_cast<size_t>(c) * n + i] * it;
        }
    }
    block_atomic_add<6>(a, red + R_Y * kShards, kShards);
}

// gy = 2 ((y - ybar) - (t - tbar)) / (3n); loss = sum of squares / (3n).
__global__ void __launch_bounds__(kThreads) k_loss_grad(int n, const float *y, const double *du, double lambda100,
                                                        double hbar, double *red, float *gy) {
    const double sm = dm_scale(red);
    const double it = sm > 0.0 ? 1.0 / (lambda100 * hbar * sm) : 0.0;
    const double *const src[6] = {red + R_Y * kShards,       red + (R_Y + 1) * kShards, red + (R_Y + 2) * kShards,
                                  red + R_T * kShards,       red + (R_T + 1) * kShards, red + (R_T + 2) * kShards};
    double mean[6];
    shard_totals<6>(src, mean);
    const double inv3n = 1.0 / (3.0 * n);
    double acc[1] = {0.0};
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double d = (y[static_cast<size_t>(i) * 3 + c] - mean[c] / n) -
                             (du[static_cast<size_t>(c) * n + i] * it - mean[3 + c] / n);
            acc[0] += d * d * inv3n;
            gy[static_cast<size_t>(i) * 3 + c] = static_cast<float>(2.0 * d * inv3n);
        }
    }
    block_atomic_add<1>(acc, red + R_LOSS * kShards, kShards);
}

// ------------------------------------------------------------ backward

// Sum NV per-lane FP32 values over the workgroup's waves; lane c (< lanes)
// writes value k to dst[c * sl + k * sk].
template <int NV>
__device__ __forceinline__ void wave_sum_to_part(const float (&v)[NV], float *dst, int lanes, int sl, int sk) {
    __shared__ float red[kWaves][NV][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wv][k][lane] = v[k];
    __syncthreads();
    if (threadIdx.x < lanes) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            float s = 0.0f;
#pragma unroll
            for (int q = 0; q < kWaves; ++q) s += red[q][k][lane];
            dst[lane * sl + k * sk] = s;
        }
    }
    __syncthreads();
}

// Partial column sums of an n x 64 FP32 matrix (the bias gradient).
__global__ void __launch_bounds__(kThreads) k_colsum(int n, const float *G, float *part) {
    const int lane = threadIdx.x & 63;
    float s[1] = {0.0f};
    for (int i = blockIdx.x * kWaves + (threadIdx.x >> 6); i < n; i += gridDim.x * kWaves)
        s[0] += G[static_cast<size_t>(i) * kHid + lane];
    wave_sum_to_part<1>(s, part + static_cast<size_t>(blockIdx.x) * kPartStride, 64, 1, 0);
}

// gh = gy Wd (n x 64); partials of dWd (3 x 64, [a][c]) and dbd (3).
__global__ void __launch_bounds__(kThreads) k_dec_bwd(int n, const uint16_t *H, const float *gy, const float *wr,
                                                      float *gh, float *part) {
    const int lane = threadIdx.x & 63;
    const float wd0 = wr[kOffWd + lane], wd1 = wr[kOffWd + kHid + lane], wd2 = wr[kOffWd + 2 * kHid + lane];
    float sw[3] = {0.0f, 0.0f, 0.0f}, sb[3] = {0.0f, 0.0f, 0.0f};
    for (int i = blockIdx.x * kWaves + (threadIdx.x >> 6); i < n; i += gridDim.x * kWaves) {
        const float g0 = gy[static_cast<size_t>(i) * 3], g1 = gy[static_cast<size_t>(i) * 3 + 1],
                    g2 = gy[static_cast<size_t>(i) * 3 + 2];
        const float h = bf2f(H[static_cast<size_t>(i) * kHid + lane]);
        gh[static_cast<size_t>(i) * kHid + lane] = g0 * wd0 + g1 * wd1 + g2 * wd2;
        sw[0] += g0 * h;
        sw[1] += g1 * h;
        sw[2] += g2 * h;
        sb[0] += g0;     // every lane sees the same gy; lane 0's sums are the ones kept
        sb[1] += g1;
        sb[2] += g2;
    }
    float *dst = part + static_cast<size_t>(blockIdx.x) * kPartStride;
    wave_sum_to_part<3>(sw, dst, 64, 1, kHid);
    wave_sum_to_part<3>(sb, dst + 3 * kHid, 1, 0, 1);
}

// Edge backward of one layer: given ga = d a (from gha[:, 64:]), writes
// gab = [dA | dB] and partials of dWe (64 x 3) and dc (64).
__global__ void __launch_bounds__(kThreads) k_edge_bwd(Graph g, MeshView mv, const float *wl, const uint16_t *AB,
                                                       const float *gha, float *gab, float *part) {
    const int lane = threadIdx.x & 63;
    const float we0 = wl[kLWe + lane * 3], we1 = wl[kLWe + lane * 3 + 1], we2 = wl[kLWe + lane * 3 + 2];
    const float cb = wl[kLC + lane];
    float s[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int v = blockIdx.x * kWaves + (threadIdx.x >> 6); v < g.n; v += gridDim.x * kWaves) {
        const int beg = g.ptr[v], end = g.ptr[v + 1], deg = end - beg;
        const float av = bf2f(AB[static_cast<size_t>(v) * 128 + lane]) + cb;
        const float bv = bf2f(AB[static_cast<size_t>(v) * 128 + 64 + lane]) + cb;
        const float gav = deg > 0 ? gha[static_cast<size_t>(v) * 128 + 64 + lane] / static_cast<float>(deg) : 0.0f;
        const double xv = mv.x[v], yv = mv.y[v], zv = mv.z[v];
        float gA = 0.0f, gB = 0.0f;
        for (int base = beg; base < end; base += 64) {
            const int cnt = min(64, end - base);
            int ul = 0;
            float ex = 0.0f, ey = 0.0f, ez = 0.0f, idu = 0.0f;
            if (lane < cnt) {
                ul = g.nbr[base + lane];
                edge_vec(mv, g.ihbar, xv, yv, zv, ul, ex, ey, ez);
                const int du = g.ptr[ul + 1] - g.ptr[ul];
                idu = du > 0 ? 1.0f / static_cast<float>(du) : 0.0f;
            }
            for (int t0 = 0; t0 < cnt; t0 += kBatch) {
                float au[kBatch], bu[kBatch], gu[kBatch];
#pragma unroll
                for (int q = 0; q < kBatch; ++q) {
                    const size_t ru = static_cast<size_t>(rdlane(ul, min(t0 + q, cnt - 1))) * 128;
                    au[q] = bf2f(AB[ru + lane]);
                    bu[q] = bf2f(AB[ru + 64 + lane]);
                    gu[q] = gha[ru + 64 + lane];
                }
#pragma unroll
                for (int q = 0; q < kBatch; ++q) {
                    const int t = t0 + q;
                    if (t >= cnt) continue;
                    const float e0 = rdlane(ex, t), e1 = rdlane(ey, t), e2 = rdlane(ez, t);
                    const float wde = we0 * e0 + we1 * e1 + we2 * e2;
                    // edge v -> u (message into v)
                    const float g1 = gav * dsilu(av + bu[q] + wde);
                    gA += g1;
                    s[0] += g1 * e0;
                    s[1] += g1 * e1;
                    s[2] += g1 * e2;
                    s[3] += g1;
                    // edge u -> v (message into u), edge vector -e
                    const float g2 = gu[q] * rdlane(idu, t) * dsilu(au[q] + bv - wde);
                    gB += g2;
                }
            }
        }
        gab[static_cast<size_t>(v) * 128 + lane] = gA;
        gab[static_cast<size_t>(v) * 128 + 64 + lane] = gB;
    }
    float *dst = part + static_cast<size_t>(blockIdx.x) * kPartStride;
    const float we[3] = {s[0], s[1], s[2]};
    wave_sum_to_part<3>(we, dst, 64, 3, 1);          // dWe[c][a]
    const float c1[1] = {s[3]};
    wave_sum_to_part<1>(c1, dst + 3 * kHid, 64, 1, 0);   // dc[c]
}

// Encoder backward: partials of dW0 (64 x 7) and db0 (64).
__global__ void __launch_bounds__(kThreads) k_enc_bwd(int n, const double *w, const double *m, const double *mp,
                                                      const double *red, const float *wr, const float *gh,
                                                      float *part) {
    const double sm = dm_scale(red), ism = sm > 0.0 ? 1.0 / sm : 0.0;
    const int lane = threadIdx.x & 63;
    float w0[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) w0[k] = wr[kOffW0 + lane * kIn + k];
    const float b0 = wr[kOffB0 + lane];
    float s[kIn + 1] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = blockIdx.x * kWaves + (threadIdx.x >> 6); i < n; i += gridDim.x * kWaves) {
        float x[kIn];
        node_features(n, i, w, m, mp, ism, x);
        float pre = b0;
#pragma unroll
        for (int k = 0; k < kIn; ++k) pre += w0[k] * x[k];
        const float gp = gh[static_cast<size_t>(i) * kHid + lane] * dsilu(pre);
#pragma unroll
        for (int k = 0; k < kIn; ++k) s[k] += gp * x[k];
        s[kIn] += gp;
    }
    float *dst = part + static_cast<size_t>(blockIdx.x) * kPartStride;
    float wv[kIn];
#pragma unroll
    for (int k = 0; k < kIn; ++k) wv[k] = s[k];
    wave_sum_to_part<kIn>(wv, dst, 64, kIn, 1);          // dW0[c][k]
    const float bb[1] = {s[kIn]};
    wave_sum_to_part<1>(bb, dst + kHid * kIn, 64, 1, 0);  // db0[c]
}

// ------------------------------------------------------------ optimiser, weights

__global__ void __launch_bounds__(kThreads) k_adam(float *p, const float *g, float *m1, float *m2, float lr, float c1,
                                                   float c2) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int j = blockIdx.x * kThreads + threadIdx.x; j < kNParam; j += gridDim.x * kThreads) {
        const float gj = g[j];
        const float a = b1 * m1[j] + (1.0f - b1) * gj;
        const float b = b2 * m2[j] + (1.0f - b2) * gj * gj;
        m1[j] = a;
        m2[j] = b;
        p[j] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
    }
}

__global__ void __launch_bounds__(kThreads) k_prepare(const float *p, float *wr, uint16_t *mats) {
    for (int j = blockIdx.x * kThreads + threadIdx.x; j < kNParam; j += gridDim.x * kThreads) wr[j] = round_bf(p[j]);
    for (int j = blockIdx.x * kThreads + threadIdx.x; j < kLayers * kMat; j += gridDim.x * kThreads) {
        const int l = j / kMat, q = j % kMat;
        const float *L = p + kOffL0 + l * kLayerSize;
        uint16_t *M = mats + static_cast<size_t>(l) * 4 * kMat;
        const uint16_t ab = f2bf(L[kLWa + q]);   // [Wa;Wb] row-major 128 x 64: row q / 64, col q % 64
        const uint16_t wu = f2bf(L[kLWu + q]);   // Wu 64 x 128: row q / 128, col q % 128
        M[q] = ab;
        M[kMat + q] = wu;
        M[2 * kMat + (q % 128) * 64 + q / 128] = wu;        // Wu^T 128 x 64
        M[3 * kMat + (q % 64) * 128 + q / 64] = ab;         // [Wa;Wb]^T 64 x 128
    }
}

// Sums of the least-squares system of the start on span{d, e}: (Kd.Kd, Kd.Ke,
// Ke.Ke, Kd.r0, Ke.r0); a null direction contributes 0.
__global__ void __launch_bounds__(kThreads) k_minres_sums(int n3, const double *d, const double *kd, const double *e,
                                                            const double *ke, const double *r0, double *red) {
    double a[kMrSums] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n3; i += gridDim.x * kThreads) {
        const double r = r0[i];
        const double kdi = d ? kd[i] : 0.0, kei = e ? ke[i] : 0.0;
        a[G_DKD] += kdi * kdi;
        a[G_DKE] += kdi * kei;
        a[G_EKE] += kei * kei;
        a[G_DR] += kdi * r;
        a[G_ER] += kei * r;
    }
    block_atomic_add<kMrSums>(a, red, kShards);
}

__device__ __forceinline__ void minres_coef(const double (&t)[kMrSums], double &ca, double &cc) {
    const double dd = t[G_DKD], de = t[G_DKE], ee = t[G_EKE], dr = t[G_DR], er = t[G_ER];
    const double det = dd * ee - de * de;
    ca = cc = 0.0;
    if (dd > 0.0 && ee > 0.0 && det > 1e-10 * dd * ee) {
        ca = (dr * ee - er * de) / det;
        cc = (er * dd - dr * de) / det;
    } else {
        const double gd = dd > 0.0 ? dr * dr / dd : 0.0, ge = ee > 0.0 ? er * er / ee : 0.0;
        if (gd >= ge) ca = dd > 0.0 ? dr / dd : 0.0;
        else cc = er / ee;
    }
    if (!__builtin_isfinite(ca) || !__builtin_isfinite(cc)) ca = cc = 0.0;
}

__global__ void __launch_bounds__(kThreads) k_minres_apply(int n3, const double *d, const double *e, double *x,
                                                             const double *red, double *coef) {
    const double *const src[kMrSums] = {red, red + kShards, red + 2 * kShards, red + 3 * kShards,
                                         red + 4 * kShards};
    double t[kMrSums];
    shard_totals<kMrSums>(src, t);
    double ca, cc;
    minres_coef(t, ca, cc);
    if (blockIdx.x == 0 && threadIdx.x == 0 && coef) {
        coef[0] = ca;
        coef[1] = cc;
    }
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < n3; i += gridDim.x * kThreads)
        x[i] += (d ? ca * d[i] : 0.0) + (e ? cc * e[i] : 0.0);
}

__global__ void __launch_bounds__(kThreads) k_sub(int64_t n3, const double *a, const double *b, double *out) {
    for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n3;
         i += static_cast<int64_t>(gridDim.x) * kThreads)
        out[i] = a[i] - b[i];
}

}  // namespace

// ------------------------------------------------------------ launchers

static void layer_gemm_ab(int n, const uint16_t *H, const uint16_t *wab, uint16_t *AB, hipStream_t s) {
    GemmArgs ga{};
    ga.out = AB;
    ga.ldo = 128;
    rowgemm<128, 64, uint16_t, EPI_BF16>(n, H, kHid, nullptr, 0, wab, ga, s);
}

void launch_forward(const Graph &g, const MeshView &mv, const Net &net, const double *m, const double *mprev,
                    double *red, const Acts &a, double lambda100, double *dvec, hipStream_t s) {
    const int n = g.n;
    launch_fill(red, R_COUNT * kShards, 0.0, s);
    hipLaunchKernelGGL(k_dm_sums, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, s, n, mv.w, m, mprev, red);
    hipLaunchKernelGGL(k_encode, dim3(grid_for(n, kWaves)), dim3(kThreads), 0, s, n, mv.w, m, mprev, red, net.wr,
                       a.H[0]);
    for (int l = 0; l < kLayers; ++l) {
        const uint16_t *mats = net.mats + static_cast<size_t>(l) * 4 * kMat;
        const float *wl = net.wr + kOffL0 + l * kLayerSize;
        layer_gemm_ab(n, a.H[l], mats, a.AB[l], s);
        hipLaunchKernelGGL(k_edge_fwd, dim3(grid_for(n, kWaves)), dim3(kThreads), 0, s, g, mv, wl, a.AB[l], a.AGG[l]);
        GemmArgs ga{};
        ga.out = a.H[l + 1];
        ga.ldo = kHid;
        ga.res = a.H[l];
        ga.ldr = kHid;
        ga.bias = wl + kLBu;
        rowgemm<64, 128, uint16_t, EPI_RESID_BF16>(n, a.H[l], kHid, a.AGG[l], kHid, mats + kMat, ga, s);
    }
    const double hbar = 1.0 / g.ihbar;
    hipLaunchKernelGGL(k_decode, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, s, n, mv.p0, a.H[kLayers], net.wr,
                       red, lambda100, hbar, a.y, dvec);
}

void launch_loss_backward(const Graph &g, const MeshView &mv, const Net &net, const double *m, const double *mprev,
                          const double *du, double lambda100, double *red, const Acts &a, const Grads &gr,
                          float *grad, hipStream_t s) {
    const int n = g.n;
    const double hbar = 1.0 / g.ihbar;
    hipLaunchKernelGGL(k_loss_sums, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, s, n, a.y, du, lambda100, hbar,
                       red);
    hipLaunchKernelGGL(k_loss_grad, dim3(grid_for(n, kThreads)), dim3(kThreads), 0, s, n, a.y, du, lambda100, hbar,
                       red, gr.gy);
    const int nwg = gr.part_wgs;
    hipLaunchKernelGGL(k_dec_bwd, dim3(nwg), dim3(kThreads), 0, s, n, a.H[kLayers], gr.gy, net.wr, gr.gh, gr.part);
    reduce_part(gr.part, nwg, kOut * kHid + kOut, grad + kOffWd, s);       // Wd then bd: contiguous
    const int rows_per_wg = ((n + nwg - 1) / nwg + 31) / 32 * 32;
    for (int l = kLayers - 1; l >= 0; --l) {
        const uint16_t *mats = net.mats + static_cast<size_t>(l) * 4 * kMat;
        const float *wl = net.wr + kOffL0 + l * kLayerSize;
        float *gl = grad + kOffL0 + l * kLayerSize;
        // d[h ; a] = gh Wu  (n x 128)
        GemmArgs g1{};
        g1.out = gr.gha;
        g1.ldo = 128;
        rowgemm<128, 64, float, EPI_F32>(n, gr.gh, kHid, nullptr, 0, mats + 2 * kMat, g1, s);
        // dWu = gh^T [H | AGG], dbu = sum gh
        hipLaunchKernelGGL((k_wgrad<64, 128>), dim3(nwg), dim3(kThreads), 0, s, n, rows_per_wg, gr.gh, kHid, a.H[l],
                           kHid, a.AGG[l], kHid, gr.part);
        reduce_part(gr.part, nwg, 64 * 128, gl + kLWu, s);
        hipLaunchKernelGGL(k_colsum, dim3(nwg), dim3(kThreads), 0, s, n, gr.gh, gr.part);
        reduce_part(gr.part, nwg, kHid, gl + kLBu, s);
        // edge pass
        hipLaunchKernelGGL(k_edge_bwd, dim3(nwg), dim3(kThreads), 0, s, g, mv, wl, a.AB[l], gr.gha, gr.gab, gr.part);
        reduce_part(gr.part, nwg, 192 + 64, gl + kLWe, s);   // We (64 x 3) then c (64): contiguous in the layout
        // dWab = gab^T H
        hipLaunchKernelGGL((k_wgrad<128, 64>), dim3(nwg), dim3(kThreads), 0, s, n, rows_per_wg, gr.gab, 128, a.H[l],
                           kHid, nullptr, 0, gr.part);
        reduce_part(gr.part, nwg, 128 * 64, gl + kLWa, s);
        // gh <- gh + d[h](from gha) + gab [Wa;Wb]
        GemmArgs g2{};
        g2.out = gr.gh;
        g2.ldo = kHid;
        g2.add0 = gr.gh;
        g2.lda0 = kHid;
        g2.add1 = gr.gha;
        g2.lda1 = 128;
        rowgemm<64, 128, float, EPI_ADD2_F32>(n, gr.gab, 128, gr.gab + 64, 128, mats + 3 * kMat, g2, s);
    }
    hipLaunchKernelGGL(k_enc_bwd, dim3(nwg), dim3(kThreads), 0, s, n, mv.w, m, mprev, red, net.wr, gr.gh, gr.part);
    reduce_part(gr.part, nwg, kHid * kIn + kHid, grad + kOffW0, s);
}

void launch_adam(float *master, const float *grad, float *m1, float *m2, float lr, int64_t t, hipStream_t s) {
    const float c1 = static_cast<float>(1.0 - std::pow(0.9, static_cast<double>(t)));
    const float c2 = static_cast<float>(1.0 - std::pow(0.999, static_cast<double>(t)));
    hipLaunchKernelGGL(k_adam, dim3(grid_for(kNParam, kThreads)), dim3(kThreads), 0, s, master, grad, m1, m2, lr, c1,
                       c2);
}

void launch_prepare_weights(const float *master, float *wr, uint16_t *mats, hipStream_t s) {
    hipLaunchKernelGGL(k_prepare, dim3(grid_for(kNParam, kThreads)), dim3(kThreads), 0, s, master, wr, mats);
}

void launch_minres(int n, const double *d, const double *kd, const double *e, const double *ke, const double *r0,
                     double *x, double *red, double *coef, hipStream_t s) {
    const int n3 = 3 * n;
    launch_fill(red, kMrSums * kShards, 0.0, s);
    hipLaunchKernelGGL(k_minres_sums, dim3(grid_for(n3, kThreads)), dim3(kThreads), 0, s, n3, d, kd, e, ke, r0, red);
    hipLaunchKernelGGL(k_minres_apply, dim3(grid_for(n3, kThreads)), dim3(kThreads), 0, s, n3, d, e, x, red, coef);
}

void launch_sub(int64_t n3, const double *a, const double *b, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_sub, dim3(grid_for(n3, kThreads)), dim3(kThreads), 0, s, n3, a, b, out);
}

}  // namespace mpnn
}  // namespace gspm
