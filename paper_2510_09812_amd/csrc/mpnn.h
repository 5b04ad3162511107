// Learned elastic warm start: the message-passing network's layout and the
// launchers of its kernels (mpnn.hip).
//
// Network (per node i of the periodic mesh graph, hidden width 64):
//   x_i  = tag_i [dm_i / s_m, m_i, 1]               dm = m^n - m^{n-1}, tag = magnetic node
//   h_i  = SiLU(W0 x_i + b0)
//   3 x: z_ij = Wa h_i + Wb h_j + We e_ij + c,  a_i = mean_j SiLU(z_ij),
//        h_i <- h_i + Wu [h_i ; a_i] + bu
//   y_i  = Wd h_i + bd
// Weights and stored activations are BF16; all arithmetic and accumulation is
// FP32 (MFMA for the node GEMMs).  Gradients are FP32.
#pragma once

#include "common.h"

namespace gspm {
namespace mpnn {

constexpr int kHid = 64, kIn = 7, kLayers = 3, kOut = 3;
constexpr int kOffW0 = 0, kOffB0 = kHid * kIn, kOffL0 = kOffB0 + kHid;
constexpr int kLWa = 0, kLWb = kHid * kHid, kLWe = 2 * kHid * kHid, kLC = kLWe + 3 * kHid, kLWu = kLC + kHid,
              kLBu = kLWu + 2 * kHid * kHid, kLayerSize = kLBu + kHid;
constexpr int kOffWd = kOffL0 + kLayers * kLayerSize, kOffBd = kOffWd + kOut * kHid, kNParam = kOffBd + kOut;
static_assert(kNParam == 50819, "parameter layout");
constexpr int kMat = 128 * 64;              // elements of each BF16 weight-matrix form
constexpr int kPartStride = 8192;           // floats of one workgroup's gradient partial

// Reduction slots (each kShards doubles) of the network's scalar buffer.
enum RedSlot { R_DM2 = 0, R_W = 1, R_Y = 2, R_T = 5, R_LOSS = 8, R_COUNT = 9 };
// Sharded sums of the minimum-residual start (their own buffer of kMrSums x kShards).
enum MrSlot { G_DKD = 0, G_DKE = 1, G_EKE = 2, G_DR = 3, G_ER = 4, kMrSums = 5 };   // Kd.Kd, Kd.Ke, Ke.Ke, Kd.r0, Ke.r0

struct Graph {
    const int32_t *ptr, *nbr;                // CSR over unique nodes, neighbours sorted
    int32_t n;
    float ihbar;                             // 1 / mean spacing: edge vectors are (x_j - x_i) / hbar
};

// Weight forms derived from the FP32 master parameters.
struct Net {
    const float *wr;                         // all parameters rounded to BF16, held as FP32
    const uint16_t *mats;                    // per layer 4 x kMat BF16: [Wa;Wb] (128 x 64), Wu (64 x 128),
                                             // Wu^T (128 x 64), [Wa;Wb]^T (64 x 128)
};

struct Acts {
    uint16_t *H[kLayers + 1];                // n x 64 BF16
    uint16_t *AB[kLayers];                   // n x 128 BF16: [Wa h | Wb h]
    uint16_t *AGG[kLayers];                  // n x 64 BF16: mean edge messages
    float *y;                                // n x 3
};

struct Grads {
    float *gh;                               // n x 64
    float *gha;                              // n x 128: d[h ; a]
    float *gab;                              // n x 128: d[A | B]
    float *gy;                               // n x 3
    float *part;                             // per-workgroup partials, kPartStride each
    int part_wgs;                            // capacity in workgroups
};

// Forward pass: node features and increment scale, encoder, layers, decoder.
// With dvec != nullptr also writes the increment d = (lambda100 hbar s_m)(y - y_p0)
// as 3 x n FP64 (component-major).
void launch_forward(const Graph &g, const MeshView &mv, const Net &net, const double *m, const double *mprev,
                    double *red, const Acts &a, double lambda100, double *dvec, hipStream_t s);
// Loss (mean-removed MSE against du / (lambda100 hbar s_m)) and its gradient
// with respect to y; then the backward pass into grad (kNParam floats).
void launch_loss_backward(const Graph &g, const MeshView &mv, const Net &net, const double *m, const double *mprev,
                          const double *du, double lambda100, double *red, const Acts &a, const Grads &gr,
                          float *grad, hipStream_t s);
void launch_adam(float *master, const float *grad, float *m1, float *m2, float lr, int64_t t, hipStream_t s);
void launch_prepare_weights(const float *master, float *wr, uint16_t *mats, hipStream_t s);
// Start on span{d, e} (either may be null): x += a d + c e with (a, c)
// minimising |r0 - a K d - c K e|, i.e. solving
// [[Kd.Kd, Kd.Ke], [Ke.Kd, Ke.Ke]] (a, c) = (Kd.r0, Ke.r0); when K d and K e are
// nearly parallel (determinant below 1e-10 of the diagonal product) the better
// single-direction step; a non-finite or non-positive system gives 0.  red
// holds 5 sharded sums; coef (device, 2 doubles) receives (a, c).
void launch_minres(int n, const double *d, const double *kd, const double *e, const double *ke, const double *r0,
                     double *x, double *red, double *coef, hipStream_t s);
// out = a - b over n3 values.
void launch_sub(int64_t n3, const double *a, const double *b, double *out, hipStream_t s);

// Host: directed edge graph of the mesh on unique nodes (every pair of
// distinct nodes sharing a tetrahedron, both directions), CSR with sorted
// neighbour lists.
void build_edge_graph(int32_t n, const std::vector<int32_t> &tets, std::vector<int32_t> &ptr,
                      std::vector<int32_t> &nbr);

}  // namespace mpnn
}  // namespace gspm
