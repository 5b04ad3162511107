// Internal declarations of the GSPM library (device data views, launchers).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "gspm.h"

namespace gspm {

#ifndef GSPM_THREADS
#define GSPM_THREADS 256
#endif
constexpr int kThreads = GSPM_THREADS;   // threads per workgroup of every kernel
constexpr int kMaxComp = 3;

// ---------------------------------------------------------------- host mesh

// Result of the one-time host preprocessing of an uploaded mesh.
struct HostMesh {
    int64_t n0 = 0;               // caller's nodes
    int32_t n = 0;                // unique nodes after periodic identification
    int64_t ne = 0;               // tetrahedra
    int32_t nb = 0;               // owned nodes per block
    int32_t nblk = 0;             // blocks
    int32_t p0 = -1;              // internal id of the pinned node (caller's node 0)
    int64_t ncopies = 0;          // element copies over all block lists
    int32_t nloc_max = 0;         // largest owned + halo node count of a block
    int64_t nhalo = 0;            // halo entries over all blocks
    double lo[3] = {0, 0, 0}, L[3] = {0, 0, 0};
    double vc = 0.0;              // cell volume
    std::vector<int32_t> user2int;        // n0
    std::vector<double> xs;               // 3 x n coordinates, component-major
    std::vector<uint16_t> lconn;          // 4 x ncopies local vertex indices (owned: id - n0; halo: nb + slot)
    std::vector<int32_t> blk_ptr;         // nblk + 1 element-copy ranges
    std::vector<int32_t> blk_nmag;        // nblk: magnetic copies come first in each list
    std::vector<int32_t> halo_ptr;        // nblk + 1
    std::vector<int32_t> halo_ids;        // halo node ids, sorted within a block
    std::vector<int32_t> halo_lo;         // nblk: halo ids below the block's range
    std::vector<uint8_t> img;             // nblk: edges need the nearest periodic image
    std::vector<double> w;                // n: lumped magnetic weights sum_e chi_e V_e / 4
    // Tet strips of the matrix-free operators (see pack_strips): per block at
    // most kThreads segments of about equal length, magnetic segments first.
    std::vector<uint16_t> seg_ent;        // window updates; each segment padded to a multiple of 8, 16 zeros at the end
    std::vector<uint32_t> seg_off;        // per segment: first entry / 8
    std::vector<uint16_t> seg_nel;        // per segment: window updates (entries)
    std::vector<int32_t> seg_ptr;         // nblk + 1
    std::vector<int32_t> seg_nmag;        // nblk
};

// A strip segment is a sequence of window updates.  Entry = local vertex id
// (13 bits) | element-complete flag (bit 13) | slot (2 bits) << 14.  The
// first four entries of a segment fill slots 0..3 in order; every later one
// makes the vertex in the named slot leave, moves the vertex of slot 3 into
// that slot and puts the new vertex in slot 3.  When the flag is set, the
// window holds exactly the four vertices of the segment's next element.
constexpr uint32_t kEntIdMask = 0x1FFFu;
constexpr uint32_t kEntElem = 1u << 13;
constexpr int kMaxLocal = 8191;           // staged nodes per block the entries can address

int prepare_mesh(int64_t n0, const double *xyz, int64_t ne, const int32_t *tets, const uint8_t *tags,
                 const double lo[3], const double hi[3], int32_t nb, HostMesh &out, std::string &err,
                 int reorder = GSPM_REORDER_MORTON);

// Rows of the GS operator's two parts over magnetic elements, K (Laplacian)
// and M (consistent mass), assembled on the host at upload (gs_rows.cpp).
// Rows are in internal node order, in slices of 64 (one per wavefront);
// slice s holds its rows' off-diagonal entries entry-major, entry k of lane l
// at off[s] + 64 k + l, padded to the slice's longest row with zero
// coefficients whose column is the row itself.  Columns index the row's
// owner-block staging: owned node j -> j - n0, halo node -> nb + its position
// in the block's halo list.
struct GsRowsHost {
    std::vector<int32_t> off;     // slices + 1
    std::vector<uint16_t> col;    // entries
    std::vector<double> kv, mv;   // entries: K_ij, M_ij (i != j)
    std::vector<double> kd, md;   // n: K_ii, M_ii
    // row blocks (ranges of nb rows in the node order; independent of the element blocks): the staged
    // nodes of block b are its owned range, then halo_ids[halo_ptr[b] .. halo_ptr[b + 1]), the sorted
    // columns of its rows outside that range
    int32_t nb = 0, nblk = 0, nloc_max = 0;
    std::vector<int32_t> halo_ptr, halo_ids;
};

// nb_rows: nodes per row block, a multiple of 64 (0: the element blocks' size)
int assemble_gs_rows(const HostMesh &hm, int64_t ne, const int32_t *tets, const uint8_t *tags, int32_t nb_rows,
                     GsRowsHost &out, std::string &err);

// ------------------------------------------------------------- device views

// Fixed-order sums of the deterministic mode.  A producer launch stores the
// workgroup totals of its sums in slots (sum, workgroup) and workgroup 0
// records each sum's destination; the finishing launch that follows
// (launch_det_finish) adds every recorded sum's slots in a fixed order to
// shard 0 of its destination and clears them.  part == nullptr: atomic adds.
constexpr int kDetSlots = 16;
struct DetSums {
    double *part = nullptr;       // [kDetSlots][max_blocks]
    double **dst = nullptr;       // [kDetSlots]: destination of each recorded sum (null: skipped)
    int32_t *count = nullptr;     // sums recorded by the last producer launch
    int32_t max_blocks = 0;       // workgroups a producer launch may have
};

// Mesh as the element kernels see it: node coordinates (FP64), and per owner
// block its element copies as local vertex indices into the block's staged
// node set [owned range | halo list].
struct MeshView {
    const double *x, *y, *z;      // n each
    const ushort4 *lconn;         // element copies, local indices
    const int32_t *blk_ptr, *blk_nmag, *halo_ptr, *halo_ids, *halo_lo;
    const uint8_t *img;
    const double *w;              // n
    const double *stc64;          // staged coordinates per block, FP64: [3][sum of n_staged] (see stage_coords)
    const float *stc32;           // the same scaled by 1 / len_scale, FP32
    int64_t nstc;                 // sum over blocks of staged nodes (nb + halo count)
    const uint4 *seg_ent;         // strip entries, 8 per uint4
    const uint32_t *seg_off;      // per segment: first uint4 of its entries
    const uint16_t *seg_nel;      // per segment: entries
    const int32_t *seg_ptr, *seg_nmag;
    int32_t n, nb, nblk, p0, nloc_max;
    double Lx, Ly, Lz, iLx, iLy, iLz;   // box edges and their inverses (nearest periodic image)
    double len_scale;                   // cube root of the mean element volume (FP32 non-dimensionalisation)
    // deterministic mode: fixed-order sums, and per owned node (block-major, nb per block) its element
    // copies as (copy index within the block's list) << 2 | vertex slot, in copy order
    DetSums det;
    const int32_t *inc_ptr;
    const uint16_t *inc_ent;
};

// Material constants in the form the kernels use.
struct Material {
    double c11, c12, c44;         // cubic stiffness
    double l100, l111;            // magnetostriction
    double kan;                   // 2 K1 / (mu0 Ms^2)
    double kme;                   // 1 / (mu0 Ms^2)
    double A;                     // exchange coefficient (energies)
    double K1;                    // anisotropy (energies)
    double mu0Ms;                 // mu0 Ms (energies)
    // crystal orientation (App. D): v_sample = R v_crystal, row-major; rot = 0
    // when the crystal axes are the sample axes.  C6 is the stiffness in the
    // sample frame as a Voigt matrix (xx yy zz yz xz xy, engineering shear).
    int32_t rot;
    double R[9];
    double C6[36];
};

// Per-stage quantities derived from the volume averages (device resident).
struct Derived {
    double mbar[3];
    double ebar[6];               // homogeneous strain, xx yy zz yz xz xy
    double hc[3];                 // h_zeeman + h_demag_far (uniform part of h)
};

// Reduction scalars are sharded: each is kShards doubles that producer
// workgroups add into (workgroup w into shard w % kShards) and consumers sum.
constexpr int kShards = 32;

// Scalars of up to kMaxComp simultaneous CG solves (device resident).  The
// per-iteration dot products live in a ring of `ring` slots: slot k % ring.
struct CGScalars {
    double *rr;                   // [comp][ring][kShards]: r_k . r_k
    double *pq;                   // [comp][ring][kShards]: p_k . A p_k
    double *bb;                   // [comp][kShards]: b . b
    double *rq, *qq;              // [ring][kShards]: r_k . A p_k, |A p_k|^2 (single-reduction CG, one scalar set)
    double *rz;                   // [comp][ring][kShards]: r_k . D^-1 r_k (Jacobi-preconditioned GS solves)
    double *rzq, *qzq;            // [comp][ring][kShards]: r_k . D^-1 q_k, q_k . D^-1 q_k (single-reduction GS solves)
    int32_t *done;                // [comp]: 0 running, 1 converged, 2 broke down (non-finite)
    int32_t *iters;               // [comp]: iterations at convergence
    int32_t ring;
    DetSums det;                  // deterministic mode: the fixed-order sums (part == nullptr: atomic adds)

    __host__ __device__ double *rr_at(int c, int k) const {
        return rr + (static_cast<size_t>(c) * ring + static_cast<size_t>(k % ring)) * kShards;
    }
    __host__ __device__ double *rz_at(int c, int k) const {
        return rz + (static_cast<size_t>(c) * ring + static_cast<size_t>(k % ring)) * kShards;
    }
    __host__ __device__ double *rzq_at(int c, int k) const {
        return rzq + (static_cast<size_t>(c) * ring + static_cast<size_t>(k % ring)) * kShards;
    }
    __host__ __device__ double *qzq_at(int c, int k) const {
        return qzq + (static_cast<size_t>(c) * ring + static_cast<size_t>(k % ring)) * kShards;
    }
    __host__ __device__ double *pq_at(int c, int k) const {
        return pq + (static_cast<size_t>(c) * ring + static_cast<size_t>(k % ring)) * kShards;
    }
    __host__ __device__ double *bb_at(int c) const { return bb + static_cast<size_t>(c) * kShards; }
    __host__ __device__ double *rq_at(int k) const { return rq + static_cast<size_t>(k % ring) * kShards; }
    __host__ __device__ double *qq_at(int k) const { return qq + static_cast<size_t>(k % ring) * kShards; }
    __host__ __device__ int comp_stride() const { return ring * kShards; }
};

enum MatvecMode { MV_APPLY = 0, MV_ITER = 1, MV_RESID = 2 };

// The GS operator A = eps K + mass M in row form (see GsRowsHost), with the
// coefficients of one (eps, mass) pair in the working precision T (FP32: A
// divided by len_scale^3, the scaling of the FP32 operators).
struct GsRowsView {
    const int32_t *off;           // per 64-row slice: first entry; width = (off[s + 1] - off[s]) / 64
    const uint16_t *col;          // entries: staged local column index
    const void *a;                // entries: off-diagonal coefficients (T)
    const void *d;                // n: diagonal (T); also the Jacobi preconditioner's D
};

// The GS operator in row form on nc components: APPLY out = A in; RESID
// r = b - A in on the components not converged, with r.r into rr[0].
template <class T>
void launch_gs_rows(const MeshView &mv, const GsRowsView &rv, int nc, MatvecMode mode, const T *in, T *out,
                    const T *b, T *r, const CGScalars &cg, hipStream_t s);
// Single-reduction CG iteration k on the GS operator in row form (nc
// components, one launch per iteration; Jacobi-preconditioned when jacobi):
// completes iteration k-1 (x, r) from the sums p.q, r.r, r.D^-1 r, r.D^-1 q
// and q.D^-1 q of launch k-1, forms p_k, and writes q_k = A p_k with the sums
// of iteration k.  Buffers and the last launch as for launch_elastic_cg; the
// start residual's |r_0|^2 must be in slot 0.
template <class T>
void launch_gs_rows_cg(const MeshView &mv, const GsRowsView &rv, int nc, int k, bool last, const T *rin, const T *pin,
                       const T *qin, T *rout, T *pout, T *qout, T *x, const CGScalars &cg, double tol, bool jacobi,
                       hipStream_t s, const hipEvent_t *ev = nullptr);
// out[i] = (T) (scale (eps kv[i] + mass mv[i])) for i < count.
template <class T>
void launch_gs_combine(int64_t count, const double *kv, const double *mv, double eps, double mass, double scale,
                       T *out, hipStream_t s);

// Preconditioned CG on the elastic system keeps r_k . z_k of iteration k in
// the single-reduction slots of its scalar set: k = 0 in rq[0], k > 0 in
// qq[k - 1] (the slots the ring zeroing clears before iteration k - 1 runs).
__host__ __device__ inline double *pcg_rz_at(const CGScalars &cg, int k) {
    return k == 0 ? cg.rq_at(0) : cg.qq_at(k - 1);
}

// ------------------------------------------- Green's-operator preconditioner

// Device data of B = Q A_g^+ Q^T + omega D^-1 (elastic_precond), in the
// working precision of the context's elastic iterations (T = double for FP64
// contexts, float for the inner solves of the mixed form, where every factor
// carries 1 / scale with scale the FP32 operator's non-dimensionalisation).
struct GreenView {
    int32_t gx, gy, gz, gxh;      // grid points per axis; gxh = gx / 2 + 1 (half spectrum along x)
    int64_t G, Gh;                // grid points, half-spectrum modes (gz x gy x gxh)
    double lo[3], h[3];           // grid origin and spacing
    const int32_t *rptr, *rnode;  // restriction lists: row t gathers (rnode, rw)[rptr[t] .. rptr[t + 1])
    const int32_t *rgrid;         // the grid point of row t (rows run in Morton order of the grid points)
    const void *rw;               // their weights (T)
    const void *dinv;             // [3][n] omega / diag(K^mech) (T)
    const void *ainv;             // [Gh][9] A(k)^-1 / G, Hermitian: re a00 a11 a22, then a01 a02 a12 (re, im) (T)
    void *grid;                   // [2][G] complex (T): x0 + i x1, x2 on the grid (restriction in, prolongation out)
    void *spec;                   // [2][G] complex (T): their spectra (forward FFT out, inverse FFT in)
};

// The preconditioner's node and grid passes (green_kernels.hip).  Every
// launch returns at once when the scalar set has converged.
template <class T>
void launch_pc_restrict(const GreenView &gv, int n, const T *r, const CGScalars &cg, int test_k, double tol,
                        hipStream_t s);
template <class T>
void launch_pc_modes(const GreenView &gv, const CGScalars &cg, hipStream_t s);
template <class T>
void launch_pc_prolong(const GreenView &gv, const MeshView &mv, const T *r, T *z, double *rz, const CGScalars &cg,
                       hipStream_t s);
// x += alpha p, r -= alpha q with alpha = rz[k] / pq[k]; rr[k + 1] += r.r.
template <class T>
void launch_pcg_update(int n, T *x, T *r, const T *p, const T *q, const CGScalars &cg, int k, hipStream_t s);
// b -= mean(b) per component; bb (zeroed here) += b.b.  aux: 3 x kShards doubles.
void launch_remove_mean3(int n, double *b, double *aux, double *bb, hipStream_t s, const DetSums &det = DetSums{});
// x -= x(p0) on every node.  aux: 3 doubles.
void launch_pin_shift(int n, double *x, int p0, double *aux, hipStream_t s);
// The symbol inverse of the grid operator for the half spectrum: stencil27 is
// the 27 3x3 blocks S(o) (o = (ox, oy, oz) in {-1,0,1}^3, index (oz+1)*9 + (oy+1)*3 + (ox+1)),
// A(k) = sum_o S(o) exp(2 pi i k.o / g), stored as A(k)^-1 * factor (zero at k = 0).
template <class T>
void launch_pc_symbol(const GreenView &gv, const double *stencil27, double factor, hipStream_t s);
// Preconditioned CG iteration k on the elastic system: p_k = z_k + beta p_{k-1}
// (beta = rz[k] / rz[k-1], p_0 = z_0) in the staging, q = A p_k (no pinned
// node), pq[k] += p_k . q.  pin = p_{k-1}, pout = p_k (alternating buffers).
template <class T>
void launch_elastic_pcg(const MeshView &mv, const Material &mat, int k, const T *z, const T *pin, T *pout, T *q,
                        const CGScalars &cg, hipStream_t s, const hipEvent_t *ev = nullptr);

// ---------------------------------------------------------------- launchers

void launch_fill(double *p, int64_t n, double v, hipStream_t s);
void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);

// The corrected start of a GS solve: x0 += corr (when use) and start = x0;
// after the solve corr = (use ? corr : 0) + x - start, the solution minus the
// lumped start, for the next step's solve of the same stage.
void launch_gs_start(int64_t n, double *x, const double *corr, double *start, bool use, hipStream_t s);
void launch_gs_correction(int64_t n, const double *x, const double *start, double *corr, bool use, hipStream_t s);

// Volume-average sums (sharded, 9 x kShards): sum w m (3), sum w E0(m) (6).
// <E0> is summed in the crystal frame when mat.rot (k_derive rotates it).
void launch_avg_sums(int n, const double *w, const double *m, const Material &mat, double *sums, hipStream_t s,
                     const DetSums &det = DetSums{});
struct DeriveArgs {
    double vc;
    double Nd[9];
    double hz[3];                 // H_ext / Ms
    double csig[6];               // C^-1 sigma_ext (sample frame)
    int32_t rot;                  // the averaged E0 sums are crystal-frame: rotate them by R
    double R[9];
};
void launch_derive(const double *sums, const DeriveArgs &a, Derived *out, hipStream_t s);

// Allocation-free volume averages (gspm_averages_noalloc).  The scratch is a
// file-scope device array of node_kernels.hip, one per GPU: partial sums of at
// most kNaMaxGroups workgroups of kNaNodesPerGroup unique nodes each.
constexpr int kNaNodesPerGroup = 4 * kThreads;
constexpr int kNaMaxGroups = 4096;
constexpr int64_t kNaMaxNodes = static_cast<int64_t>(kNaMaxGroups) * kNaNodesPerGroup;
constexpr int kNaMaxDevices = 64;
// Device address of the scratch on `device` (which must be current), looked
// up once per device with hipGetSymbolAddress.  Returns a hipError_t value.
int noalloc_scratch_address(int device, double **out);
// mbar and ebar of m_user (caller node order, device) into out[9] (device), on
// stream s, through the scratch at scr.  Returns a hipError_t value.
int launch_averages_noalloc(double *scr, int n, const double *w, const int32_t *rep, const double *m_user,
                            const Material &mat, const DeriveArgs &da, double *out, hipStream_t s);

// Element passes (one workgroup per owner block).
void launch_elastic_rhs(const MeshView &mv, const Material &mat, const double *m, double *b, double *x,
                        double *bb, hipStream_t s);
// ud (nullable): the local magnetostatic potential; its element field
// -grad ud * inv_ms joins h on every vertex of a magnetic element.
void launch_field_rhs(const MeshView &mv, const Material &mat, const double *m, const double *u,
                      const Derived *d, double c, double *b, double *x0, double *ch2, double *bb, int bbstride,
                      const double *ud, double inv_ms, hipStream_t s);
// Right-hand side of Eq. (weak_demag): b_i = Ms sum_e V_e grad(lambda_i) . <m>_e
// over all elements (zero at the pinned node, whose potential x is zeroed);
// bb[0] += b.b.
void launch_ms_rhs(const MeshView &mv, double Ms, const double *m, double *b, double *x, double *bb,
                   hipStream_t s);
void launch_mass_rhs(const MeshView &mv, const double *y, const double *ch2, double *b, double *x0,
                     double *bb, int bbstride, hipStream_t s);
// Matrix-free operators.  APPLY: out = A in.  RESID: r = b - A x (x = in),
// rr[0] += r.r.  ITER (CG iteration k): p_new = r + beta_k p_old (p_new = r at
// k = 0, with beta_k = rr[k] / rr[k-1] and the convergence test of rr[k] done
// first), q = A p_new, pq[k] += p_new.q; p_old = in, p_new = pout.
// ev (nullable): two events the runtime records at the kernel's own start and
// end (profiling: the pair times the kernel alone, without launch gaps).
template <class T>
void launch_elastic_matvec(const MeshView &mv, const Material &mat, MatvecMode mode, const T *in, T *out, const T *b,
                           const T *r, T *pout, const CGScalars &cg, int k, double tol, hipStream_t s,
                           const hipEvent_t *ev = nullptr);
// Single-reduction CG iteration k on the elastic system (one launch per
// iteration): tests |r_{k-1}|, completes iteration k-1 (x, r) and computes
// q_k = A p_k with the sums p.q, r.q, q.q, r.r of iteration k.  Buffers
// alternate by the parity of k: (rin, pin, qin) hold iteration k-1, (rout,
// pout, qout) receive iteration k; at k = 0, rin holds r_0 and rout is unused.
// A solve that converges at iteration j is recorded (iters = j) by launch
// j + 1.  last: the launch after the last permitted iteration (the test of
// |r_{k-1}|, and the x update when it fails).  ev as for launch_elastic_matvec.
template <class T>
void launch_elastic_cg(const MeshView &mv, const Material &mat, int k, bool last, const T *rin, const T *pin,
                       const T *qin, T *rout, T *pout, T *qout, T *x, const CGScalars &cg, double tol, hipStream_t s,
                       const hipEvent_t *ev = nullptr);
// K^ms (Laplacian over all elements) on nc = 1 or 3 components, rows of the
// pinned node zero; modes as above.  FP32: A' = K^ms / len_scale^3.
// One launch of single-reduction CG on K^ms (one component), with the
// buffer and scalar conventions of launch_elastic_cg.
template <class T>
void launch_ms_cg(const MeshView &mv, int k, bool last, const T *rin, const T *pin, const T *qin, T *rout, T *pout,
                  T *qout, T *x, const CGScalars &cg, double tol, hipStream_t s);
template <class T>
void launch_ms_matvec(const MeshView &mv, int nc, MatvecMode mode, const T *in, T *out, const T *b, const T *r,
                      T *pout, const CGScalars &cg, int k, double tol, hipStream_t s);
// out2[0 .. kShards), out2[kShards .. 2 kShards): exchange and magnetoelastic
// sums; with ud, out2[4 kShards .. 5 kShards): sum_e V_e |grad ud|^2.
void launch_energy_elem(const MeshView &mv, const Material &mat, const double *m, const double *u,
                        const double *ud, const Derived *d, double *out2, hipStream_t s);
void launch_energy_nodes(int n, const double *w, const double *m, const Material &mat, const double hext[3],
                         double *out2, hipStream_t s, const DetSums &det = DetSums{});

// CG vector kernels on [nc][n] component-major vectors; joint: one set of
// scalars for all components (the elastic solve), else one per component.
template <class T>
void launch_cg_start(int n, int nc, bool joint, T *x, const CGScalars &cg, double tol, hipStream_t s);
template <class T>
void launch_cg_update(int n, int nc, bool joint, T *x, T *r, const T *p, const T *q, const CGScalars &cg, int k,
                      hipStream_t s);
void launch_cg_check(int nc, bool joint, const CGScalars &cg, int k, double tol, hipStream_t s);
// Small values for the host: count (<= 64) int32 copied into pinned host
// memory; the totals of up to six sharded sums into pinned host memory.
struct ShardSources {
    static constexpr int kMax = 6;
    const double *p[kMax];
};
void launch_i32_to_host(const int32_t *src, int count, int32_t *host_dst, hipStream_t s);
void launch_totals_to_host(const ShardSources &src, int count, double *host_dst, hipStream_t s);
// The start of an inner FP32 solve of the mixed form, in one launch: the
// inner threshold bb[q] (shard 0; the other shards zero) and done[q] per
// component with iters zero; r32 = (float) (scale * r64) on nc components
// with ||r32||^2 per scalar set into slot 0 of the ring (zeroed by an
// earlier launch); x32 = 0 on nx values.
struct InnerStart {
    double bb[kMaxComp];
    int32_t done[kMaxComp];
};
void launch_inner_start(int n, int nc, bool joint, const double *src, double scale, float *dst, float *x32,
                        int64_t nx, const CGScalars &cg, const InnerStart &st, hipStream_t s);

// Precision conversions of the mixed form: dst = (float) src; x += (double) d.
void launch_to_f32(int64_t n, const double *src, float *dst, hipStream_t s);
void launch_add_f32(int64_t n, double *x, const float *d, hipStream_t s);
void launch_fill_f32(float *p, int64_t n, hipStream_t s);

// GSPM node updates (Algorithm B.1, Step 2 and Step 4).
void launch_update_m12(int n, const double *m, const double *g, double *ms, hipStream_t s);
void launch_update_m3(int n, const double *m, const double *gs, double *ms, hipStream_t s);
void launch_normalize(int n, const double *w, const double *mss, const double *mold, double *mnew, double *dm_sum,
                      int32_t *bad, hipStream_t s, const DetSums &det = DetSums{});
// Deterministic mode: adds the sums the last producer launch recorded (no-op when det.part is null).
void launch_det_finish(const DetSums &det, hipStream_t s);
void launch_zero_ring(const CGScalars &cg, int ns, int rr_from, int rr_to, int pq_from, int pq_to, hipStream_t s);
// A new solve on `cg`: slot 0 of the r.r ring of ns components, the b.b
// shards and the done and iteration flags of every component cleared in one
// launch.
void launch_cg_reset(const CGScalars &cg, int ns, hipStream_t s);

// --------------------------------------------------------------- utilities

int nodes_per_block(int32_t requested, int64_t n);
// Staged coordinates of every block, in block order: slot l of block b is at
// b nb + halo_ptr[b] + l; coordinates relative to the block's first node
// (nearest image), FP64 as is and FP32 scaled by 1 / len_scale.
void launch_stage_coords(const MeshView &mv, double *stc64, float *stc32, hipStream_t s);
// Largest dynamic LDS request of the element kernels for blocks of nb owned
// nodes and at most nloc_max staged nodes (elem_kernels.hip).
size_t elem_lds_bytes(int32_t nb, int32_t nloc_max);
// Largest LDS request of the GS row kernels for row blocks of nb nodes and
// at most nloc_max staged nodes (row_kernels.hip); fp64_cg: FP64 CG
// iterations run too (FP64 contexts).
size_t rows_lds_bytes(int32_t nb, int32_t nloc_max, bool fp64_cg);
double carlson_rd(double x, double y, double z);
void demag_factors(double a, double b, double c, double N[3]);

}  // namespace gspm
